"""Seeded synthetic inputs for the wildfire cellular automaton.

This package only draws landscapes, wind fields, ignition patterns and
fire-state snapshots.  It holds none of the automaton's arithmetic: no
propagation probability, no sampling, no state transition.  Both the CPU
oracle's tests and the GPU path's tests and benchmark consume what it
produces, so that the two sides always see identical FP32 bytes.
"""

from .fields import (  # noqa: F401
    Scenario,
    PARAMS_TRUE,
    C_NORMALISER,
    make_plain,
    make_rough,
    make_lakes,
    config0,
    config1,
    config2,
    config3_scenario,
    config3_sizes,
    paper_plain,
    config4_scenario,
    synthetic_front_state,
    encode_planes,
    decode_planes,
)
