"""MI355X-native wildfire cellular automaton (Xia & Cheng, PyTorchFire, 2025).

The compute path is the HIP library ``libfiresim.so`` (C ABI in
``include/firesim.h``); this package only marshals arguments to it.  Importing
a submodule that needs the library raises ImportError when it is not built.
"""

from ._abi import (  # noqa: F401
    SIM_F_CALIB,
    SIM_F_STATS,
    SIM_LOSS_BCE,
    SIM_LOSS_BCE_MSE,
    SIM_LOSS_MSE,
    SimError,
    load,
)

__all__ = ["load", "Sim", "SimError", "FireCalib", "calibrate", "calibrate_sequence",
           "ensemble_arrival"]


def __getattr__(name):
    if name in ("Sim", "ensemble_arrival"):
        from . import sim
        return getattr(sim, name)
    if name in ("FireCalib", "calibrate", "calibrate_sequence"):
        from . import calib
        return getattr(calib, name)
    raise AttributeError(name)
