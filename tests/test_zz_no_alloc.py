"""sim_init_static, the entry point that allocates no device memory (its
workspace is the library's static scratch array), against sim_init with a
caller-allocated workspace on the same seeded inputs: states, the p_ignite
map, the accumulator, the Eq. 10 loss and the gradient must be identical
(both handles run the same kernels on the same inputs; integer and bit-plane
results are bit-exact, the FP32/FP64 values come from the same operations in
the same order).  Two inputs in a row, the second smaller, so the second
handle reuses an array that still holds the first handle's data."""

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def _pair(Sim, s, **kw):
    ref = Sim([s], **kw)
    st = Sim([s], static_scratch=True, **kw)
    assert st.workspace is None
    return ref, st


def _same(a, b, what):
    a, b = a.cpu().numpy(), b.cpu().numpy()
    assert a.shape == b.shape, what
    assert np.array_equal(a, b), f"{what}: {int((a != b).sum())} entries differ"


@pytest.fixture(scope="module")
def Sim():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2502_18738_amd.sim import Sim
    return Sim


CASES = [("300x260", lambda: synth.make_lakes(300, 260, 11, T=60, n_ignitions=3)),
         ("97x130", lambda: synth.make_lakes(97, 130, 12, T=60, n_ignitions=2))]


def test_static_scratch_forward_and_calibration_match(Sim):
    import torch
    for name, make in CASES:      # the second call has the smaller input
        s = make()
        T = 60
        say("static scratch, forward", name)
        ref, st = _pair(Sim, s)
        try:
            ref.run(T)
            st.run(T)
            torch.cuda.synchronize()
            _same(ref.get_state(0), st.get_state(0), f"{name}: state")
            _same(ref.pignite(0), st.pignite(0), f"{name}: p_ignite")
        finally:
            st.close()
            del ref
        say("static scratch, calibration", name)
        tgt = np.zeros(s.H * s.W, np.uint8)
        tgt[: s.H * s.W // 3] = 1
        ref, st = _pair(Sim, s, calib=True, T_max=T, ckpt_every=20)
        try:
            ref.run(T)
            st.run(T)
            l1, g1 = ref.loss_grad(tgt, 0)
            l2, g2 = st.loss_grad(tgt, 0)
            torch.cuda.synchronize()
            _same(ref.accumulator(0), st.accumulator(0), f"{name}: accumulator")
            _same(l1, l2, f"{name}: loss")
            _same(g1, g2, f"{name}: gradient")
            say(name, "loss", float(l2[0]), "grad", g2.cpu().numpy()[0].tolist())
        finally:
            st.close()
            del ref


def test_static_scratch_limits(Sim):
    from paper_2502_18738_amd._abi import SIM_E_STATE, SIM_E_WORKSPACE, SimError
    s = synth.make_lakes(64, 80, 13, T=20, n_ignitions=2)
    st = Sim([s], static_scratch=True)
    try:
        # one static handle per device at a time
        with pytest.raises(SimError) as e:
            Sim([s], static_scratch=True)
        assert e.value.code == SIM_E_STATE
    finally:
        st.close()
    # released: a new one may be created (and matches the workspace handle)
    ref, st = _pair(Sim, s)
    try:
        ref.run(20)
        st.run(20)
        _same(ref.get_state(0), st.get_state(0), "after release: state")
    finally:
        st.close()
    big = synth.make_plain(1400, 1400, 14, T=10)
    with pytest.raises(SimError) as e:
        Sim([big], static_scratch=True)
    assert e.value.code == SIM_E_WORKSPACE and "static scratch" in str(e.value)
