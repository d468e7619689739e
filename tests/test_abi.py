"""C-ABI checks that need no GPU: the library loads, exports every entry point
that include/firesim.h declares, and rejects bad arguments on the host before
any GPU work (so these calls never touch a device)."""

import ctypes
import os
import re

import pytest

from paper_2502_18738_amd import _abi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "firesim.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_abi.LIB_PATH):
        from paper_2502_18738_amd import build
        build.build()
    return _abi.load()


def declared_symbols():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^SIM_API\s+[\w\s\*]+?\b(sim_\w+)\s*\(", text, re.M)))


def test_header_declares_every_binding_export():
    assert declared_symbols() == sorted(_abi.EXPORTS)


def test_library_exports_every_declared_symbol(lib):
    for name in declared_symbols():
        assert hasattr(lib, name), name
    assert lib.sim_version().decode().startswith("firesim")


def test_struct_layout_matches_header():
    # sizes follow from the header's field order on LP64
    assert ctypes.sizeof(_abi.sim_params) == 20
    assert ctypes.sizeof(_abi.sim_fields) == 64
    assert ctypes.sizeof(_abi.sim_desc) == 24 + 20 + 4 + 64
    assert ctypes.sizeof(_abi.sim_exec) == 20
    assert ctypes.sizeof(_abi.sim_tie) == 32


def fake_desc(H=64, W=80, **kw):
    f = _abi.sim_fields(0x1000, 0x2000, 0x3000, None, None, 5.0, 45.0, 0x4000, None)
    p = _abi.sim_params(0.58, 0.078, 0.045, 0.131, 0.3)
    d = _abi.sim_desc(H, W, 30.0, 0, 1, p, f)
    for k, v in kw.items():
        setattr(d, k, v)
    return d


def test_workspace_size_host_only(lib):
    d = (_abi.sim_desc * 2)(fake_desc(), fake_desc(H=33, W=129))
    n1 = lib.sim_workspace_size(d, 2, 0, 0, 0)
    n2 = lib.sim_workspace_size(d, 2, _abi.SIM_F_CALIB, 20, 200)
    assert n1 > 64 * 80 * 16 and n2 > n1
    assert n1 % 256 == 0
    # invalid inputs give 0
    assert lib.sim_workspace_size(d, 0, 0, 0, 0) == 0
    assert lib.sim_workspace_size(d, 2, _abi.SIM_F_CALIB, 0, 200) == 0
    bad = (_abi.sim_desc * 1)(fake_desc(H=0))
    assert lib.sim_workspace_size(bad, 1, 0, 0, 0) == 0


def _init(lib, descs, n, ws, nbytes, flags=0, ck=0, T=0):
    h = ctypes.c_void_p()
    rc = lib.sim_init(ctypes.byref(h), descs, n, ws, nbytes, None, flags, ck, T)
    return rc, h, lib.sim_last_error(None).decode()


@pytest.mark.parametrize("mutate,code,frag", [
    (lambda d: setattr(d, "H", -3), _abi.SIM_E_SHAPE, "H, W"),
    (lambda d: setattr(d, "W", 1 << 20), _abi.SIM_E_SHAPE, "H, W"),
    (lambda d: setattr(d, "cell_m", 0.0), _abi.SIM_E_PARAM, "cell_m"),
    (lambda d: setattr(d.params, "p_h", float("nan")), _abi.SIM_E_PARAM, "finite"),
    (lambda d: setattr(d.params, "p_continue", 1.5), _abi.SIM_E_PARAM, "p_continue"),
    (lambda d: setattr(d.f, "p_veg", None), _abi.SIM_E_ARG, "NULL"),
    (lambda d: setattr(d.f, "elevation_m", 0x3002), _abi.SIM_E_ARG, "aligned"),
    (lambda d: setattr(d.f, "wind_speed_scalar", -1.0), _abi.SIM_E_PARAM, "wind_speed"),
])
def test_init_rejects_bad_descriptions(lib, mutate, code, frag):
    d = fake_desc()
    mutate(d)
    descs = (_abi.sim_desc * 1)(d)
    rc, h, msg = _init(lib, descs, 1, 0x100000, 1 << 30)
    assert rc == code and not h.value and frag in msg


def test_init_rejects_workspace_problems(lib):
    descs = (_abi.sim_desc * 1)(fake_desc())
    need = lib.sim_workspace_size(descs, 1, 0, 0, 0)
    rc, h, msg = _init(lib, descs, 1, None, need)
    assert rc == _abi.SIM_E_ARG and "workspace" in msg
    rc, h, msg = _init(lib, descs, 1, 0x100010, need)
    assert rc == _abi.SIM_E_WORKSPACE and "aligned" in msg
    rc, h, msg = _init(lib, descs, 1, 0x100000, need - 256)
    assert rc == _abi.SIM_E_WORKSPACE and "too small" in msg
    rc, h, msg = _init(lib, descs, 1, 0x100000, need, flags=_abi.SIM_F_CALIB, ck=0, T=10)
    assert rc == _abi.SIM_E_SHAPE
    rc, h, msg = _init(lib, descs, 1, 0x100000, need, flags=0x80)
    assert rc == _abi.SIM_E_ARG and "flag" in msg
    rc = lib.sim_init(None, descs, 1, 0x100000, need, None, 0, 0, 0)
    assert rc == _abi.SIM_E_ARG


def test_null_handle_calls_are_rejected(lib):
    assert lib.sim_run(None, 1) == _abi.SIM_E_ARG
    assert lib.sim_get_state(None, 0, None) == _abi.SIM_E_ARG
    assert lib.sim_adjoint(None, None, None) == _abi.SIM_E_ARG
    assert lib.sim_set_params_device(None, None) == _abi.SIM_E_ARG
    assert lib.sim_params_rejected(None, None) == _abi.SIM_E_ARG
    lib.sim_destroy(None)


def test_init_static_rejects_before_any_gpu_work(lib):
    """Size and argument checks of sim_init_static run on the host first."""
    h = ctypes.c_void_p()
    big = (_abi.sim_desc * 1)(fake_desc(H=1400, W=1400))
    assert lib.sim_workspace_size(big, 1, 0, 0, 0) > _abi.SIM_STATIC_SCRATCH_BYTES
    rc = lib.sim_init_static(ctypes.byref(h), big, 1, None, 0, 0, 0)
    assert rc == _abi.SIM_E_WORKSPACE and not h.value
    assert "static scratch" in lib.sim_last_error(None).decode()
    small = (_abi.sim_desc * 1)(fake_desc())
    assert lib.sim_init_static(ctypes.byref(h), small, 1, None, 0x80, 0, 0) == _abi.SIM_E_ARG
    assert lib.sim_init_static(ctypes.byref(h), small, 1, None, _abi.SIM_F_CALIB, 0, 10) \
        == _abi.SIM_E_SHAPE
    assert lib.sim_init_static(None, small, 1, None, 0, 0, 0) == _abi.SIM_E_ARG
