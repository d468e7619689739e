"""ctypes declarations of libfiresim's C ABI (include/firesim.h).

Loading fails loudly when the library has not been built: there is no
fallback implementation of any entry point.
"""

from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfiresim.so")

SIM_OK = 0
SIM_E_ARG = -1
SIM_E_SHAPE = -2
SIM_E_PARAM = -3
SIM_E_WORKSPACE = -4
SIM_E_HIP = -5
SIM_E_STATE = -6

SIM_F_CALIB = 1
SIM_F_STATS = 2
SIM_F_TIELOG = 4
SIM_TIELOG_CAP = 1 << 20
SIM_STATIC_SCRATCH_BYTES = 128 << 20

SIM_LOSS_BCE = 0
SIM_LOSS_BCE_MSE = 1
SIM_LOSS_MSE = 2

SIM_ADJ_CHECKPOINT = 0
SIM_ADJ_TIMEMAP = 1

ERROR_NAMES = {
    SIM_E_ARG: "SIM_E_ARG", SIM_E_SHAPE: "SIM_E_SHAPE", SIM_E_PARAM: "SIM_E_PARAM",
    SIM_E_WORKSPACE: "SIM_E_WORKSPACE", SIM_E_HIP: "SIM_E_HIP", SIM_E_STATE: "SIM_E_STATE",
}


class sim_params(ctypes.Structure):
    _fields_ = [("p_h", ctypes.c_float), ("a", ctypes.c_float), ("c1", ctypes.c_float),
                ("c2", ctypes.c_float), ("p_continue", ctypes.c_float)]


class sim_fields(ctypes.Structure):
    _fields_ = [("p_veg", ctypes.c_void_p), ("p_den", ctypes.c_void_p),
                ("elevation_m", ctypes.c_void_p), ("wind_speed", ctypes.c_void_p),
                ("wind_dir_deg", ctypes.c_void_p), ("wind_speed_scalar", ctypes.c_float),
                ("wind_dir_deg_scalar", ctypes.c_float), ("init_burning", ctypes.c_void_p),
                ("slope_deg", ctypes.c_void_p)]


class sim_desc(ctypes.Structure):
    _fields_ = [("H", ctypes.c_int32), ("W", ctypes.c_int32), ("cell_m", ctypes.c_float),
                ("scenario_id", ctypes.c_uint32), ("seed", ctypes.c_uint64),
                ("params", sim_params), ("f", sim_fields)]


class sim_tie(ctypes.Structure):
    _fields_ = [("scenario", ctypes.c_int32), ("step", ctypes.c_int32), ("cell", ctypes.c_int64),
                ("p_ignite", ctypes.c_float), ("draw", ctypes.c_float),
                ("ignited", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class sim_exec(ctypes.Structure):
    _fields_ = [("tile_rows", ctypes.c_int32), ("tile_words", ctypes.c_int32),
                ("depth", ctypes.c_int32), ("skip", ctypes.c_int32),
                ("threads", ctypes.c_int32)]


EXPORTS = (
    "sim_workspace_size", "sim_init", "sim_set_exec", "sim_get_exec", "sim_run", "sim_step",
    "sim_get_step", "sim_set_params", "sim_reset", "sim_get_state", "sim_set_state",
    "sim_pignite", "sim_accumulator", "sim_adjoint", "sim_loss_grad", "sim_stats",
    "sim_last_error", "sim_destroy", "sim_version", "sim_autotune", "sim_use_graphs",
    "sim_set_adjoint", "sim_set_wind", "sim_ignite", "sim_counts", "sim_overlap", "sim_arrival", "sim_tielog",
    "sim_metrics", "sim_prepare", "sim_init_static", "sim_set_params_device",
    "sim_params_rejected",
)

_lib = None


def load():
    """Load libfiresim.so and declare every entry point's signature."""
    global _lib
    if _lib is not None:
        return _lib
    # torch ships its own HIP runtime under the same soname; load it first so
    # that the library binds to the runtime that owns torch's streams and memory
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with `python -m paper_2502_18738_amd.build` "
            "(the HIP library is the only implementation)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, u32, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint32, ctypes.c_size_t
    H = vp  # sim_handle*
    sig = {
        "sim_workspace_size": (sz, [ctypes.POINTER(sim_desc), i32, u32, i32, i32]),
        "sim_init": (ctypes.c_int, [ctypes.POINTER(vp), ctypes.POINTER(sim_desc), i32, vp, sz,
                                    vp, u32, i32, i32]),
        "sim_init_static": (ctypes.c_int, [ctypes.POINTER(vp), ctypes.POINTER(sim_desc), i32,
                                           vp, u32, i32, i32]),
        "sim_set_exec": (ctypes.c_int, [H, ctypes.POINTER(sim_exec)]),
        "sim_get_exec": (ctypes.c_int, [H, ctypes.POINTER(sim_exec)]),
        "sim_run": (ctypes.c_int, [H, i32]),
        "sim_step": (ctypes.c_int, [H]),
        "sim_get_step": (ctypes.c_int, [H, ctypes.POINTER(i32)]),
        "sim_set_params": (ctypes.c_int, [H, ctypes.POINTER(sim_params)]),
        "sim_set_params_device": (ctypes.c_int, [H, vp]),
        "sim_params_rejected": (ctypes.c_int, [H, ctypes.POINTER(i32)]),
        "sim_reset": (ctypes.c_int, [H, ctypes.POINTER(ctypes.c_uint64)]),
        "sim_get_state": (ctypes.c_int, [H, i32, vp]),
        "sim_set_state": (ctypes.c_int, [H, i32, vp, i32]),
        "sim_pignite": (ctypes.c_int, [H, i32, vp]),
        "sim_accumulator": (ctypes.c_int, [H, i32, vp]),
        "sim_adjoint": (ctypes.c_int, [H, vp, vp]),
        "sim_loss_grad": (ctypes.c_int, [H, vp, i32, vp, vp]),
        "sim_stats": (ctypes.c_int, [H, ctypes.POINTER(ctypes.c_uint64)]),
        "sim_last_error": (ctypes.c_char_p, [H]),
        "sim_destroy": (None, [H]),
        "sim_version": (ctypes.c_char_p, []),
        "sim_autotune": (ctypes.c_int, [H, i32, ctypes.POINTER(sim_exec)]),
        "sim_use_graphs": (ctypes.c_int, [H, i32]),
        "sim_set_adjoint": (ctypes.c_int, [H, i32, i32, i32, i32]),
        "sim_set_wind": (ctypes.c_int, [H, i32, vp, vp, ctypes.c_float, ctypes.c_float]),
        "sim_ignite": (ctypes.c_int, [H, i32, vp, i32]),
        "sim_counts": (ctypes.c_int, [H, vp]),
        "sim_overlap": (ctypes.c_int, [H, i32, vp, vp]),
        "sim_arrival": (ctypes.c_int, [H, i32, i32, vp]),
        "sim_metrics": (ctypes.c_int, [H, vp, vp]),
        "sim_prepare": (ctypes.c_int, [H, i32]),
        "sim_tielog": (ctypes.c_int, [H, vp, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class SimError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code
