"""ctypes declarations of the C ABI in include/lbm.h and include/lbm3d.h (argument
marshalling only).

The HIP library must have been built (``python -m paper_2108_13241_amd.build``); there
is no fallback: loading fails loudly when it is missing.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbm_hip.so")

DTYPES = {"f64": 0, "f32": 1, "f16s": 2, "bf16s": 3}
POP_BYTES = {"f64": 8, "f32": 4, "f16s": 2, "bf16s": 2}
LAYOUTS = {"dense_ab": 0, "dense_aa": 1, "tiled16": 2, "indirect": 3, "tiled16_all": 4}
STATUS = {0: "LBM_OK", -1: "LBM_ERR_INVALID", -2: "LBM_ERR_NOMEM", -3: "LBM_ERR_DEVICE",
          -4: "LBM_ERR_UNSUPPORTED", -5: "LBM_ERR_STATE"}


class LbmError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


class LbmInfo(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("dtype", ctypes.c_int32),
                ("layout", ctypes.c_int32), ("n_nodes", ctypes.c_int64),
                ("n_fluid", ctypes.c_int64), ("n_tiles", ctypes.c_int64),
                ("time_step", ctypes.c_int64), ("pop_bytes", ctypes.c_int32),
                ("has_porosity", ctypes.c_int32), ("bytes_per_fluid_node", ctypes.c_double),
                ("bytes_moved_per_step", ctypes.c_double), ("device_bytes", ctypes.c_size_t)]


class Lbm3dInfo(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("dtype", ctypes.c_int32), ("layout", ctypes.c_int32), ("n_nodes", ctypes.c_int64),
                ("n_fluid", ctypes.c_int64), ("time_step", ctypes.c_int64),
                ("pop_bytes", ctypes.c_int32), ("bytes_per_fluid_node", ctypes.c_double),
                ("device_bytes", ctypes.c_size_t)]


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)

# Every function declared in include/*.h: name -> (restype, argtypes).
_c = ctypes
_vp, _dp, _i32, _i64, _sz = _c.c_void_p, _c.POINTER(_c.c_double), _c.c_int32, _c.c_int64, _c.c_size_t
SIGNATURES = {
    "lbm_set_allocator": (_c.c_int, [_vp, _vp, _vp]),
    "lbm_create": (_c.c_int, [_c.POINTER(_vp), _i32, _i32, _c.POINTER(_c.c_uint8), _c.c_double,
                              _dp, _c.c_int, _c.c_int]),
    "lbm_set_stream": (_c.c_int, [_vp, _vp]),
    "lbm_init_equilibrium": (_c.c_int, [_vp, _dp, _dp, _dp]),
    "lbm_set_porosity": (_c.c_int, [_vp, _c.POINTER(_c.c_float)]),
    "lbm_set_boundaries": (_c.c_int, [_vp, _c.c_void_p, _c.c_void_p]),
    "lbm_set_trt": (_c.c_int, [_vp, _c.c_double]),
    "lbm_set_mrt": (_c.c_int, [_vp, _c.c_void_p]),
    "lbm_set_bounce_back": (_c.c_int, [_vp, _i32]),
    "lbm_set_force": (_c.c_int, [_vp, _dp]),
    "lbm_step": (_c.c_int, [_vp, _i64]),
    "lbm_set_graph_steps": (_c.c_int, [_vp, _i32]),
    "lbm_macroscopic": (_c.c_int, [_vp, _dp, _dp, _dp]),
    "lbm_macroscopic_device": (_c.c_int, [_vp, _vp, _vp, _vp]),
    "lbm_get_populations": (_c.c_int, [_vp, _dp]),
    "lbm_set_populations": (_c.c_int, [_vp, _dp]),
    "lbm_mass": (_c.c_int, [_vp, _dp]),
    "lbm_state_bytes": (_c.c_int, [_vp, _c.POINTER(_sz)]),
    "lbm_save_state": (_c.c_int, [_vp, _vp]),
    "lbm_load_state": (_c.c_int, [_vp, _vp]),
    "lbm_objective_outlet_ux": (_c.c_int, [_vp, _i32, _dp]),
    "lbm_adjoint_bytes": (_c.c_int, [_vp, _c.POINTER(_sz), _c.POINTER(_i32)]),
    "lbm_adjoint_get": (_c.c_int, [_vp, _vp, _dp]),
    "lbm_adjoint_set": (_c.c_int, [_vp, _vp, _dp]),
    "lbm_adjoint_seed_outlet_ux": (_c.c_int, [_vp, _i32, _c.c_double, _vp, _vp, _vp]),
    "lbm_adjoint_step": (_c.c_int, [_vp, _vp, _vp, _vp, _vp, _vp]),
    "lbm_adjoint_step_noalloc": (_c.c_int, [_vp, _vp, _vp, _vp, _vp, _vp]),
    "lbm_run_checkpointed": (_c.c_int, [_vp, _i64, _i64, _vp]),
    "lbm_adjoint_checkpointed": (_c.c_int, [_vp, _i64, _i64, _vp, _vp, _i32, _c.c_double, _vp,
                                            _vp]),
    "lbm_get_info": (_c.c_int, [_vp, _c.POINTER(LbmInfo)]),
    "lbm_plan_tiles": (_c.c_int, [_i32, _i32, _c.POINTER(_c.c_uint8), _c.POINTER(_i64),
                                  _c.POINTER(_i32), _c.POINTER(_i32)]),
    "lbm_plan_indirect": (_c.c_int, [_i32, _i32, _c.POINTER(_c.c_uint8), _c.POINTER(_i64),
                                     _c.POINTER(_i32), _c.POINTER(_i32)]),
    "lbm_copy_kernel": (_c.c_int, [_vp, _vp, _sz, _vp]),
    "lbm_error_string": (_c.c_char_p, [_c.c_int]),
    "lbm_last_error": (_c.c_char_p, [_vp]),
    "lbm_destroy": (None, [_vp]),
    # include/lbm3d.h
    "lbm3d_create": (_c.c_int, [_c.POINTER(_vp), _i32, _i32, _i32, _c.POINTER(_c.c_uint8),
                                _c.c_double, _dp, _c.c_int, _c.c_int]),
    "lbm3d_set_stream": (_c.c_int, [_vp, _vp]),
    "lbm3d_set_mrt": (_c.c_int, [_vp, _vp]),
    "lbm3d_macroscopic_device": (_c.c_int, [_vp, _vp, _vp, _vp, _vp]),
    "lbm3d_state_bytes": (_c.c_int, [_vp, _c.POINTER(_c.c_size_t)]),
    "lbm3d_save_state": (_c.c_int, [_vp, _vp]),
    "lbm3d_load_state": (_c.c_int, [_vp, _vp]),
    "lbm3d_init_equilibrium": (_c.c_int, [_vp, _dp, _dp, _dp, _dp]),
    "lbm3d_set_force": (_c.c_int, [_vp, _dp]),
    "lbm3d_set_trt": (_c.c_int, [_vp, _c.c_double]),
    "lbm3d_set_bounce_back": (_c.c_int, [_vp, _i32]),
    "lbm3d_step": (_c.c_int, [_vp, _i64]),
    "lbm3d_macroscopic": (_c.c_int, [_vp, _dp, _dp, _dp, _dp]),
    "lbm3d_get_populations": (_c.c_int, [_vp, _dp]),
    "lbm3d_set_populations": (_c.c_int, [_vp, _dp]),
    "lbm3d_mass": (_c.c_int, [_vp, _dp]),
    "lbm3d_get_info": (_c.c_int, [_vp, _c.POINTER(Lbm3dInfo)]),
    "lbm3d_last_error": (_c.c_char_p, [_vp]),
    "lbm3d_destroy": (None, [_vp]),
}

_lib = None


def load():
    """Load liblbm_hip.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"HIP library not built: {LIB_PATH} is missing "
                              "(run `python -m paper_2108_13241_amd.build`)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(status: int, ctx=None):
    if status != 0:
        msg = load().lbm_last_error(ctx)
        raise LbmError(status, msg.decode() if msg else "")


def check3(status: int, ctx=None):
    if status != 0:
        msg = load().lbm3d_last_error(ctx)
        raise LbmError(status, msg.decode() if msg else "")
