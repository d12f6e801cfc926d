"""ctypes binding of ``libamgp2.so`` (the C ABI in include/amg_p2.h).

Argument marshalling only: every step of setup and solve runs in the
library's HIP kernels and host setup code. Device vectors are torch CUDA
tensors (float64, contiguous); streams are torch CUDA streams. If the library
is missing the binding raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libamgp2.so")

# status codes and options (mirrors amg_p2.h)
AMG_OK, AMG_NOT_CONVERGED, AMG_BREAKDOWN, AMG_DIVERGED = 0, 1, 2, 3
AMG_EINVAL, AMG_EHIP, AMG_ENOMEM, AMG_EUNSUPPORTED = -1, -2, -3, -4
AMG_MEM_HOST, AMG_MEM_DEVICE = 0, 1
SMOOTH = {"JA": 0, "GS": 1, "SGS": 2, "BS": 3, "VANKA": 4}
KRYLOV = {"PCG": 0, "FCG": 1, "FGMRES": 2, "NONE": 3}
PREC = {"FP64": 0, "MIXED": 1, "FP32": 2}
SHAPE = {"natural": 0, "sweep": 1, "natural_rp": 2, "sweep_rp": 3, "vanka": 4, "vanka_apply": 5}

_i32p = ctypes.POINTER(ctypes.c_int32)
_f64p = ctypes.POINTER(ctypes.c_double)
_f32p = ctypes.POINTER(ctypes.c_float)


class AmgSystem(ctypes.Structure):
    _fields_ = [
        ("n_lin", ctypes.c_int32), ("n_quad", ctypes.c_int32), ("n_pres", ctypes.c_int32),
        ("bs", ctypes.c_int32),
        ("A_rowptr", _i32p), ("A_col", _i32p), ("A_val", _f64p),
        ("B_rowptr", _i32p), ("B_col", _i32p), ("B_val", _f64p),
        ("C_rowptr", _i32p), ("C_col", _i32p), ("C_val", _f64p),
        ("pressure_kernel", ctypes.c_int32), ("memory", ctypes.c_int32),
    ]


class AmgParams(ctypes.Structure):
    _fields_ = [
        ("smoother", ctypes.c_int32), ("pre", ctypes.c_int32), ("post", ctypes.c_int32),
        ("omega", ctypes.c_double), ("sgs_omega", ctypes.c_double), ("sgs_damping", ctypes.c_double),
        ("cycles", ctypes.c_int32), ("nu", ctypes.c_int32), ("max_levels", ctypes.c_int32),
        ("coarse_max", ctypes.c_int32), ("separate", ctypes.c_int32), ("krylov", ctypes.c_int32),
        ("restart", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("n_level_omega", ctypes.c_int32), ("level_omega", _f64p),
        ("fuse_coarse", ctypes.c_int32), ("autotune", ctypes.c_int32),
        ("omega_model", ctypes.c_void_p), ("graph", ctypes.c_int32), ("vanka_omega", ctypes.c_double),
        ("gs_post", ctypes.c_int32),
    ]


class AmgResult(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("status", ctypes.c_int32),
                ("relres", ctypes.c_double), ("solve_ms", ctypes.c_double)]


class AmgLevelInfo(ctypes.Structure):
    _fields_ = [
        ("n_lin", ctypes.c_int32), ("n_quad", ctypes.c_int32), ("n_pres", ctypes.c_int32),
        ("bs", ctypes.c_int32),
        ("nnz_A", ctypes.c_int64), ("nnz_B", ctypes.c_int64), ("nnz_C", ctypes.c_int64),
        ("nnz_P", ctypes.c_int64),
        ("n_colors", ctypes.c_int32), ("is_coarsest", ctypes.c_int32),
        ("lanes_A", ctypes.c_int32), ("lanes_gs", ctypes.c_int32), ("fused", ctypes.c_int32),
        ("omega", ctypes.c_double), ("schur_levels", ctypes.c_int32), ("nnz_S", ctypes.c_int64),
        ("gs_xcd", ctypes.c_int32), ("trip_A", ctypes.c_int32), ("trip_gs", ctypes.c_int32),
        ("lanes64_A", ctypes.c_int32), ("trip64_A", ctypes.c_int32),
        ("kept_A", ctypes.c_int64), ("kept_B", ctypes.c_int64),
        ("coarse_map", ctypes.c_int32), ("learned", ctypes.c_int32), ("omega_max", ctypes.c_double),
        ("omega_fallbacks", ctypes.c_int32),
    ]


# every entry point declared in include/amg_p2.h, with its signature
_H = ctypes.c_void_p
_S = ctypes.c_void_p
SIGNATURES = {
    "amg_default_params": (None, [ctypes.POINTER(AmgParams)]),
    "amg_setup": (ctypes.c_int, [ctypes.POINTER(AmgSystem), ctypes.POINTER(AmgParams), _S,
                                 ctypes.POINTER(_H)]),
    "amg_solve": (ctypes.c_int, [_H, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double, ctypes.c_int32, _S,
                                 ctypes.POINTER(AmgResult)]),
    "amg_solve_multi": (ctypes.c_int, [_H, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double,
                                       ctypes.c_int32, _S, ctypes.POINTER(AmgResult)]),
    "amg_precondition": (ctypes.c_int, [_H, ctypes.c_void_p, ctypes.c_void_p, _S]),
    "amg_apply": (ctypes.c_int, [_H, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, _S]),
    "amg_smooth": (ctypes.c_int, [_H, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, _S]),
    "amg_num_levels": (ctypes.c_int, [_H]),
    "amg_get_level_info": (ctypes.c_int, [_H, ctypes.c_int32, ctypes.POINTER(AmgLevelInfo)]),
    "amg_get_level_matrix": (ctypes.c_int, [_H, ctypes.c_int32, ctypes.c_int32, _i32p, _i32p, _f64p]),
    "amg_get_level_colors": (ctypes.c_int, [_H, ctypes.c_int32, _i32p]),
    "amg_set_launch_shape": (ctypes.c_int, [_H, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                            ctypes.c_int32]),
    "amg_profile_enable": (ctypes.c_int, [_H, ctypes.c_int32]),
    "amg_profile_read": (ctypes.c_int, [_H, ctypes.c_char_p, ctypes.POINTER(ctypes.c_int64),
                                        ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]),
    "amg_destroy": (None, [_H]),
    "amg_setup_batched": (ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(AmgSystem), ctypes.POINTER(AmgParams), _S,
                                         ctypes.POINTER(_H)]),
    "amg_solve_batched": (ctypes.c_int, [_H, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double, ctypes.c_int32, _S,
                                         ctypes.POINTER(AmgResult)]),
    "amg_batch_offsets": (ctypes.c_int, [_H, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]),
    "amg_mlp_create": (ctypes.c_int, [_f32p, _S, ctypes.POINTER(ctypes.c_void_p)]),
    "amg_mlp_get_params": (ctypes.c_int, [ctypes.c_void_p, _f32p]),
    "amg_mlp_forward": (ctypes.c_int, [ctypes.c_void_p, _f32p, ctypes.c_int32, _f32p]),
    "amg_mlp_gradient": (ctypes.c_int, [ctypes.c_void_p, _f32p, _f32p, ctypes.c_int32, _f32p, _f32p]),
    "amg_mlp_train": (ctypes.c_int, [ctypes.c_void_p, _f32p, _f32p, ctypes.c_int32, ctypes.c_int32,
                                     ctypes.c_float, _f32p]),
    "amg_mlp_destroy": (None, [ctypes.c_void_p]),
    "amg_level_features": (ctypes.c_int, [_H, ctypes.c_int32, _f64p]),
    "amg_level_features_noalloc": (ctypes.c_int, [_H, ctypes.c_int32, ctypes.c_void_p, _S]),
    "amg_set_level_omega": (ctypes.c_int, [_H, ctypes.c_int32, _f64p]),
    "amg_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "amg_last_error": (ctypes.c_char_p, []),
}

_lib = None


class AmgError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        msg = ""
        if _lib is not None:
            msg = (_lib.amg_last_error() or b"").decode()
        super().__init__(f"{where}: status {code} ({status_string(code)}): {msg}")


def lib() -> ctypes.CDLL:
    """Load the HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} not found: build it with "
                               "`python -m paper_1503_01287_amd.build` (no CPU fallback exists)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def status_string(code: int) -> str:
    return lib().amg_status_string(int(code)).decode()


def check(code: int, where: str) -> int:
    if code < 0:
        raise AmgError(code, where)
    return code


def _ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def default_params() -> AmgParams:
    p = AmgParams()
    lib().amg_default_params(ctypes.byref(p))
    return p
