"""ctypes binding of libmpcr.so (the C interface declared in include/mpcr.h).

Argument marshalling only: every function below forwards to the C entry point
of the same name.  Device buffers are passed as integer addresses (for example
``tensor.data_ptr()`` of a torch tensor on the GPU), host arrays as numpy
arrays or ctypes pointers.  Importing this module raises ImportError when the
library has not been built; there is no fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmpcr.so")

MPCR_FP64, MPCR_FP32, MPCR_FP16, MPCR_BF16, MPCR_FP8_E4M3 = 0, 1, 2, 3, 4
MPCR_OK = 0
MPCR_ERR_ARG = -1
MPCR_ERR_NOT_SPD = -2
MPCR_ERR_NOT_CONVERGED = -3
MPCR_ERR_NOMEM = -4
MPCR_ERR_DEVICE = -5
MPCR_ERR_REJECTED = -6
STATUS_NAMES = {0: "OK", -1: "ERR_ARG", -2: "ERR_NOT_SPD", -3: "ERR_NOT_CONVERGED", -4: "ERR_NOMEM",
                -5: "ERR_DEVICE", -6: "ERR_REJECTED"}
PREC = {"fp64": 0, "fp32": 1, "fp16": 2, "bf16": 3, "fp8_e4m3": 4, "fp8": 4}


class mpcr_tilemap_t(C.Structure):
    _fields_ = [("n", C.c_int64), ("nb", C.c_int64), ("nt", C.c_int64), ("h_map", C.POINTER(C.c_uint8))]


class mpcr_theta_t(C.Structure):
    _fields_ = [("sigma2", C.c_double), ("range", C.c_double), ("nu", C.c_double), ("nugget", C.c_double)]


class mpcr_refine_opts_t(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iter", C.c_int), ("solver", C.c_int), ("recompute", C.c_int),
                ("residual", C.c_int), ("promote_on_breakdown", C.c_int), ("direct_eta", C.c_int),
                ("gmres_m", C.c_int), ("gmres_inner_tol", C.c_double), ("block_size", C.c_int)]


class mpcr_diag_t(C.Structure):
    _fields_ = [("iters", C.c_int), ("converged", C.c_int), ("eta", C.c_double), ("rel_resid2", C.c_double),
                ("logdet", C.c_double), ("quad0", C.c_double), ("info", C.c_int64),
                ("t_gen_ms", C.c_double), ("t_factor_ms", C.c_double), ("t_solve_ms", C.c_double),
                ("t_refine_ms", C.c_double), ("flops_by_prec", C.c_double * 5), ("promotions", C.c_int)]


# The library must share the process's HIP runtime with PyTorch, which ships its
# own copy of libamdhip64: load torch first so that libmpcr binds to that one.
try:
    import torch  # noqa: F401
except ImportError:  # no torch: the system HIP runtime is used
    torch = None

class mpcr_serve_opts_t(C.Structure):
    _fields_ = [("nb", C.c_int64), ("band_fp64", C.c_int), ("band_fp32", C.c_int), ("far_prec", C.c_int),
                ("guard", C.c_double), ("refine", mpcr_refine_opts_t), ("fallback_fp64", C.c_int)]


if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built (run __graft_entry__.build() or "
                      "python -m paper_2406_02701_amd.build)")
lib = C.CDLL(LIB_PATH)

_vp, _i64, _i32, _d = C.c_void_p, C.c_int64, C.c_int, C.c_double
_P = C.POINTER
# name: (restype, argtypes)
_SIGS = {
    "mpcr_version": (C.c_char_p, []),
    "mpcr_ctx_create": (_i32, [_i32, _vp, _P(_vp)]),
    "mpcr_ctx_destroy": (_i32, [_vp]),
    "mpcr_last_error": (C.c_char_p, [_vp]),
    "mpcr_ctx_set_profiling": (_i32, [_vp, _i32]),
    "mpcr_ctx_set_fp32_split": (_i32, [_vp, _i32]),
    "mpcr_ctx_reset_stats": (_i32, [_vp]),
    "mpcr_ctx_kernel_stats": (_i32, [_vp, _i32, _P(_d), _P(_i64), _P(_d)]),
    "mpcr_tilemap_banded": (_i32, [_i64, _i64, _P(_i32), _P(_i32), _i32, _P(C.c_uint8)]),
    "mpcr_tilemap_guarded": (_i32, [_i64, _i64, _P(C.c_uint8), _P(_d), _d, _P(C.c_uint8)]),
    "mpcr_morton_order": (_i32, [_vp, _i64, _vp, _vp]),
    "mpcr_morton_order_noalloc": (_i32, [_vp, _i64, _vp, _vp]),
    "mpcr_covariance": (_i32, [_vp, _i64, _vp, _P(mpcr_theta_t), _vp, _i64]),
    "mpcr_covariance_tile_amax": (_i32, [_vp, _i64, _i64, _vp, _P(mpcr_theta_t), _P(_d)]),
    "mpcr_potrf_tiled": (_i32, [_vp, _i64, _vp, _i64, _P(mpcr_tilemap_t), _P(_vp), _P(_i64)]),
    "mpcr_potrf_tiled_covariance": (_i32, [_vp, _i64, _vp, _P(mpcr_theta_t), _P(mpcr_tilemap_t), _P(_vp),
                                           _P(_i64)]),
    "mpcr_factor_destroy": (_i32, [_vp]),
    "mpcr_factor_logdet": (_i32, [_vp, _vp, _P(_d)]),
    "mpcr_factor_to_dense": (_i32, [_vp, _vp, _vp, _i64]),
    "mpcr_factor_flops": (_i32, [_vp, _P(_d)]),
    "mpcr_trsm_forward": (_i32, [_vp, _vp, _i64, _vp, _i64, _vp, _i64]),
    "mpcr_potrs": (_i32, [_vp, _vp, _i64, _vp, _i64, _vp, _i64, _vp, _i64, _P(mpcr_refine_opts_t),
                          _P(mpcr_diag_t)]),
    "mpcr_gauss_loglik": (_i32, [_vp, _i64, _vp, _vp, _i64, _P(mpcr_theta_t), _P(mpcr_tilemap_t), _i32,
                                 _P(mpcr_refine_opts_t), _P(_d), _P(mpcr_diag_t)]),
    "mpcr_loglik_map": (_i32, [_vp, _P(_i64), _P(C.c_uint8), _i64]),
    "mpcr_mle_fit": (_i32, [_vp, _i64, _vp, _vp, _d, _d, _P(mpcr_tilemap_t), _P(mpcr_refine_opts_t), _P(_d), _i32,
                            _d, _P(_d), _P(_d), _P(_i32), _P(_i32)]),
    "mpcr_inla_posterior": (_i32, [_vp, _i64, _vp, _vp, _d, _d, _d, _P(_d), _i32, _d, _i32, _P(mpcr_tilemap_t),
                                   _P(_d), _P(_d), _P(_i32), _vp]),
    "mpcr_mala_run": (_i32, [_vp, _i64, _vp, _P(mpcr_theta_t), _P(mpcr_theta_t), _d, _vp, _i32, _vp, _P(_d),
                             _P(mpcr_tilemap_t), _vp, _vp, _P(_i32), _P(_d)]),
    "mpcr_convert": (_i32, [_vp, _i32, _i64, _i64, _vp, _i64, _vp, _i64, _vp]),
    "mpcr_serve_create": (_i32, [_i32, C.c_size_t, _i32, _P(mpcr_serve_opts_t), _P(_vp)]),
    "mpcr_serve_destroy": (_i32, [_vp]),
    "mpcr_serve_submit": (_i32, [_vp, C.c_uint64, _i64, _P(_d), _P(_d), _P(mpcr_theta_t)]),
    "mpcr_serve_poll": (_i32, [_vp, _P(C.c_uint64), _P(_d), _P(mpcr_diag_t), _P(_d), _P(_d), _P(_i32), _P(_i32)]),
    "mpcr_serve_clock": (_d, [_vp]),
    "mpcr_serve_stats": (_i32, [_vp, _P(_i64), _P(_i64), _P(_i64), _P(_i64), _P(C.c_size_t)]),
    "mpcr_serve_footprint": (C.c_size_t, [_i64, _i64]),
    "mpcr_gemm": (_i32, [_vp, _i32, _i32, _i32, _i64, _i64, _i64, _d, _vp, _i64, _vp, _vp, _i64, _vp, _d, _vp,
                         _i64, _i32]),
}

for _name, (_res, _args) in _SIGS.items():
    _f = getattr(lib, _name)
    _f.restype = _res
    _f.argtypes = _args
    globals()[_name] = _f


class MpcrError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


def check(status: int, ctx=None) -> int:
    """Raise MpcrError for a non-zero status (with the context's last error)."""
    if status != MPCR_OK:
        msg = mpcr_last_error(ctx).decode()
        raise MpcrError(status, msg)
    return status


def tilemap(n: int, nb: int, h_map: np.ndarray) -> mpcr_tilemap_t:
    """mpcr_tilemap_t over a host uint8 array (kept alive by the caller)."""
    nt = (n + nb - 1) // nb
    assert h_map.dtype == np.uint8 and h_map.shape == (nt, nt) and h_map.flags.c_contiguous
    return mpcr_tilemap_t(n, nb, nt, h_map.ctypes.data_as(_P(C.c_uint8)))


def f64p(a: np.ndarray):
    return a.ctypes.data_as(_P(C.c_double))
