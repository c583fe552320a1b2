"""Helpers for the GPU tests: device buffers in column-major order and a library
context bound to torch's current stream."""
import ctypes

import numpy as np
import torch

from paper_2406_02701_amd import mpcr


def dev(x: np.ndarray, dtype=None) -> torch.Tensor:
    """Device copy of x laid out column-major (Fortran order)."""
    x = np.asarray(x)
    if dtype is not None:
        x = x.astype(dtype)
    if x.ndim == 2:
        return torch.from_numpy(np.ascontiguousarray(x.T)).cuda()
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def host(t: torch.Tensor, shape=None) -> np.ndarray:
    """numpy array of a column-major device buffer of the given (rows, cols)."""
    a = t.detach().cpu().numpy()
    if shape is not None and len(shape) == 2:
        return np.asfortranarray(a.reshape(shape[1], shape[0]).T)
    return a


def empty(rows, cols, dtype=torch.float64) -> torch.Tensor:
    return torch.zeros((cols, rows), dtype=dtype, device="cuda")


class Ctx:
    def __init__(self):
        self.ptr = ctypes.c_void_p()
        stream = torch.cuda.current_stream().cuda_stream
        mpcr.check(mpcr.mpcr_ctx_create(0, ctypes.c_void_p(stream), ctypes.byref(self.ptr)))

    def check(self, st):
        return mpcr.check(st, self.ptr)

    def close(self):
        mpcr.mpcr_ctx_destroy(self.ptr)


def theta(sigma2, range_, nu, nugget):
    return mpcr.mpcr_theta_t(sigma2, range_, nu, nugget)


def u8map(m: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(m.astype(np.uint8))


def guarded_map(ctx, locs: np.ndarray, th, n: int, nb: int, start: np.ndarray, guard: float) -> np.ndarray:
    """The norm-guarded version of `start` for the Morton-ordered covariance of
    `locs` (per-tile max |Sigma| from the library, then mpcr_tilemap_guarded)."""
    dl = dev(locs)
    perm = torch.zeros(n, dtype=torch.int64, device="cuda")
    ctx.check(mpcr.mpcr_morton_order(ctx.ptr, n, dl.data_ptr(), perm.data_ptr()))
    dls = dev(locs[perm.cpu().numpy()])
    nt = start.shape[0]
    amax = np.zeros((nt, nt))
    ctx.check(mpcr.mpcr_covariance_tile_amax(ctx.ptr, n, nb, dls.data_ptr(), ctypes.byref(th), mpcr.f64p(amax)))
    out = np.zeros_like(start)
    st0 = np.ascontiguousarray(start.astype(np.uint8))
    mpcr.check(mpcr.mpcr_tilemap_guarded(n, nb, st0.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), mpcr.f64p(amax),
                                         guard, out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))))
    torch.cuda.synchronize()
    return out
