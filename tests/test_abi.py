"""Host-side checks of the C-ABI library: it loads, exports every function that
include/mpcr.h declares, and its pure host helpers (precision maps, argument
checks) behave as documented.  No GPU is needed: nothing here launches a kernel.
"""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mpcr.h")

mpcr = pytest.importorskip("paper_2406_02701_amd.mpcr", reason="libmpcr.so not built")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\*?\s+\**(mpcr_\w+)\s*\(", text, flags=re.M)))


def test_every_declared_symbol_is_exported():
    names = declared_functions()
    assert len(names) >= 18
    lib = ctypes.CDLL(mpcr.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert set(names) <= set(mpcr._SIGS), set(names) - set(mpcr._SIGS)


def test_version_names_target():
    assert b"gfx950" in mpcr.mpcr_version()


def _banded(n, nb, dmax, precs):
    nt = (n + nb - 1) // nb
    out = np.zeros((nt, nt), np.uint8)
    d = (ctypes.c_int * len(dmax))(*dmax)
    p = (ctypes.c_int * len(precs))(*precs)
    st = mpcr.mpcr_tilemap_banded(n, nb, d, p, len(dmax), out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)))
    return st, out


def test_banded_map_matches_oracle():
    from oracle import tiled
    st, m = _banded(32768, 512, [2, 8, -1], [0, 1, 3])
    assert st == 0
    ref = tiled.tilemap_banded(32768, 512, ((2, "fp64"), (8, "fp32"), (None, "bf16")))
    assert np.array_equal(m, ref)
    st, m = _banded(1000, 256, [0, -1], [0, 2])
    ref = tiled.tilemap_banded(1000, 256, ((0, "fp64"), (None, "fp16")))
    assert st == 0 and np.array_equal(m, ref)


def test_banded_map_rejects_low_precision_diagonal():
    st, _ = _banded(1024, 256, [-1], [1])
    assert st == mpcr.MPCR_ERR_ARG
    st, _ = _banded(1024, 256, [1], [0])   # distance 2 has no band
    assert st == mpcr.MPCR_ERR_ARG


def test_guarded_map_promotes_large_tiles():
    nt = 4
    banded = np.full((nt, nt), 255, np.uint8)
    for i in range(nt):
        for j in range(i + 1):
            banded[i, j] = 0 if i == j else 3
    amax = np.zeros((nt, nt))
    amax[1, 0], amax[2, 0], amax[3, 0] = 1.0, 1e-3, 1e-9
    amax[2, 1], amax[3, 1], amax[3, 2] = 0.5, 1e-6, 1e-5
    out = np.zeros((nt, nt), np.uint8)
    st = mpcr.mpcr_tilemap_guarded(nt * 128, 128, banded.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                                   mpcr.f64p(amax), 1e-7, out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)))
    assert st == 0
    # bf16 kept iff 2^-8 amax <= 1e-7; fp32 iff 2^-24 amax <= 1e-7; else fp64
    for i in range(nt):
        for j in range(i):
            a = amax[i, j]
            want = 3 if 2.0 ** -8 * a <= 1e-7 else (1 if 2.0 ** -24 * a <= 1e-7 else 0)
            assert out[i, j] == want, (i, j, out[i, j], want)
    assert all(out[i, i] == 0 for i in range(nt))


def test_guarded_map_fp16_subnormal_floor():
    """FP16 rounds values below its normal range (6.1e-5) with absolute error
    up to 2^-25 ~ 3.0e-8: with a guard below that, FP16 is never kept, however
    small the tile; above it, the relative rule decides."""
    nt = 3
    banded = np.full((nt, nt), 255, np.uint8)
    for i in range(nt):
        for j in range(i + 1):
            banded[i, j] = 0 if i == j else 2
    amax = np.zeros((nt, nt))
    amax[1, 0], amax[2, 0], amax[2, 1] = 1e-9, 1e-4, 1e-12
    for guard, want in ((1e-8, 1), (1e-7, 2)):
        out = np.zeros((nt, nt), np.uint8)
        st = mpcr.mpcr_tilemap_guarded(nt * 128, 128, banded.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                                       mpcr.f64p(amax), guard, out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)))
        assert st == 0
        assert out[1, 0] == want and out[2, 1] == want
        # 2^-11 * 1e-4 = 4.9e-8: FP16 only under the looser guard
        assert out[2, 0] == (2 if 2.0 ** -11 * 1e-4 <= guard else 1)


def test_null_context_arguments_are_rejected():
    assert mpcr.mpcr_ctx_create(0, None, None) == mpcr.MPCR_ERR_ARG
    assert mpcr.mpcr_ctx_destroy(None) == mpcr.MPCR_ERR_ARG
    assert mpcr.mpcr_factor_destroy(None) == mpcr.MPCR_ERR_ARG
    th = mpcr.mpcr_theta_t(1.0, 0.1, 0.5, 0.0)
    assert mpcr.mpcr_gauss_loglik(None, 10, None, None, 1, ctypes.byref(th), None, 1, None, None, None) \
        == mpcr.MPCR_ERR_ARG
    assert mpcr.mpcr_gemm(None, 0, 0, 0, 1, 1, 1, 1.0, None, 1, None, None, 1, None, 0.0, None, 1, 0) \
        == mpcr.MPCR_ERR_ARG
