"""Elementwise GPU parity of the mixed-precision tile factor against the
emulated oracle at the tile sizes of the large workloads (through the C-ABI).

* nb = 256, 33 tiles per dimension with a ragged last tile: the updates run on
  two 128-row sub-blocks per tile and the factorisation takes the next-column
  stream (more than 32 tiles); five formats (FP64, FP32, BF16, FP16 and FP8
  with per-tile scales).
* nb = 512 with a BF16 far band (the tile size of the 32768-site workload).
* nb = 1024 with FP16 and FP8 bands (the tile size of the 65536-site workload).

Two inputs.  "dominant": A = 1e4 (I + 1e-5 KMS(rho)) with rho close to 1:
every tile, also the far ones, holds entries well inside the low formats'
normal range, the Schur-complement updates are a few percent of the entries
(no cancellation) and cond(A) < 1.05.  The emulation rounds exactly where the
GPU accumulates in FP32, so the two factors differ only where a rounding
flips to the neighbouring value of a format.  Gate per tile:
||dT||_F <= u ||T_emu||_F, with u the tile's own unit roundoff for 16- and
8-bit tiles and, for FP32 and FP64 tiles (which receive the low tiles through
their updates), the coarsest non-FP8 unit roundoff of the map.
"cancelling": KMS(rho) + 10 I, whose far factor entries are small
differences of entries near 1, so that low-precision differences are
amplified; there the factor-level gate 8 u_c sqrt(nt) applies to every
non-FP8 tile and to their whole, u_c the coarsest non-FP8 unit roundoff, and
FP8 tiles are within two FP8 units (2^-3) of the emulation.
Every stored tile must hold values of its format (FP8: of its own scale).
"""
import ctypes
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import fpformat as ff  # noqa: E402
from oracle import tiled  # noqa: E402
from tests.test_oracle_dense import kms  # noqa: E402

CASES = {
    "nb256_nt33_five_formats": dict(n=8448 - 100, nb=256, rho=0.9995, matrix="dominant",
                                    bands=((1, "fp64"), (3, "fp32"), (6, "bf16"), (12, "fp16"),
                                           (None, "fp8_e4m3"))),
    "nb512_bf16": dict(n=4096 - 37, nb=512, rho=0.999, matrix="dominant",
                       bands=((1, "fp64"), (2, "fp32"), (None, "bf16"))),
    "nb512_bf16_cancelling": dict(n=4096 - 37, nb=512, rho=0.999, matrix="cancelling",
                                  bands=((1, "fp64"), (2, "fp32"), (None, "bf16"))),
    "nb1024_fp16_fp8": dict(n=4096, nb=1024, rho=0.9995, matrix="dominant",
                            bands=((0, "fp64"), (1, "fp32"), (2, "fp16"), (None, "fp8_e4m3"))),
    "nb1024_fp16_fp8_cancelling": dict(n=4096, nb=1024, rho=0.9995, matrix="cancelling",
                                       bands=((0, "fp64"), (1, "fp32"), (2, "fp16"), (None, "fp8_e4m3"))),
}


def matrix(c):
    K = kms(c["n"], c["rho"])
    if c["matrix"] == "dominant":
        return np.asfortranarray(1e4 * (np.eye(c["n"]) + 1e-5 * K))
    return np.asfortranarray(K + 10.0 * np.eye(c["n"]))


@pytest.fixture(scope="module")
def g():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from tests import gpu_util
    ctx = gpu_util.Ctx()
    yield gpu_util, ctx
    ctx.close()


@pytest.mark.timeout(900)
@pytest.mark.parametrize("name", list(CASES))
def test_mixed_factor_elementwise_vs_emulation(g, name):
    from paper_2406_02701_amd import mpcr
    gu, ctx = g
    c = CASES[name]
    n, nb = c["n"], c["nb"]
    print(f"case {name}: n {n} nb {nb}", flush=True)
    A = matrix(c)
    m = tiled.tilemap_banded(n, nb, c["bands"])
    nt = m.shape[0]
    dA = gu.dev(A)
    hm = gu.u8map(m)
    tm = mpcr.tilemap(n, nb, hm)
    f = ctypes.c_void_p()
    info = ctypes.c_int64(-1)
    ctx.check(mpcr.mpcr_potrf_tiled(ctx.ptr, n, dA.data_ptr(), n, ctypes.byref(tm), ctypes.byref(f),
                                    ctypes.byref(info)))
    assert info.value == 0
    dL = gu.empty(n, n)
    ctx.check(mpcr.mpcr_factor_to_dense(ctx.ptr, f, dL.data_ptr(), n))
    torch.cuda.synchronize()
    L = gu.host(dL, (n, n))
    del dL, dA
    mpcr.mpcr_factor_destroy(f)
    emu = tiled.tile_cholesky_emulated(A, nb, m)
    assert emu["info"] == 0
    E = emu["L"][:n, :n]
    F8 = ff.CODE["fp8_e4m3"]
    u_c = max(ff.fmt_of(int(m[i, j])).unit_roundoff for i in range(nt) for j in range(i + 1) if m[i, j] != F8)
    tight = c["matrix"] == "dominant"
    gate = u_c if tight else 8 * u_c * math.sqrt(nt)
    worst = {}
    num = den = 0.0
    for i in range(nt):
        for j in range(i + 1):
            sl = (slice(i * nb, min((i + 1) * nb, n)), slice(j * nb, min((j + 1) * nb, n)))
            t, te, p = L[sl], E[sl], int(m[i, j])
            assert np.array_equal(tiled.round_tile(t, p), t), (i, j, p)
            d = np.linalg.norm(t - te)
            ref = np.linalg.norm(te)
            assert ref > 0, (i, j)
            rel = d / ref
            worst[p] = max(worst.get(p, 0.0), rel)
            u_p = ff.fmt_of(p).unit_roundoff
            if p == F8:
                assert rel <= (u_p if tight else 2 * u_p), (i, j, rel)
                continue
            g_t = u_p if (tight and p in (ff.CODE["fp16"], ff.CODE["bf16"])) else gate
            assert rel <= g_t, (i, j, p, rel, g_t)
            num += d * d
            den += ref * ref
    print(f"case {name}: worst per-tile relative difference by format {worst}; gate {gate:.3g}", flush=True)
    assert math.sqrt(num / den) <= gate


@pytest.mark.parametrize("split", [1, 0])
def test_fp32_tiles_match_emulation_both_product_modes(g, split):
    """FP64 near the diagonal, FP32 beyond, nb = 256 (two sub-blocks per tile):
    with the FP32 products formed by the three-way BF16 split (split = 1) and
    by the FP32 MFMA (split = 0), every FP32 tile agrees with the emulation
    (exact products, one FP32 rounding per update) to the FP32 unit roundoff
    in norm: the updates are a few percent of the entries of the dominant
    matrix, so the accumulation errors of both modes stay below one FP32
    rounding of the tile."""
    from paper_2406_02701_amd import mpcr
    gu, ctx = g
    n, nb = 4096 - 37, 256
    A = matrix(dict(n=n, rho=0.999, matrix="dominant"))
    m = tiled.tilemap_banded(n, nb, ((1, "fp64"), (None, "fp32")))
    nt = m.shape[0]
    ctx.check(mpcr.mpcr_ctx_set_fp32_split(ctx.ptr, split))
    try:
        dA = gu.dev(A)
        hm = gu.u8map(m)
        tm = mpcr.tilemap(n, nb, hm)
        f = ctypes.c_void_p()
        info = ctypes.c_int64(-1)
        ctx.check(mpcr.mpcr_potrf_tiled(ctx.ptr, n, dA.data_ptr(), n, ctypes.byref(tm), ctypes.byref(f),
                                        ctypes.byref(info)))
        dL = gu.empty(n, n)
        ctx.check(mpcr.mpcr_factor_to_dense(ctx.ptr, f, dL.data_ptr(), n))
        torch.cuda.synchronize()
        L = gu.host(dL, (n, n))
        mpcr.mpcr_factor_destroy(f)
    finally:
        ctx.check(mpcr.mpcr_ctx_set_fp32_split(ctx.ptr, 1))
    E = tiled.tile_cholesky_emulated(A, nb, m)["L"][:n, :n]
    u32 = ff.fmt_of(ff.CODE["fp32"]).unit_roundoff
    worst = 0.0
    for i in range(nt):
        for j in range(i + 1):
            sl = (slice(i * nb, min((i + 1) * nb, n)), slice(j * nb, min((j + 1) * nb, n)))
            t, te = L[sl], E[sl]
            assert np.array_equal(ff.round_to(t, int(m[i, j])), t), (i, j)
            rel = np.linalg.norm(t - te) / np.linalg.norm(te)
            worst = max(worst, rel)
            assert rel <= u32, (i, j, rel)
    print(f"split {split}: worst per-tile relative difference {worst:.2e} (u32 {u32:.2e})", flush=True)

