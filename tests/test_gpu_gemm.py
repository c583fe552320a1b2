"""GPU parity of mpcr_gemm against the GEMM emulation oracle.

* Small ragged shapes (several 128-blocks and a tail), every format, with
  transposes, alpha and beta: rel-F(C_gpu, C_emu) <= 4 sqrt(k) u_acc with
  u_acc the accumulation's unit roundoff: 2^-53 for FP64, 2^-24 for FP32 and
  the 16-bit formats, and 2^-16 for FP8, whose gfx950 MFMA sums each group of
  32 products with a narrower internal adder than FP32 (measured on
  integer-free E4M3 inputs with the lane-layout probe: about 2^-16 relative).
* Integer entries in [-4, 4] with k = 8192: every partial sum is an exact
  integer in FP32, so every format must equal the FP64 product exactly.
* Full size (m = n = k = 8192, U(-1,1)): a sample of 48 output entries is
  recomputed one by one from the rounded operands in FP64.
"""
import ctypes
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import synth  # noqa: E402
from oracle import fpformat as ff  # noqa: E402
from oracle import gemm as og  # noqa: E402

FMTS = ["fp64", "fp32", "fp16", "bf16", "fp8_e4m3"]


@pytest.fixture(scope="module")
def g():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from tests import gpu_util
    ctx = gpu_util.Ctx()
    yield gpu_util, ctx
    ctx.close()


def u_acc(fmt):
    return {"fp64": 2.0 ** -53, "fp8_e4m3": 2.0 ** -16}.get(fmt, 2.0 ** -24)


def _tdtype(fmt):
    return {"fp64": torch.float64, "fp32": torch.float32, "fp16": torch.int16, "bf16": torch.int16,
            "fp8_e4m3": torch.uint8}[fmt]


def convert(gu, ctx, X, fmt):
    """Device copy of X in format fmt (and its FP8 block exponents)."""
    from paper_2406_02701_amd import mpcr
    m, n = X.shape
    dX = gu.dev(np.asfortranarray(X))
    dY = gu.empty(m, n, _tdtype(fmt))
    sc = None
    if fmt == "fp8_e4m3":
        sc = torch.zeros(((n + 127) // 128, (m + 127) // 128), dtype=torch.int8, device="cuda")
    ctx.check(mpcr.mpcr_convert(ctx.ptr, mpcr.PREC[fmt], m, n, dX.data_ptr(), m, dY.data_ptr(), m,
                                None if sc is None else sc.data_ptr()))
    torch.cuda.synchronize()
    return dY, sc


def run_gemm(gu, ctx, fmt, A, B, tA, tB, alpha=1.0, beta=0.0, C0=None, cfmt=None):
    from paper_2406_02701_amd import mpcr
    cfmt = cfmt or ("fp64" if fmt == "fp64" else "fp32")
    m = A.shape[1] if tA else A.shape[0]
    k = A.shape[0] if tA else A.shape[1]
    n = B.shape[0] if tB else B.shape[1]
    dA, sA = convert(gu, ctx, A, fmt)
    dB, sB = convert(gu, ctx, B, fmt)
    cdt = torch.float64 if cfmt == "fp64" else torch.float32
    dC = gu.empty(m, n, cdt) if C0 is None else gu.dev(np.asfortranarray(C0), np.float64 if cfmt == "fp64" else np.float32)
    ctx.check(mpcr.mpcr_gemm(ctx.ptr, mpcr.PREC[fmt], int(tA), int(tB), m, n, k, alpha, dA.data_ptr(), A.shape[0],
                             None if sA is None else sA.data_ptr(), dB.data_ptr(), B.shape[0],
                             None if sB is None else sB.data_ptr(), beta, dC.data_ptr(), m, mpcr.PREC[cfmt]))
    return gu.host(dC, (m, n)).astype(np.float64)


@pytest.mark.parametrize("fmt", FMTS)
@pytest.mark.parametrize("tA,tB", [(False, False), (True, False), (False, True), (True, True)])
def test_gemm_matches_emulation(g, fmt, tA, tB):
    gu, ctx = g
    m, n, k = 300, 200, 260
    A = synth.uniform_matrix(k if tA else m, m if tA else k, 100)
    B = synth.uniform_matrix(n if tB else k, k if tB else n, 101)
    C0 = synth.uniform_matrix(m, n, 102)
    cf = "fp64" if fmt == "fp64" else "fp32"
    C0r = ff.round_to(C0, cf)
    got = run_gemm(gu, ctx, fmt, A, B, tA, tB, alpha=0.75, beta=-0.5, C0=C0r)
    ref = og.gemm_emulated(A, B, fmt, transA=tA, transB=tB, alpha=0.75, beta=-0.5, C=C0r, c_fmt=cf)
    err = og.rel_frobenius(got, ref)
    assert err <= 4 * math.sqrt(k) * u_acc(fmt), err


@pytest.mark.parametrize("fmt", FMTS)
def test_gemm_integer_inputs_exact(g, fmt):
    gu, ctx = g
    A = synth.integer_matrix(256, 8192, 103)
    B = synth.integer_matrix(8192, 192, 104)
    got = run_gemm(gu, ctx, fmt, A, B, False, False)
    assert np.array_equal(got, A @ B)


def test_gemm_fp8_wide_dynamic_range(g):
    gu, ctx = g
    A = synth.uniform_matrix(256, 384, 105) * np.logspace(-6, 3, 384)[None, :]
    B = synth.uniform_matrix(384, 256, 106) * np.logspace(2, -4, 384)[:, None]
    got = run_gemm(gu, ctx, "fp8_e4m3", A, B, False, False)
    ref = og.gemm_emulated(A, B, "fp8_e4m3", c_fmt="fp32")
    assert og.rel_frobenius(got, ref) <= 4 * math.sqrt(384) * u_acc("fp8_e4m3")


@pytest.mark.parametrize("fmt", FMTS)
def test_gemm_full_size_sampled(g, fmt):
    gu, ctx = g
    N = 8192
    A = synth.uniform_matrix(N, N, 3)
    B = synth.uniform_matrix(N, N, 3 + 1000)
    got = run_gemm(gu, ctx, fmt, A, B, False, False)
    Ar = og.input_rounded(A, fmt)
    Br = og.input_rounded(B, fmt)
    rng = np.random.default_rng(7)
    rows, cols = rng.integers(0, N, 48), rng.integers(0, N, 48)
    ref = np.array([np.dot(Ar[i, :], Br[:, j]) for i, j in zip(rows, cols)])
    scale = np.sqrt(N) / 3.0   # typical |C_ij| for U(-1,1) entries
    err = np.max(np.abs(got[rows, cols] - ref))
    assert err <= 4 * N * u_acc(fmt) * scale, err
    assert got.shape == (N, N) and np.all(np.isfinite(got))


@pytest.mark.parametrize("fmt", ["fp16", "bf16", "fp8_e4m3"])
def test_gemm_k_contiguous_operands_read_in_place(g, fmt):
    """op(A) = A^T and B untransposed with 16-byte aligned leading dimensions
    larger than the rows (k = 376, ld = 384): the 16/8-bit kernel reads both
    operands in place, including the ragged last k chunk."""
    from paper_2406_02701_amd import mpcr
    gu, ctx = g
    m, n, k, ld = 300, 200, 376, 384
    A = np.zeros((ld, m))
    A[:k] = synth.uniform_matrix(k, m, 107)     # stored k x m, op(A) = A^T
    B = np.zeros((ld, n))
    B[:k] = synth.uniform_matrix(k, n, 108)
    dA, sA = convert(gu, ctx, A, fmt)
    dB, sB = convert(gu, ctx, B, fmt)
    dC = gu.empty(m, n, torch.float32)
    ctx.check(mpcr.mpcr_gemm(ctx.ptr, mpcr.PREC[fmt], 1, 0, m, n, k, 1.0, dA.data_ptr(), ld,
                             None if sA is None else sA.data_ptr(), dB.data_ptr(), ld,
                             None if sB is None else sB.data_ptr(), 0.0, dC.data_ptr(), m, mpcr.PREC["fp32"]))
    got = gu.host(dC, (m, n)).astype(np.float64)
    ref = og.gemm_emulated(A[:k], B[:k], fmt, transA=True, c_fmt="fp32")
    assert og.rel_frobenius(got, ref) <= 4 * math.sqrt(k) * u_acc(fmt)
