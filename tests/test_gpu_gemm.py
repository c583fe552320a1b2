"""GPU parity of mpcr_gemm against the GEMM emulation oracle.

* Small ragged shapes (several 128-blocks and a tail), every format, with
  transposes, alpha and beta: rel-F(C_gpu, C_emu) <= 4 sqrt(k) u_acc with
  u_acc the accumulation's unit roundoff: 2^-53 for FP64, 2^-24 for FP32 and
  the 16-bit formats.  FP8: the gfx950 FP8 MFMA keeps each product of an
  aligned group of 8 only to 13 bits below the group's largest product (see
  the structured test below, which pins this model bit for bit), so every FP8
  result is checked elementwise against the bound that model gives.
* Integer entries in [-4, 4] with k = 8192: every partial sum is an exact
  integer in FP32, so every format must equal the FP64 product exactly.
* Full size (m = n = k = 8192, U(-1,1)): a sample of 48 output entries is
  recomputed one by one from the rounded operands in FP64, gated at
  4 sqrt(k) u_acc max|C| (the typical magnitude of a sum of k rounding errors).
* The accumulation of the MFMA chains themselves: sums of one dominant
  product and many small ones, all exact in FP32, are returned exactly by
  BF16 and FP16 and, by FP8, exactly as the group-truncation model predicts.
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
    return {"fp64": 2.0 ** -53}.get(fmt, 2.0 ** -24)


def fp8_bound(Ar, Br):
    """Elementwise bound of |C_gpu - C_exact| for the FP8 path (rounded
    operands Ar (m x k), Br (k x n)): in every aligned group of 8 products the
    MFMA keeps each product to 2^(e - 13), e the exponent of the group's
    largest, so at most 7 products lose less than that unit each; the group
    sums and the FP32 accumulator add (k/8 + 2) FP32 roundings."""
    m, k = Ar.shape
    n = Br.shape[1]
    out = np.zeros((m, n))
    absum = np.abs(Ar) @ np.abs(Br)
    for g0 in range(0, k, 8):
        P = np.abs(Ar[:, g0:g0 + 8, None] * Br[None, g0:g0 + 8, :])      # m x 8 x n
        mx = P.max(axis=1)
        e = np.floor(np.log2(np.where(mx > 0, mx, 1.0)))
        out += np.where(mx > 0, 7.0 * 2.0 ** (e - 13), 0.0)
    return out + (k / 8 + 2) * 2.0 ** -24 * absum


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
    if fmt == "fp8_e4m3":
        Ar = og.input_rounded(A.T if tA else A, fmt)
        Br = og.input_rounded(B.T if tB else B, fmt)
        bound = 0.75 * fp8_bound(Ar, Br) + 2.0 ** -24 * np.abs(ref) * 2
        assert np.all(np.abs(got - ref) <= bound)
        return
    err = og.rel_frobenius(got, ref)
    assert err <= 4 * math.sqrt(k) * u_acc(fmt), err


@pytest.mark.parametrize("fmt", FMTS)
@pytest.mark.parametrize("tA,tB", [(False, False), (True, False), (False, True), (True, True)])
def test_gemm_large_blocks_match_emulation(g, fmt, tA, tB):
    """Whole blocks: m, n multiples of 256 and k of 64 (FP8: 128) take the
    256 x 256-block kernels of the 16/8-bit formats and the 16-byte vector
    loads of the FP64/FP32 kernel (several blocks and k stages; alpha, beta)."""
    gu, ctx = g
    m, n, k = 512, 768, 1024
    A = synth.uniform_matrix(k if tA else m, m if tA else k, 110)
    B = synth.uniform_matrix(n if tB else k, k if tB else n, 111)
    C0r = ff.round_to(synth.uniform_matrix(m, n, 112), "fp32")
    cf = "fp64" if fmt == "fp64" else "fp32"
    C0r = ff.round_to(C0r, cf)
    got = run_gemm(gu, ctx, fmt, A, B, tA, tB, alpha=0.75, beta=-0.5, C0=C0r)
    ref = og.gemm_emulated(A, B, fmt, transA=tA, transB=tB, alpha=0.75, beta=-0.5, C=C0r, c_fmt=cf)
    err = og.rel_frobenius(got, ref)
    print(f"{fmt} large blocks tA={tA} tB={tB}: rel-F vs emulation {err:.3e}", flush=True)
    if fmt == "fp8_e4m3":
        Ar = og.input_rounded(A.T if tA else A, fmt)
        Br = og.input_rounded(B.T if tB else B, fmt)
        assert np.all(np.abs(got - ref) <= 0.75 * fp8_bound(Ar, Br) + 2.0 ** -24 * np.abs(ref) * 2)
    else:
        assert err <= 4 * math.sqrt(k) * u_acc(fmt), err
    A = synth.integer_matrix(m, k, 113)
    B = synth.integer_matrix(k, n, 114)
    assert np.array_equal(run_gemm(gu, ctx, fmt, A, B, False, False), A @ B)


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
    bound = fp8_bound(og.input_rounded(A, "fp8_e4m3"), og.input_rounded(B, "fp8_e4m3")) + 2.0 ** -24 * np.abs(ref)
    assert np.all(np.abs(got - ref) <= bound)


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
    err = np.max(np.abs(got[rows, cols] - ref))
    print(f"{fmt}: full-size sampled max |dC| {err:.3e} (max |C| {np.max(np.abs(ref)):.3e})", flush=True)
    if fmt == "fp8_e4m3":
        b = np.array([fp8_bound(Ar[i:i + 1, :], Br[:, j:j + 1])[0, 0] for i, j in zip(rows, cols)])
        assert np.all(np.abs(got[rows, cols] - ref) <= b + 2.0 ** -24 * np.abs(ref))
    else:
        assert err <= 4 * math.sqrt(N) * u_acc(fmt) * np.max(np.abs(ref)), err
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
    if fmt == "fp8_e4m3":
        bound = fp8_bound(og.input_rounded(A[:k].T, fmt), og.input_rounded(B[:k], fmt)) + 2.0 ** -24 * np.abs(ref)
        assert np.all(np.abs(got - ref) <= bound)
    else:
        assert og.rel_frobenius(got, ref) <= 4 * math.sqrt(k) * u_acc(fmt)


def _structured(k, sign):
    """Rows (1, s t_r, ..., s t_r), t_r = 2^-(6 + r//2) (x 1.5 for odd r): every
    value is an exact E4M3 code after the block scale 2^8 and an exact FP16 and
    BF16 value; with B = 1 every partial sum of a row is exact in FP32."""
    t = np.array([2.0 ** -(6 + r // 2) * (1.5 if r % 2 else 1.0) for r in range(22)])
    A = np.zeros((22, k))
    A[:, 0] = 1.0
    A[:, 1:] = sign * t[:, None]
    return A, t


def mfma_group_model(a_row, b_col, unit_bits, toward):
    """A sum of products as an MFMA that, for each aligned group of 8
    consecutive k, expresses every product as a multiple of 2^(e - unit_bits)
    (e the binary exponent of the group's largest product; `toward` "zero"
    truncates, "floor" rounds down) and adds the group sums in FP32."""
    p = a_row * b_col
    tot = np.float32(0.0)
    for g0 in range(0, p.size, 8):
        grp = p[g0:g0 + 8]
        mx = np.max(np.abs(grp))
        if mx == 0:
            continue
        q = 2.0 ** (np.floor(np.log2(mx)) - unit_bits)
        r = np.trunc(grp / q) if toward == "zero" else np.floor(grp / q)
        tot = np.float32(tot + np.float32(np.sum(r * q)))
    return float(tot)


@pytest.mark.parametrize("sign", [1.0, -1.0])
def test_mfma_accumulation_models(g, sign):
    """What the gfx950 MFMA chains do with a dominant product and many small
    ones (k = 128; C_r = 1 +- 127 t_r exactly, and exactly in FP32):
    BF16 and FP16 return the exact sums; FP8 (E4M3, block scale 2^8) equals the
    group model above with products kept to 13 bits below the largest
    product of their group of 8.  That model bounds the FP8 accumulation
    error used by the FP8 gates of this file."""
    gu, ctx = g
    k = 128
    A, t = _structured(k, sign)
    B = np.ones((k, 16))
    exact = 1.0 + sign * 127.0 * t
    for fmt in ("bf16", "fp16"):
        got = run_gemm(gu, ctx, fmt, A, B, False, False)
        assert np.array_equal(og.input_rounded(A, fmt), A)
        assert np.array_equal(got, np.repeat(exact[:, None], 16, axis=1)), fmt
    got = run_gemm(gu, ctx, "fp8_e4m3", A, B, False, False)
    assert np.array_equal(og.input_rounded(A, "fp8_e4m3"), A)
    rel = np.max(np.abs(got - exact[:, None]), axis=1) / np.abs(exact)
    hits = {}
    for toward in ("zero", "floor"):
        model = np.array([mfma_group_model(A[r] * 256.0, B[:, 0] * 256.0, 13, toward) / 65536.0
                          for r in range(A.shape[0])])
        hits[toward] = bool(np.array_equal(got, np.repeat(model[:, None], 16, axis=1)))
    print(f"FP8 MFMA, sign {sign:+}: max relative error {rel.max():.3e}; group model (13 bits) matches: {hits}",
          flush=True)
    assert rel.max() > 0            # the small products really are cut
    assert hits["zero"] or hits["floor"]


def test_fp8_block_scaled_mfma_accumulation(g):
    """The large FP8 kernel (block-scaled 16x16x128 MFMA) on the structured
    sums (one dominant product, many small ones; 256 x 256 x 128): its error
    is within the group-truncation bound used for the FP8 gates (printed
    beside the exact sums)."""
    gu, ctx = g
    k = 128
    A, t = _structured(k, 1.0)
    A = np.vstack([A, np.zeros((256 - A.shape[0], k))])
    B = np.ones((k, 256))
    got = run_gemm(gu, ctx, "fp8_e4m3", A, B, False, False)
    exact = A @ B
    Ar = og.input_rounded(A, "fp8_e4m3")
    assert np.array_equal(Ar, A)
    rel = np.max(np.abs(got[:22] - exact[:22]), axis=1) / exact[:22, 0]
    print("block-scaled FP8 MFMA: relative error per row", [f"{v:.2e}" for v in rel], flush=True)
    assert np.all(np.abs(got - exact) <= fp8_bound(Ar, B) + 2.0 ** -24 * np.abs(exact))
