"""Pins for the emulated mixed-precision tile Cholesky (oracle/tiled.py),
PCG / IR refinement (oracle/refine.py) and the end-to-end log-likelihood
(oracle/loglik.py).

* all-FP64 map: the tile factor equals the dense column Cholesky up to
  rounding for every tile size, including ragged sizes padded with identity
  (tiling and padding invariance);
* low-precision map on a well-conditioned KMS matrix: every stored tile is a
  value of its format, and the factor stays within the format's error bound of
  the exact closed-form factor; with FP64 everywhere it equals it at FP64 level;
* breakdown of an indefinite input reports the global 1-based column;
* the algorithmic flop split matches the task counts of the right-looking tile
  DAG (NT POTRF, NT(NT-1)/2 TRSM and SYRK, C(NT,3) GEMM);
* PCG and IR reach the plain FP64 solution; the refined quadratic form equals
  z^T Sigma^{-1} z;
* the mixed log-likelihood on the exponential 1-D grid matches the KMS closed form;
* permuting the sites jointly with z leaves the log-likelihood unchanged.
"""
import math

import numpy as np
import pytest

import synth
from oracle import covariance as cov
from oracle import dense, fpformat as ff, loglik, refine, tiled
from tests.test_oracle_dense import kms, kms_loglik_closed_form


@pytest.mark.parametrize("n,nb", [(256, 256), (256, 128), (256, 64), (250, 64), (200, 48), (97, 32)])
def test_fp64_tiles_equal_dense(n, nb):
    locs = synth.locations(n, 40)
    S = cov.covariance(locs[cov.morton_order(locs)], 1.0, 0.1, 1.5, 1e-4)
    m = tiled.tilemap_uniform(n, nb)
    out = tiled.tile_cholesky_emulated(S, nb, m)
    assert out["info"] == 0
    L = out["L"]
    Ld = dense.cholesky_lower(S)
    np.testing.assert_allclose(L[:n, :n], Ld, rtol=0, atol=64 * n * 2.0 ** -53 * np.abs(Ld).max())
    N = out["N"]
    assert np.array_equal(L[n:, n:], np.eye(N - n)) and not np.any(L[n:, :n])


def test_low_precision_tiles_hold_format_values_and_bound():
    n, nb, rho = 512, 64, 0.5
    A = kms(n, rho)
    m = tiled.tilemap_banded(n, nb, ((1, "fp64"), (3, "fp32"), (4, "fp16"), (5, "fp8_e4m3"), (None, "bf16")))
    out = tiled.tile_cholesky_emulated(A, nb, m)
    assert out["info"] == 0
    L = out["L"]
    nt = n // nb
    for i in range(nt):
        for j in range(i):
            t = L[i * nb:(i + 1) * nb, j * nb:(j + 1) * nb]
            assert np.array_equal(tiled.round_tile(t, int(m[i, j])), t)
    i = np.arange(n)
    ref = np.where(i[:, None] >= i[None, :], rho ** (i[:, None] - i[None, :]) * math.sqrt(1 - rho ** 2), 0.0)
    ref[:, 0] = rho ** i
    err = np.linalg.norm(L - ref) / np.linalg.norm(ref)
    assert err <= 8 * ff.BF16.unit_roundoff * math.sqrt(nt)
    assert err > 0  # the rounding really happened
    m64 = tiled.tilemap_uniform(n, nb)
    e64 = np.linalg.norm(tiled.tile_cholesky_emulated(A, nb, m64)["L"] - ref) / np.linalg.norm(ref)
    assert e64 <= 1e-14


def test_breakdown_reports_global_column():
    A = kms(128, 0.5)
    A[70, 70] = 0.2
    m = tiled.tilemap_uniform(128, 32)
    out = tiled.tile_cholesky_emulated(A, 32, m)
    assert out["info"] == 71


def test_flop_split_matches_task_counts():
    nt, nb = 64, 512
    m = tiled.tilemap_banded(nt * nb, nb, ((2, "fp64"), (8, "fp32"), (None, "bf16")))
    f = tiled.flops_by_format(nt, nb, m)
    n_potrf, n_trsm, n_syrk, n_gemm = nt, nt * (nt - 1) // 2, nt * (nt - 1) // 2, math.comb(nt, 3)
    assert (n_potrf, n_trsm, n_gemm) == (64, 2016, 41664)
    total = n_potrf * nb ** 3 / 3 + (n_trsm + n_syrk) * nb ** 3 + n_gemm * 2 * nb ** 3
    assert abs(sum(f.values()) - total) <= 1e-9 * total
    # GEMM tasks at tile distance d = i - j: (NT-1-d)(NT-d)/2 of them (j >= 1)
    per_d = {d: (nt - 1 - d) * (nt - d) // 2 for d in range(1, nt)}
    assert sum(per_d.values()) == n_gemm
    g = 2.0 * nb ** 3
    fp64 = n_potrf * nb ** 3 / 3 + (n_trsm + n_syrk) * nb ** 3 + g * sum(per_d[d] for d in (1, 2))
    fp32 = g * sum(per_d[d] for d in range(3, 9))
    bf16 = g * sum(per_d[d] for d in range(9, nt))
    assert f[0] == pytest.approx(fp64, rel=1e-12)
    assert f[1] == pytest.approx(fp32, rel=1e-12)
    assert f[3] == pytest.approx(bf16, rel=1e-12)


def _matern_case(n, seed, a=0.1, nu=1.5, tau=1e-6):
    locs = synth.locations(n, seed)
    locs = locs[cov.morton_order(locs)]
    return locs, cov.covariance(locs, 1.0, a, nu, tau)


@pytest.mark.parametrize("solver", ["pcg", "ir", "gmres", "bpcg"])
def test_refinement_reaches_fp64_solution(solver):
    n, nb = 384, 64
    locs, S = _matern_case(n, 41, a=0.05, nu=0.5, tau=1e-4)
    m = tiled.tilemap_banded(n, nb, ((1, "fp64"), (None, "fp32")))
    L = tiled.tile_cholesky_emulated(S, nb, m)["L"][:n, :n]
    B = synth.normal_rhs(n, 3, 42)
    sig_inf = np.max(np.sum(np.abs(S), axis=1))
    pre = lambda R: dense.cholesky_solve(L, R)
    run = {"pcg": refine.pcg, "ir": refine.iterative_refinement, "gmres": refine.gmres_ir,
           "bpcg": refine.block_pcg}[solver]
    out = run(lambda X: S @ X, B, pre, sig_inf, tol=1e-14, max_iter=50)
    assert out["converged"] and out["eta"] <= 1e-14
    Xd = dense.cholesky_solve(dense.cholesky_lower(S), B)
    np.testing.assert_allclose(out["X"], Xd, rtol=1e-8, atol=1e-10 * np.abs(Xd).max())
    q = refine.quad_refined(B, out["X"], out["R"])
    np.testing.assert_allclose(q, np.sum(B * Xd, axis=0), rtol=1e-11)


def test_pcg_exact_preconditioner_needs_no_iteration():
    n = 128
    locs, S = _matern_case(n, 43)
    L = dense.cholesky_lower(S)
    B = synth.normal_rhs(n, 2, 44)
    out = refine.pcg(lambda X: S @ X, B, lambda R: dense.cholesky_solve(L, R),
                     np.max(np.sum(np.abs(S), axis=1)), tol=1e-12)
    assert out["iters"] == 0 and out["converged"]


def test_mixed_loglik_kms_closed_form():
    n, nb, h, a = 512, 64, 0.01, 0.03
    locs = synth.grid_1d(n, h)
    z = synth.normal_rhs(n, 2, 45)
    m = tiled.tilemap_banded(n, nb, ((1, "fp64"), (None, "fp32")))
    out = loglik.loglik_mixed(locs, z, 1.0, a, 0.5, 0.0, nb, m, tol=1e-13)
    assert out["info"] == 0 and out["converged"]
    rho = math.exp(-h / a)
    for c in range(2):
        logdet, q, ll = kms_loglik_closed_form(z[:, c], 1.0, rho)
        assert abs(out["quad"][c] - q) <= 1e-9 * abs(q)
        assert abs(out["logdet"] - logdet) <= 1e-5 * abs(logdet)   # FP32 tiles: logdet is not refined
        assert abs(out["loglik"][c] - ll) <= 1e-5 * abs(ll)


def test_loglik_permutation_invariance():
    n = 300
    locs = synth.locations(n, 46)
    z = synth.normal_rhs(n, 1, 47)
    a = loglik.loglik_plain(locs, z, 1.2, 0.1, 2.5, 1e-4)
    lo, zo, _ = loglik.order_sites(locs, z)
    b = loglik.loglik_plain(lo, zo, 1.2, 0.1, 2.5, 1e-4)
    assert abs(a["loglik"][0] - b["loglik"][0]) <= 1e-10 * abs(a["loglik"][0])
    m = tiled.tilemap_uniform(n, 64)
    c = loglik.loglik_mixed(lo, zo, 1.2, 0.1, 2.5, 1e-4, 64, m, tol=1e-14)
    assert abs(c["loglik"][0] - a["loglik"][0]) <= 1e-10 * abs(a["loglik"][0])


def test_three_tile_step_by_hand():
    """One explicit run of the tile steps on a 3 x 3 tile matrix (nb = 8) with a
    map in which the GEMM of tile (2, 1) must narrow an FP64 operand to BF16."""
    g = np.random.default_rng(60)
    M = g.standard_normal((24, 24))
    A = M @ M.T + 24 * np.eye(24)
    m = np.full((3, 3), 255, np.uint8)
    m[0, 0] = m[1, 1] = m[2, 2] = 0
    m[1, 0] = 0            # fp64
    m[2, 0] = 1            # fp32
    m[2, 1] = 3            # bf16
    out = tiled.tile_cholesky_emulated(A, 8, m)["L"]
    R = lambda x, f: ff.round_to(x, f)
    t = lambda X, i, j: X[8 * i:8 * i + 8, 8 * j:8 * j + 8]
    W = A.copy()
    for (i, j, f) in [(1, 0, "fp64"), (2, 0, "fp32"), (2, 1, "bf16")]:
        W[8 * i:8 * i + 8, 8 * j:8 * j + 8] = R(t(W, i, j), f)
    L00 = np.linalg.cholesky(t(W, 0, 0))
    L10 = R(np.linalg.solve(L00, t(W, 1, 0).T).T, "fp64")
    L20 = R(np.linalg.solve(L00, t(W, 2, 0).T).T, "fp32")
    A11 = t(W, 1, 1) - L10 @ L10.T
    A22 = t(W, 2, 2) - L20 @ L20.T
    A21 = R(t(W, 2, 1) - R(L20, "bf16") @ R(L10, "bf16").T, "bf16")
    L11 = np.linalg.cholesky(A11)
    L21 = R(np.linalg.solve(L11, A21.T).T, "bf16")
    L22 = np.linalg.cholesky(A22 - L21 @ L21.T)
    for (i, j, ref) in [(0, 0, L00), (1, 0, L10), (2, 0, L20), (1, 1, L11), (2, 1, L21), (2, 2, L22)]:
        np.testing.assert_allclose(t(out, i, j), ref, rtol=1e-13, atol=1e-14)
    # the narrowing of L10 matters here: without it the result is different
    A21_wrong = R(t(W, 2, 1) - R(L20, "bf16") @ L10.T, "bf16")
    assert not np.array_equal(A21_wrong, A21)


def test_fp8_tile_rounding_scale_and_grid():
    """An FP8 tile is held as E4M3 codes times 2^-s with s the largest integer
    such that max|X| 2^s <= 448 (found here by a plain search), every stored
    value lies on the E4M3 grid after scaling, and values in E4M3's normal range
    round with relative error <= 2^-4."""
    g = np.random.default_rng(70)
    for scale in (1e-30, 3e-7, 1.0, 5e3):
        X = g.standard_normal((32, 32)) * scale
        amax = np.max(np.abs(X))
        s = -200
        while amax * 2.0 ** (s + 1) <= 448:
            s += 1
        assert tiled.tile_scale_exponent(X) == s
        R = tiled.round_tile(X, ff.CODE["fp8_e4m3"])
        Y = np.ldexp(R, s)
        assert np.all(np.abs(Y) <= 448)
        assert np.array_equal(ff.round_to(Y, ff.FP8_E4M3), Y)
        normal = np.abs(np.ldexp(X, s)) >= 2.0 ** -6
        assert np.all(np.abs(R - X)[normal] <= 2.0 ** -4 * np.abs(X)[normal])
    assert tiled.tile_scale_exponent(np.zeros((4, 4))) == 0


def test_three_tile_step_by_hand_fp8():
    """The hand computation of the 3 x 3 tile case with tile (2, 1) in FP8: the
    FP8 roundings are done with the GEMM oracle's block quantiser (one block
    per tile), an independent implementation of the per-tile scale."""
    from oracle import gemm as og
    g = np.random.default_rng(61)
    M = g.standard_normal((24, 24))
    A = M @ M.T + 24 * np.eye(24)
    m = np.full((3, 3), 255, np.uint8)
    m[0, 0] = m[1, 1] = m[2, 2] = 0
    m[1, 0] = 1            # fp32
    m[2, 0] = 0            # fp64
    m[2, 1] = 4            # fp8
    out = tiled.tile_cholesky_emulated(A, 8, m)["L"]

    def R(x, f):
        if f == "fp8":
            Q, S = og.fp8_block_quantize(x, block=8)
            return og.fp8_block_dequantize(Q, S, block=8)
        return ff.round_to(x, f)
    t = lambda X, i, j: X[8 * i:8 * i + 8, 8 * j:8 * j + 8]
    W = A.copy()
    for (i, j, f) in [(1, 0, "fp32"), (2, 0, "fp64"), (2, 1, "fp8")]:
        W[8 * i:8 * i + 8, 8 * j:8 * j + 8] = R(t(W, i, j), f)
    L00 = np.linalg.cholesky(t(W, 0, 0))
    L10 = R(np.linalg.solve(L00, t(W, 1, 0).T).T, "fp32")
    L20 = np.linalg.solve(L00, t(W, 2, 0).T).T
    A11 = t(W, 1, 1) - L10 @ L10.T
    A22 = t(W, 2, 2) - L20 @ L20.T
    A21 = R(t(W, 2, 1) - R(L20, "fp8") @ R(L10, "fp8").T, "fp8")
    L11 = np.linalg.cholesky(A11)
    L21 = R(np.linalg.solve(L11, A21.T).T, "fp8")
    L22 = np.linalg.cholesky(A22 - L21 @ L21.T)
    for (i, j, ref) in [(0, 0, L00), (1, 0, L10), (2, 0, L20), (1, 1, L11), (2, 1, L21), (2, 2, L22)]:
        np.testing.assert_allclose(t(out, i, j), ref, rtol=1e-13, atol=1e-14)


# ---------------------------------------------------------------------------
# norm-guarded map and promotion after a breakdown
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("fmt", ["fp32", "fp16", "bf16", "fp8_e4m3"])
@pytest.mark.parametrize("amax", [0.7, 3e-5, 2e-8])
def test_rounding_bound_holds_and_is_attained(fmt, amax):
    """rounding_bound(p, amax) bounds |round(x) - x| for every |x| <= amax
    (an FP8 tile is rounded with its own power-of-two scale), and half of it is
    reached: a wrong unit roundoff or subnormal floor fails one of the two."""
    code = ff.CODE[fmt]
    rng = np.random.default_rng(5)
    x = amax * rng.uniform(-1, 1, 200000)
    x[0] = amax
    err = np.abs(tiled.round_tile(x, code) - x)
    b = tiled.rounding_bound(code, amax)
    assert err.max() <= b
    assert err.max() >= 0.5 * b


def test_guarded_map_hand_example():
    """3 x 3 and 2 x 2 tile examples worked out by hand with guard 1e-8."""
    F64, F32, F16, BF16, F8 = (ff.CODE[k] for k in ("fp64", "fp32", "fp16", "bf16", "fp8_e4m3"))
    U = tiled.UNUSED
    banded = np.array([[F64, U, U], [F32, F64, U], [BF16, F32, F64]], np.uint8)
    amax = np.array([[1, 0, 0], [0.5, 1, 0], [1e-9, 1e-3, 1]])
    # (1,0): 2^-24 * 0.5 = 3.0e-8 > 1e-8 -> FP64; (2,1): 2^-24 * 1e-3 = 6e-11 -> FP32;
    # (2,0): 2^-8 * 1e-9 = 3.9e-12 -> BF16
    got = tiled.tilemap_guarded(banded, amax, 1e-8)
    assert got.tolist() == [[F64, U, U], [F64, F64, U], [BF16, F32, F64]]
    # FP16 tile of magnitude 1e-7: relative 4.9e-11 but values below 2^-14 round
    # with absolute error up to 2^-25 = 3.0e-8 > 1e-8 -> FP32.
    # FP8 tile (own scale) of magnitude 1e-7: 2^-4 * 1e-7 = 6.25e-9 -> stays FP8;
    # of magnitude 1e-6: 6.25e-8 -> FP16 -> floor 3.0e-8 -> FP32.
    banded = np.array([[F64, U], [F16, F64]], np.uint8)
    assert tiled.tilemap_guarded(banded, np.array([[1, 0], [1e-7, 1]]), 1e-8)[1, 0] == F32
    banded = np.array([[F64, U], [F8, F64]], np.uint8)
    assert tiled.tilemap_guarded(banded, np.array([[1, 0], [1e-7, 1]]), 1e-8)[1, 0] == F8
    assert tiled.tilemap_guarded(banded, np.array([[1, 0], [1e-6, 1]]), 1e-8)[1, 0] == F32
    # magnitude 1e-2, guard 1e-4: FP8 6.25e-4 is too coarse, FP16 4.9e-6 is not
    assert tiled.tilemap_guarded(banded, np.array([[1, 0], [1e-2, 1]]), 1e-4)[1, 0] == F16


def test_guarded_map_is_the_first_format_meeting_the_guard():
    n, nb = 2048, 128
    locs = synth.locations(n, 4)
    S = cov.covariance(locs[cov.morton_order(locs)], 1.0, 0.05, 1.5, 1e-6)
    amax = tiled.tile_amax(S, nb)
    # tile maxima by a plain scan
    t = S[3 * nb:4 * nb, 1 * nb:2 * nb]
    assert amax[3, 1] == np.abs(t).max()
    banded = tiled.tilemap_banded(n, nb, ((1, "fp64"), (4, "fp32"), (8, "fp16"), (None, "fp8_e4m3")))
    for guard in (1e-6, 1e-8, 1e-10):
        gm = tiled.tilemap_guarded(banded, amax, guard)
        ladder = {ff.CODE["fp8_e4m3"]: ["fp8_e4m3", "fp16", "fp32", "fp64"], ff.CODE["fp16"]: ["fp16", "fp32", "fp64"],
                  ff.CODE["fp32"]: ["fp32", "fp64"], ff.CODE["fp64"]: ["fp64"]}
        for i in range(gm.shape[0]):
            for j in range(i + 1):
                ok = [f for f in ladder[int(banded[i, j])] if f == "fp64" or
                      tiled.rounding_bound(ff.CODE[f], amax[i, j]) <= guard]
                assert gm[i, j] == ff.CODE[ok[0]]


def test_promote_after_breakdown_hand_examples():
    F64, F32, F16, BF16, F8 = (ff.CODE[k] for k in ("fp64", "fp32", "fp16", "bf16", "fp8_e4m3"))
    U = tiled.UNUSED
    m = np.array([[F64, U, U, U],
                  [F32, F64, U, U],
                  [BF16, F32, F64, U],
                  [BF16, BF16, F32, F64]], np.uint8)
    # nb = 2, info = 5 -> tile step 2; leading tiles (1,0) FP32, (2,0) BF16,
    # (2,1) FP32: coarsest BF16 at distance 2 -> every BF16 tile with d >= 2
    # ((2,0), (3,0), (3,1)) becomes FP32
    got = tiled.promote_after_breakdown(m, 2, 5)
    assert got.tolist() == [[F64, U, U, U], [F32, F64, U, U], [F32, F32, F64, U], [F32, F32, F32, F64]]
    # again at the same step: now FP32 is the coarsest, first at distance 1
    got2 = tiled.promote_after_breakdown(got, 2, 5)
    assert all(got2[i, j] == F64 for i in range(4) for j in range(i + 1))
    # nothing left to promote
    assert np.array_equal(tiled.promote_after_breakdown(got2, 2, 5), got2)
    # FP8 far tiles, breakdown in step 3: only FP8 tiles at distance >= 3 move (to FP16)
    m = np.array([[F64, U, U, U],
                  [F32, F64, U, U],
                  [F16, F32, F64, U],
                  [F8, F16, F32, F64]], np.uint8)
    got = tiled.promote_after_breakdown(m, 4, 13)
    assert got[3, 0] == F16 and np.array_equal(np.delete(got.ravel(), 12), np.delete(m.ravel(), 12))
    # breakdown in step 1: the leading block holds only (1,0) FP32
    got = tiled.promote_after_breakdown(m, 4, 7)
    assert got[1, 0] == F64 and got[2, 1] == F64 and got[3, 2] == F64
    assert got[2, 0] == F16 and got[3, 0] == F8


def test_promotion_recovers_a_breakdown_and_refines_to_fp64():
    """The BF16 far band makes this Matern 3/2 covariance's stored tiles
    indefinite; promoting after the breakdown gives a factor, and the refined
    quadratic form is the FP64 one."""
    n, nb = 1024, 128
    locs = synth.locations(n, 4)
    z = synth.normal_rhs(n, 1, 5)
    lo, zo, _ = loglik.order_sites(locs, z)
    m = tiled.tilemap_banded(n, nb, ((1, "fp64"), (2, "fp32"), (None, "bf16")))
    plain = loglik.loglik_mixed(lo, zo, 1.0, 0.05, 1.5, 1e-6, nb, m, tol=1e-13)
    assert plain["info"] > 0
    out = loglik.loglik_mixed(lo, zo, 1.0, 0.05, 1.5, 1e-6, nb, m, tol=1e-13, promote=True)
    assert out["info"] == 0 and out["promotions"] >= 1 and out["converged"]
    ref = loglik.loglik_plain(lo, zo, 1.0, 0.05, 1.5, 1e-6)
    assert abs(out["quad"][0] - ref["quad"][0]) <= 1e-8 * abs(ref["quad"][0])
    used = out["map"]
    assert all(used[i, j] >= 0 for i in range(used.shape[0]) for j in range(i + 1))
