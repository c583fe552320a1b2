"""Pins for the refinement variants of the oracle (oracle/refine.py): GMRES
and GMRES-based iterative refinement, block PCG.

* GMRES after j steps is, by its definition, the minimiser of
  ||r0 - op(d)|| over the Krylov space K_j(op, r0): compared with a least-
  squares solve over an explicitly built Krylov basis, and its rotated
  residual estimates with the true residual norms;
* on an operator with three distinct eigenvalues GMRES terminates in at most
  three steps (the degree of the minimal polynomial);
* block CG on Sigma = I + U U^T with rank(U) equal to the block size s solves
  the system in two block iterations (the error A^{-1} R0 lies in
  span(R0) + span(U), which is the block Krylov space of two blocks when
  U^T R0 is invertible), where CG on single columns needs one more step than
  the s distinct eigenvalues away from 1;
* the block directions are Sigma-conjugate (P_i^T Sigma P_j = 0, i != j) and
  the residuals are M^{-1}-orthogonal (Z_i^T R_j = 0, i != j);
* with one column per block, block PCG is PCG;
* the Cholesky solve of the s x s systems reports a singular system.
The refinement variants' convergence to the FP64 solution with a mixed
factor is pinned with PCG and IR in test_oracle_tiled.py.
"""
import numpy as np
import pytest

import synth
from oracle import dense, refine


def _spd(n, seed, cond=100.0):
    g = synth.rng(seed)
    Q, _ = np.linalg.qr(g.standard_normal((n, n)))
    ev = np.geomspace(1.0, cond, n)
    return (Q * ev) @ Q.T


def _op(n, seed):
    """M^{-1} S with S and M different SPD matrices: a nonsymmetric operator."""
    S = _spd(n, seed)
    M = S + 0.3 * _spd(n, seed + 1, cond=10.0)
    Lm = dense.cholesky_lower(M)
    return lambda v: dense.cholesky_solve(Lm, (S @ v)[:, None])[:, 0]


@pytest.mark.parametrize("j", [1, 2, 3, 5, 8])
def test_gmres_minimises_over_the_krylov_space(j):
    n = 40
    op = _op(n, 11)
    r0 = synth.rng(12).standard_normal(n)
    d, k, est = refine.gmres_correction(op, r0, j, 0.0)
    assert k == j
    K = np.empty((n, j))
    K[:, 0] = r0
    for i in range(1, j):
        K[:, i] = op(K[:, i - 1])
    AK = np.column_stack([op(K[:, i]) for i in range(j)])
    y, *_ = np.linalg.lstsq(AK, r0, rcond=None)
    d_ref = K @ y
    np.testing.assert_allclose(d, d_ref, rtol=1e-7, atol=1e-9 * np.abs(d_ref).max())
    for i in range(1, j + 1):
        di, _, _ = refine.gmres_correction(op, r0, i, 0.0)
        assert abs(est[i - 1] - np.linalg.norm(r0 - op(di))) <= 1e-10 * np.linalg.norm(r0)
    assert all(est[i] <= est[i - 1] * (1 + 1e-12) for i in range(1, j))


def test_gmres_terminates_at_the_minimal_polynomial_degree():
    n = 30
    g = synth.rng(13)
    Q, _ = np.linalg.qr(g.standard_normal((n, n)))
    A = (Q * np.array([1.0, 2.0, 5.0] * 10)) @ Q.T
    r0 = g.standard_normal(n)
    d, k, est = refine.gmres_correction(lambda v: A @ v, r0, 10, 1e-13)
    assert k <= 3
    assert np.linalg.norm(r0 - A @ d) <= 1e-12 * np.linalg.norm(r0)


def test_block_cg_low_rank_two_iterations():
    n, r, s = 200, 6, 6
    g = synth.rng(14)
    U = 0.3 * g.standard_normal((n, r))
    S = np.eye(n) + U @ U.T
    B = g.standard_normal((n, s))
    sig_inf = np.max(np.sum(np.abs(S), axis=1))
    pre = lambda R: 0.5 * R                       # M = 2 I: block PCG is block CG
    out = refine.block_pcg(lambda X: S @ X, B, pre, sig_inf, tol=1e-14, max_iter=20, block=s)
    assert out["converged"] and out["iters"] == 2 and not out["fallback"]
    np.testing.assert_allclose(out["X"], np.linalg.solve(S, B), rtol=1e-12, atol=1e-13)
    single = refine.pcg(lambda X: S @ X, B, pre, sig_inf, tol=1e-14, max_iter=50)
    assert single["converged"] and single["iters"] == r + 1


def test_block_pcg_conjugacy_and_orthogonality():
    n, s, k = 60, 3, 4
    S = _spd(n, 15, cond=1e3)
    M = S + 2.0 * _spd(n, 16, cond=10.0)
    Lm = dense.cholesky_lower(M)
    B = synth.normal_rhs(n, s, 17)
    out = refine.block_pcg(lambda X: S @ X, B, lambda R: dense.cholesky_solve(Lm, R),
                           np.max(np.sum(np.abs(S), axis=1)), tol=0.0, max_iter=k, recompute=100, block=s,
                           history=True)
    h = out["history"]
    assert len(h["P"]) == k
    for i in range(k):
        for j in range(k):
            if i == j:
                continue
            Pi, Pj = h["P"][i], h["P"][j]
            c = np.abs(Pi.T @ S @ Pj).max() / (np.linalg.norm(S @ Pi) * np.linalg.norm(Pj))
            o = np.abs(h["Z"][i].T @ h["R"][j]).max() / (np.linalg.norm(h["Z"][i]) * np.linalg.norm(h["R"][j]))
            assert c <= 1e-9 and o <= 1e-9, (i, j, c, o)


def test_block_pcg_with_one_column_blocks_is_pcg():
    n = 80
    S = _spd(n, 18, cond=1e4)
    M = S + 0.5 * _spd(n, 19, cond=10.0)
    Lm = dense.cholesky_lower(M)
    B = synth.normal_rhs(n, 3, 20)
    args = (lambda X: S @ X, B, lambda R: dense.cholesky_solve(Lm, R), np.max(np.sum(np.abs(S), axis=1)))
    for k in (1, 2, 5):                         # the same iterates (rounding of the 1 x 1 solves aside)
        a = refine.block_pcg(*args, tol=0.0, max_iter=k, block=1)
        b = refine.pcg(*args, tol=0.0, max_iter=k)
        assert a["iters"] == b["iters"] == k
        np.testing.assert_allclose(a["X"], b["X"], rtol=0, atol=1e-12 * np.abs(b["X"]).max())
    a = refine.block_pcg(*args, tol=1e-14, max_iter=60, block=1)
    b = refine.pcg(*args, tol=1e-14, max_iter=60)
    assert a["converged"] and b["converged"] and a["iters"] == b["iters"]


def test_spd_solve_reports_singular_systems():
    g = synth.rng(21)
    A = g.standard_normal((5, 5))
    G = A @ A.T + 5 * np.eye(5)
    F = g.standard_normal((5, 5))
    np.testing.assert_allclose(refine._spd_solve(G, F), np.linalg.solve(G, F), rtol=1e-12)
    V = g.standard_normal((5, 3))
    assert refine._spd_solve(V @ V.T, F) is None
