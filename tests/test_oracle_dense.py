"""Pins for the plain FP64 oracle (oracle/dense.py).

P1  Kac-Murdock-Szego A_ij = rho^|i-j|: closed-form factor, determinant
    (1 - rho^2)^(n-1) and tridiagonal inverse.
P2  The exponential covariance of the paper's MLE section on a regular 1-D grid
    is sigma^2 KMS(exp(-h/a)), so the whole log-likelihood has an O(n) closed form.
P3  Pascal matrix C(i+j, i): factor C(i, j), determinant 1 (exact integers).
P4  Reconstruction ||L L^T - A|| / ||A|| at the rounding level.
P5  Exact rational arithmetic (fractions) on tiny inputs: determinant, solve.
P7  LAPACK (numpy.linalg.cholesky, scipy solve_triangular) as a second opinion.
"""
import math
from fractions import Fraction

import numpy as np
import pytest
from scipy.linalg import solve_triangular

import synth
from oracle import covariance as cov
from oracle import dense


def kms(n, rho):
    i = np.arange(n)
    return rho ** np.abs(i[:, None] - i[None, :])


@pytest.mark.parametrize("rho", [0.5, 0.9, 0.99])
def test_kms_factor_det_inverse(rho):
    n = 200
    A = kms(n, rho)
    L = dense.cholesky_lower(A)
    i = np.arange(n)
    ref = np.where(i[:, None] >= i[None, :], rho ** (i[:, None] - i[None, :]) * math.sqrt(1 - rho ** 2), 0.0)
    ref[:, 0] = rho ** i
    np.testing.assert_allclose(L, ref, rtol=1e-12, atol=1e-14)
    assert abs(dense.logdet_from_cholesky(L) - (n - 1) * math.log(1 - rho ** 2)) < 1e-10 * n
    Ainv = (np.diag(np.r_[1.0, np.full(n - 2, 1 + rho ** 2), 1.0])
            - rho * np.eye(n, k=1) - rho * np.eye(n, k=-1)) / (1 - rho ** 2)
    B = synth.normal_rhs(n, 3, 11)
    X = dense.cholesky_solve(L, B)
    np.testing.assert_allclose(X, Ainv @ B, rtol=1e-9, atol=1e-9 * np.abs(Ainv @ B).max())


def kms_loglik_closed_form(z, sigma2, rho):
    n = z.shape[0]
    logdet = n * math.log(sigma2) + (n - 1) * math.log(1 - rho * rho)
    q = (z[0] ** 2 + z[-1] ** 2 + (1 + rho * rho) * np.sum(z[1:-1] ** 2)
         - 2 * rho * np.sum(z[:-1] * z[1:])) / (sigma2 * (1 - rho * rho))
    return logdet, q, -0.5 * n * math.log(2 * math.pi) - 0.5 * logdet - 0.5 * q


def test_exponential_1d_grid_is_kms_and_loglik_closed_form():
    n, h, a, s2 = 400, 0.01, 0.05, 1.7
    locs = synth.grid_1d(n, h)
    S = cov.covariance(locs, s2, a, 0.5, 0.0)
    rho = math.exp(-h / a)
    np.testing.assert_allclose(S, s2 * kms(n, rho), rtol=1e-13)
    z = synth.normal_rhs(n, 2, 12)
    out = dense.loglik_fp64(S, z)
    for c in range(2):
        logdet, q, ll = kms_loglik_closed_form(z[:, c], s2, rho)
        assert abs(out["logdet"] - logdet) <= 1e-11 * abs(logdet)
        assert abs(out["quad"][c] - q) <= 1e-11 * abs(q)
        assert abs(out["loglik"][c] - ll) <= 1e-11 * abs(ll)


def test_pascal_exact():
    n = 20
    P = np.array([[math.comb(i + j, i) for j in range(n)] for i in range(n)], dtype=np.float64)
    L = dense.cholesky_lower(P)
    ref = np.array([[math.comb(i, j) for j in range(n)] for i in range(n)], dtype=np.float64)
    assert np.array_equal(L, ref)
    assert dense.logdet_from_cholesky(L) == 0.0


def test_reconstruction_backward_stable():
    locs = synth.locations(512, 13)
    S = cov.covariance(locs, 1.0, 0.1, 1.5, 1e-6)
    L = dense.cholesky_lower(S)
    err = np.linalg.norm(L @ L.T - S) / np.linalg.norm(S)
    assert err <= 512 * 2.0 ** -53
    assert np.array_equal(L, np.tril(L))


def _frac_det_and_solve(A, b):
    n = len(A)
    M = [[Fraction(float(A[i][j])) for j in range(n)] + [Fraction(float(b[i]))] for i in range(n)]
    det = Fraction(1)
    for c in range(n):
        p = next(r for r in range(c, n) if M[r][c] != 0)
        if p != c:
            M[c], M[p] = M[p], M[c]
            det = -det
        det *= M[c][c]
        for r in range(c + 1, n):
            f = M[r][c] / M[c][c]
            M[r] = [M[r][k] - f * M[c][k] for k in range(n + 1)]
    x = [Fraction(0)] * n
    for r in range(n - 1, -1, -1):
        x[r] = (M[r][n] - sum(M[r][k] * x[k] for k in range(r + 1, n))) / M[r][r]
    return det, x


@pytest.mark.parametrize("n", [1, 2, 3, 5, 6])
def test_bruteforce_rational(n):
    locs = synth.locations(n, 20 + n)
    S = cov.covariance(locs, 1.3, 0.4, 2.5, 1e-3)
    z = synth.normal_rhs(n, 1, 30 + n)[:, 0]
    det, x = _frac_det_and_solve(S, z)
    L = dense.cholesky_lower(S)
    assert abs(dense.logdet_from_cholesky(L) - math.log(det)) <= 1e-10
    xo = dense.cholesky_solve(L, z)
    np.testing.assert_allclose(xo, [float(v) for v in x], rtol=1e-8)
    quad_exact = float(sum(Fraction(float(z[i])) * x[i] for i in range(n)))
    w = dense.forward_substitution(L, z)
    assert abs(np.sum(w * w) - quad_exact) <= 1e-8 * abs(quad_exact)


def test_lapack_cross_check():
    locs = synth.locations(300, 14)
    S = cov.covariance(locs, 1.0, 0.2, 0.5, 1e-4)
    L = dense.cholesky_lower(S)
    np.testing.assert_allclose(L, np.linalg.cholesky(S), rtol=1e-10, atol=1e-13)
    B = synth.normal_rhs(300, 4, 15)
    W = dense.forward_substitution(L, B)
    np.testing.assert_allclose(W, solve_triangular(L, B, lower=True), rtol=1e-9, atol=1e-11)
    X = dense.backward_substitution_transpose(L, W)
    np.testing.assert_allclose(X, solve_triangular(L.T, W, lower=False), rtol=1e-9, atol=1e-11)


def test_not_positive_definite_info():
    A = kms(10, 0.5)
    A[6, 6] = 0.1            # leading minor of order 7 fails
    with pytest.raises(dense.NotPositiveDefinite) as e:
        dense.cholesky_lower(A)
    assert e.value.info == 7


def test_neumaier_sum_and_loglik_formula():
    assert dense.neumaier_sum([1.0, 1e100, 1.0, -1e100]) == 2.0
    ll = dense.gaussian_loglik(10, 2.0, 3.0)
    assert ll == -5 * math.log(2 * math.pi) - 1.0 - 1.5


def test_gemm_definition():
    A = synth.uniform_matrix(7, 5, 16)
    B = synth.uniform_matrix(7, 4, 17)
    C = synth.uniform_matrix(5, 4, 18)
    out = dense.gemm(A, B, transA=True, alpha=2.0, beta=-0.5, C=C)
    ref = np.array([[2.0 * sum(A[k, i] * B[k, j] for k in range(7)) - 0.5 * C[i, j] for j in range(4)] for i in range(5)])
    np.testing.assert_allclose(out, ref, rtol=1e-14)
