"""Plain FP64 linear algebra: the definitions the FP64 path reaches exactly
(up to rounding order).

Follows the paper's section "Maximum Likelihood Estimation of Matérn Covariance
Function": the log-likelihood
    l(theta) = -(n/2) log(2 pi) - (1/2) log|Sigma| - (1/2) z^T Sigma^{-1} z
is evaluated by factoring Sigma = L L^T (the paper's R code takes
L = t(chol(V))), log|Sigma| = 2 sum_i log L_ii, w = L^{-1} z by forward
substitution and z^T Sigma^{-1} z = ||w||^2.  The GEMM is the product of the
paper's section "Linear Algebra Functions Performance" (A %*% B).
"""
from __future__ import annotations

import math

import numpy as np


class NotPositiveDefinite(Exception):
    def __init__(self, info: int):
        super().__init__(f"leading minor of order {info} is not positive definite")
        self.info = info


def cholesky_lower(A: np.ndarray) -> np.ndarray:
    """Lower Cholesky factor of a symmetric positive definite matrix by the
    textbook column (left-looking) algorithm; only the lower triangle of A is
    read.  Raises NotPositiveDefinite(info) with the 1-based column of the
    first non-positive pivot (LAPACK convention)."""
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    L = np.zeros((n, n))
    for j in range(n):
        d = A[j, j] - np.dot(L[j, :j], L[j, :j])
        if not d > 0.0:
            raise NotPositiveDefinite(j + 1)
        L[j, j] = math.sqrt(d)
        if j + 1 < n:
            L[j + 1:, j] = (A[j + 1:, j] - L[j + 1:, :j] @ L[j, :j]) / L[j, j]
    return L


def forward_substitution(L: np.ndarray, B: np.ndarray) -> np.ndarray:
    """Solve L W = B for lower-triangular L (column-oriented substitution)."""
    W = np.array(B, dtype=np.float64, copy=True)
    vec = W.ndim == 1
    if vec:
        W = W[:, None]
    n = L.shape[0]
    for j in range(n):
        W[j, :] = W[j, :] / L[j, j]
        if j + 1 < n:
            W[j + 1:, :] -= np.outer(L[j + 1:, j], W[j, :])
    return W[:, 0] if vec else W


def backward_substitution_transpose(L: np.ndarray, W: np.ndarray) -> np.ndarray:
    """Solve L^T X = W for lower-triangular L (row-oriented on L^T)."""
    X = np.array(W, dtype=np.float64, copy=True)
    vec = X.ndim == 1
    if vec:
        X = X[:, None]
    n = L.shape[0]
    for j in range(n - 1, -1, -1):
        if j + 1 < n:
            X[j, :] -= L[j + 1:, j] @ X[j + 1:, :]
        X[j, :] = X[j, :] / L[j, j]
    return X[:, 0] if vec else X


def cholesky_solve(L: np.ndarray, B: np.ndarray) -> np.ndarray:
    """x = Sigma^{-1} B with Sigma = L L^T: forward then backward substitution."""
    return backward_substitution_transpose(L, forward_substitution(L, B))


def neumaier_sum(values) -> float:
    """Compensated (Neumaier) summation in float64, sequential order."""
    s = 0.0
    c = 0.0
    for v in np.asarray(values, dtype=np.float64).ravel():
        v = float(v)
        t = s + v
        if abs(s) >= abs(v):
            c += (s - t) + v
        else:
            c += (v - t) + s
        s = t
    return s + c


def logdet_from_cholesky(L: np.ndarray) -> float:
    """log|Sigma| = 2 sum_i log L_ii."""
    return 2.0 * neumaier_sum(np.log(np.diag(L)))


def gaussian_loglik(n: int, logdet: float, quad) -> np.ndarray:
    """l = -(n/2) log(2 pi) - logdet/2 - quad/2 (quad may be one value per
    observation vector)."""
    return -0.5 * n * math.log(2.0 * math.pi) - 0.5 * logdet - 0.5 * np.asarray(quad, dtype=np.float64)


def loglik_fp64(Sigma: np.ndarray, Z: np.ndarray):
    """Plain FP64 evaluation: returns dict(logdet, quad, loglik, L, W, X).
    quad_c = ||w_c||^2 for each column c of Z."""
    Z2 = Z[:, None] if Z.ndim == 1 else Z
    L = cholesky_lower(Sigma)
    W = forward_substitution(L, Z2)
    X = backward_substitution_transpose(L, W)
    logdet = logdet_from_cholesky(L)
    quad = np.array([neumaier_sum(W[:, c] * W[:, c]) for c in range(W.shape[1])])
    return dict(logdet=logdet, quad=quad, loglik=gaussian_loglik(Sigma.shape[0], logdet, quad),
                L=L, W=W, X=X)


def gemm(A: np.ndarray, B: np.ndarray, transA=False, transB=False, alpha=1.0, beta=0.0, C=None):
    """C <- alpha op(A) op(B) + beta C in float64."""
    opA = A.T if transA else A
    opB = B.T if transB else B
    P = np.matmul(np.asarray(opA, np.float64), np.asarray(opB, np.float64))
    out = alpha * P
    if C is not None and beta != 0.0:
        out = out + beta * np.asarray(C, np.float64)
    return out
