"""Iterative refinement of Sigma x = b with the mixed-precision factor as
preconditioner (oracle side).

The paper's introduction defines multi-precision algorithms as ones that use
different precisions in different stages, for example running most iterations
in a low precision and switching to double precision for refinement.  Reading
used here: the low-precision tile factor L~ gives the preconditioner
M = L~ L~^T, applied by a forward and a backward substitution in FP64; the
residual r = b - Sigma x, the iterate and all vectors are FP64.

* PCG (default): conjugate gradients on Sigma x = b preconditioned by M, the
  true residual recomputed every ``recompute`` iterations.
* IR: classical refinement x <- x + M^{-1}(b - Sigma x).

Stopping rule: the normwise backward error
    eta = ||b - Sigma x||_inf / (||Sigma||_inf ||x||_inf + ||b||_inf)
of every column is <= tol, with eta taken from the true residual.  Columns are
independent: a column that has converged is frozen.

Quadratic form for the mixed path: with x ~ Sigma^{-1} z and r = z - Sigma x,
z^T Sigma^{-1} z = z^T x + x^T r up to a term of second order in r.
"""
from __future__ import annotations

import numpy as np


def _eta(R, X, B, sig_inf):
    return np.max(np.abs(R), axis=0) / (sig_inf * np.max(np.abs(X), axis=0) + np.max(np.abs(B), axis=0))


def pcg(matvec, B, precond, sig_inf, tol=1e-9, max_iter=200, recompute=20):
    """Returns dict(X, R, iters, eta, converged).  ``matvec`` applies Sigma
    (FP64), ``precond`` applies M^{-1}; both act on n x c blocks."""
    B = np.asarray(B, dtype=np.float64)
    X = precond(B)
    R = B - matvec(X)
    eta = _eta(R, X, B, sig_inf)
    active = eta > tol
    Z = precond(R)
    P = Z.copy()
    rz = np.sum(R * Z, axis=0)
    it = 0
    while np.any(active) and it < max_iter:
        it += 1
        Q = matvec(P)
        pq = np.sum(P * Q, axis=0)
        alpha = np.where(active, rz / np.where(pq != 0, pq, 1.0), 0.0)
        X = X + alpha * P
        if it % recompute == 0:
            R = np.where(active, B - matvec(X), R)
        else:
            R = R - alpha * Q
        eta_rec = _eta(R, X, B, sig_inf)
        check = active & (eta_rec <= tol)
        if np.any(check):
            Rt = B - matvec(X)
            eta_t = _eta(Rt, X, B, sig_inf)
            R = np.where(check, Rt, R)
            done = check & (eta_t <= tol)
            active = active & ~done
        Z = precond(R)
        rz_new = np.sum(R * Z, axis=0)
        beta = np.where(active, rz_new / np.where(rz != 0, rz, 1.0), 0.0)
        rz = np.where(active, rz_new, rz)
        P = np.where(active, Z + beta * P, P)
    R = B - matvec(X)
    eta = _eta(R, X, B, sig_inf)
    return dict(X=X, R=R, iters=it, eta=float(np.max(eta)), converged=bool(np.all(eta <= tol)))


def iterative_refinement(matvec, B, precond, sig_inf, tol=1e-9, max_iter=200):
    B = np.asarray(B, dtype=np.float64)
    X = precond(B)
    it = 0
    while True:
        R = B - matvec(X)
        eta = _eta(R, X, B, sig_inf)
        if np.all(eta <= tol) or it >= max_iter:
            break
        X = X + precond(R) * (eta > tol)
        it += 1
    return dict(X=X, R=R, iters=it, eta=float(np.max(eta)), converged=bool(np.all(eta <= tol)))


def quad_refined(Z, X, R) -> np.ndarray:
    """z^T x + x^T r per column."""
    return np.sum(Z * X, axis=0) + np.sum(X * R, axis=0)
