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
* GMRES-IR: refinement whose correction equation Sigma d = r is solved by
  GMRES on the left-preconditioned system M^{-1} Sigma d = M^{-1} r (Carson
  and Higham, SIAM J. Sci. Comput. 40 (2018)), with the residual r in FP64.
  The inner GMRES is the method of Saad and Schultz (1986): Arnoldi with
  modified Gram-Schmidt, the Hessenberg least-squares problem reduced by
  Givens rotations, stopped when the rotated residual |g_{j+1}| drops to
  inner_tol times |M^{-1} r| or after m steps.
* Block PCG: the block conjugate gradient method of O'Leary (Linear Algebra
  Appl. 29 (1980)) with the preconditioner M, run on groups of up to
  ``block`` consecutive right-hand sides: with Z = M^{-1} R,
      alpha = (P^T Sigma P)^{-1} (Z^T R),  X += P alpha,  R -= Sigma P alpha,
      beta = (Z^T R)_old^{-1} (Z^T R)_new,  P = Z + P beta,
  the s x s systems solved by Cholesky.  If P^T Sigma P is not numerically
  positive definite (a pivot of its unit-diagonal scaling below 1e-12) the
  group continues with PCG from its current iterate.

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


def pcg(matvec, B, precond, sig_inf, tol=1e-9, max_iter=200, recompute=20, X0=None):
    """Returns dict(X, R, iters, eta, converged).  ``matvec`` applies Sigma
    (FP64), ``precond`` applies M^{-1}; both act on n x c blocks.  The start
    is X0, or M^{-1} B when X0 is None."""
    B = np.asarray(B, dtype=np.float64)
    X = precond(B) if X0 is None else np.array(X0, dtype=np.float64)
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


def gmres_correction(apply_op, r0, m, inner_tol):
    """GMRES on op(d) = r0 for one column: returns (d, steps, estimates), the
    estimates being the rotated residual norms |g_1|, ..., |g_k| of the
    Hessenberg least-squares problem (each equals ||r0 - op(d_j)||)."""
    n = r0.shape[0]
    beta = float(np.linalg.norm(r0))
    if beta == 0.0:
        return np.zeros(n), 0, []
    V = np.zeros((n, m + 1))
    H = np.zeros((m + 1, m))
    cs = np.zeros(m)
    sn = np.zeros(m)
    g = np.zeros(m + 1)
    g[0] = beta
    V[:, 0] = r0 / beta
    k = 0
    est = []
    for j in range(m):
        w = apply_op(V[:, j])
        for i in range(j + 1):                      # modified Gram-Schmidt
            H[i, j] = V[:, i] @ w
            w = w - H[i, j] * V[:, i]
        H[j + 1, j] = float(np.linalg.norm(w))
        for i in range(j):                          # earlier rotations on the new column
            t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
            H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
            H[i, j] = t
        a, b = H[j, j], H[j + 1, j]
        r = float(np.hypot(a, b))
        cs[j], sn[j] = (a / r, b / r) if r != 0.0 else (1.0, 0.0)
        H[j, j] = r
        H[j + 1, j] = 0.0
        g[j + 1] = -sn[j] * g[j]
        g[j] = cs[j] * g[j]
        k = j + 1
        est.append(abs(g[j + 1]))
        if abs(g[j + 1]) <= inner_tol * beta or b == 0.0:
            break
        V[:, j + 1] = w / b
    y = np.zeros(k)
    for i in range(k - 1, -1, -1):                  # back substitution with the rotated H
        y[i] = (g[i] - H[i, i + 1:k] @ y[i + 1:k]) / H[i, i]
    return V[:, :k] @ y, k, est


def gmres_ir(matvec, B, precond, sig_inf, tol=1e-9, max_iter=50, m=20, inner_tol=1e-6):
    """GMRES-based iterative refinement.  Returns dict(X, R, iters, eta,
    converged, inner_steps) with ``iters`` the outer refinement steps and
    ``inner_steps`` the GMRES steps of every (outer step, column)."""
    B = np.asarray(B, dtype=np.float64)
    X = precond(B)
    it = 0
    inner = []
    while True:
        R = B - matvec(X)
        eta = _eta(R, X, B, sig_inf)
        if np.all(eta <= tol) or it >= max_iter:
            break
        steps = []
        for c in range(B.shape[1]):
            if eta[c] <= tol:
                steps.append(0)
                continue
            op = lambda v: precond(matvec(v[:, None]))[:, 0]
            d, k, _ = gmres_correction(op, precond(R[:, c:c + 1])[:, 0], m, inner_tol)
            X[:, c] += d
            steps.append(k)
        inner.append(steps)
        it += 1
    return dict(X=X, R=R, iters=it, eta=float(np.max(eta)), converged=bool(np.all(eta <= tol)),
                inner_steps=inner)


def _spd_solve(G, F):
    """G^{-1} F by Cholesky of the unit-diagonal scaling D G D (D = diag(G)^-1/2);
    None when a pivot of the scaled matrix is below 1e-12."""
    d = np.diag(G)
    if np.any(d <= 0.0):
        return None
    D = 1.0 / np.sqrt(d)
    Gs = D[:, None] * G * D[None, :]
    s = G.shape[0]
    L = np.zeros_like(Gs)
    for j in range(s):
        v = Gs[j, j] - L[j, :j] @ L[j, :j]
        if v <= 1e-12:
            return None
        L[j, j] = np.sqrt(v)
        L[j + 1:, j] = (Gs[j + 1:, j] - L[j + 1:, :j] @ L[j, :j]) / L[j, j]
    Y = np.linalg.solve(L, D[:, None] * F)
    return D[:, None] * np.linalg.solve(L.T, Y)


def block_pcg(matvec, B, precond, sig_inf, tol=1e-9, max_iter=200, recompute=20, block=32, history=False):
    """Block PCG over groups of up to ``block`` consecutive columns.  Returns
    dict(X, R, iters, eta, converged, fallback) (``iters``: the largest
    number of block iterations of a group; ``fallback``: groups that broke
    down and finished with PCG); with ``history`` also the direction blocks
    P_k and residual blocks R_k, Z_k of the first group."""
    B = np.asarray(B, dtype=np.float64)
    n, c = B.shape
    X = np.zeros_like(B)
    R = np.zeros_like(B)
    iters, fallback = 0, []
    hist = dict(P=[], R=[], Z=[])
    for g0 in range(0, c, block):
        cols = slice(g0, min(c, g0 + block))
        Bg = B[:, cols]
        Xg = precond(Bg)
        Rg = Bg - matvec(Xg)
        it = 0
        done = bool(np.all(_eta(Rg, Xg, Bg, sig_inf) <= tol))
        broke = False
        if not done:
            Zg = precond(Rg)
            Pg = Zg.copy()
            ZR = Zg.T @ Rg
            while it < max_iter:
                if history and g0 == 0:
                    hist["P"].append(Pg.copy()); hist["R"].append(Rg.copy()); hist["Z"].append(Zg.copy())
                Q = matvec(Pg)
                alpha = _spd_solve(Pg.T @ Q, ZR)
                if alpha is None:
                    broke = True
                    break
                it += 1
                Xg = Xg + Pg @ alpha
                if it % recompute == 0:
                    Rg = Bg - matvec(Xg)
                else:
                    Rg = Rg - Q @ alpha
                if np.all(_eta(Rg, Xg, Bg, sig_inf) <= tol):
                    Rg = Bg - matvec(Xg)            # confirm with the true residual
                    if np.all(_eta(Rg, Xg, Bg, sig_inf) <= tol):
                        done = True
                        break
                Zg = precond(Rg)
                ZRn = Zg.T @ Rg
                beta = _spd_solve(ZR, ZRn)
                if beta is None:
                    broke = True
                    break
                ZR = ZRn
                Pg = Zg + Pg @ beta
        if broke:
            fallback.append(g0 // block)
            out = pcg(matvec, Bg, precond, sig_inf, tol=tol, max_iter=max_iter - it, recompute=recompute, X0=Xg)
            Xg, it = out["X"], it + out["iters"]
        X[:, cols] = Xg
        R[:, cols] = Bg - matvec(Xg)
        iters = max(iters, it)
    eta = _eta(R, X, B, sig_inf)
    out = dict(X=X, R=R, iters=iters, eta=float(np.max(eta)), converged=bool(np.all(eta <= tol)), fallback=fallback)
    if history:
        out["history"] = hist
    return out
