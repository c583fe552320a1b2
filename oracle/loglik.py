"""End-to-end oracle for the Gaussian log-likelihood of a Matérn field.

Section "Maximum Likelihood Estimation of Matérn Covariance Function" of the
paper: l(theta) = -(n/2) log 2 pi - (1/2) log|Sigma(theta)| - (1/2) z^T
Sigma(theta)^{-1} z, evaluated through the Cholesky factor.  Two variants:

* ``loglik_plain``: the plain FP64 definition (dense Cholesky, forward solve,
  quad = ||L^{-1} z||^2);
* ``loglik_mixed``: the emulated mixed-precision tile factor, the log-
  determinant from its FP64 diagonal tiles, and the solve refined in FP64 to
  the backward-error tolerance (quad = z^T x + x^T r).

Sites are taken in the order given; ``order_sites`` applies the Morton order.
"""
from __future__ import annotations

import numpy as np

from . import covariance as cov
from .dense import (NotPositiveDefinite, backward_substitution_transpose, forward_substitution,
                    gaussian_loglik, logdet_from_cholesky, loglik_fp64)
from .refine import block_pcg, gmres_ir, iterative_refinement, pcg, quad_refined
from .tiled import promote_after_breakdown, tile_cholesky_emulated


def order_sites(locs, Z):
    perm = cov.morton_order(locs)
    return locs[perm], (Z[perm] if Z is not None else None), perm


def loglik_plain(locs, Z, sigma2, range_, nu, nugget):
    S = cov.covariance(locs, sigma2, range_, nu, nugget)
    return loglik_fp64(S, Z)


def loglik_mixed(locs, Z, sigma2, range_, nu, nugget, nb, tmap, tol=1e-9, max_iter=200, solver="pcg",
                 promote=False):
    """With ``promote``, a breakdown is followed by a refactorisation with the
    map of ``promote_after_breakdown`` until the factor exists or nothing is
    left to promote; the map used and the number of promotions are returned."""
    Z = np.asarray(Z, dtype=np.float64)
    Z2 = Z[:, None] if Z.ndim == 1 else Z
    n = locs.shape[0]
    S = cov.covariance(locs, sigma2, range_, nu, nugget)
    promotions = 0
    while True:
        fac = tile_cholesky_emulated(S, nb, tmap)
        if not (fac["info"] and promote):
            break
        nxt = promote_after_breakdown(tmap, nb, fac["info"])
        if np.array_equal(nxt, tmap):
            break
        tmap, promotions = nxt, promotions + 1
    if fac["info"]:
        return dict(info=fac["info"], L=fac["L"], map=tmap, promotions=promotions)
    L = fac["L"][:n, :n]
    logdet = logdet_from_cholesky(L)
    sig_inf = float(np.max(np.sum(np.abs(S), axis=1)))
    matvec = lambda X: S @ X
    precond = lambda R: backward_substitution_transpose(L, forward_substitution(L, R))
    run = {"pcg": pcg, "ir": iterative_refinement, "gmres": gmres_ir, "bpcg": block_pcg}[solver]
    res = run(matvec, Z2, precond, sig_inf, tol=tol, max_iter=max_iter)
    quad = quad_refined(Z2, res["X"], res["R"])
    rel = np.linalg.norm(res["R"], axis=0) / np.linalg.norm(Z2, axis=0)
    return dict(info=0, L=L, logdet=logdet, quad=quad, loglik=gaussian_loglik(n, logdet, quad),
                X=res["X"], iters=res["iters"], eta=res["eta"], converged=res["converged"],
                rel_resid2=float(np.max(rel)), map=tmap, promotions=promotions)
