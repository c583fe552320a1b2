"""Maximum likelihood estimation of the Matern covariance parameters (oracle side).

The paper's MLE section minimises the negative log-likelihood
    nll(theta) = -l(theta) = (n/2) log 2 pi + (1/2) log|Sigma| + (1/2) z^T Sigma^{-1} z
over theta with R's optim, whose default method is the Nelder-Mead simplex,
with the smoothness nu held fixed and the parameters on the log scale
(range a = exp(p[0]), variance sigma^2 = exp(p[1])).

The simplex method here is the one defined by Nelder and Mead (1965) in the
form stated by Lagarias, Reeds, Wright and Wright (1998), with reflection 1,
expansion 2, contraction 1/2 and shrink 1/2:
  order the vertices by f; reflect the worst through the centroid of the
  others, xr = c + (c - x_worst); if f(best) <= f(xr) < f(second worst) accept
  xr; if f(xr) < f(best) try the expansion xe = c + 2 (xr - c) and keep the
  better of xe, xr; otherwise contract: outside, xc = c + (xr - c)/2, accepted
  if f(xc) <= f(xr), or inside, xcc = c - (c - x_worst)/2, accepted if
  f(xcc) < f(worst); a rejected contraction shrinks every vertex halfway
  towards the best.
Start: x0 and x0 + s e_i with s = 0.1 max|x0_i| (0.1 if x0 = 0), as R's optim
builds its first simplex.  Stop when f(worst) - f(best) <= reltol (|f(best)|
+ reltol) (R's relative tolerance test) or after max_iter iterations.  Ties in
the ordering keep the earlier vertex first (stable sort).
"""
from __future__ import annotations

import math

import numpy as np

from . import covariance as cov
from .dense import NotPositiveDefinite, loglik_fp64


def nelder_mead(f, x0, max_iter=500, reltol=1e-8):
    """Returns dict(x, fx, iters, evals)."""
    x0 = np.asarray(x0, dtype=np.float64)
    d = x0.size
    s = 0.1 * float(np.max(np.abs(x0))) if np.any(x0 != 0) else 0.1
    pts = [x0.copy()] + [x0 + s * np.eye(d)[i] for i in range(d)]
    vals = [f(p) for p in pts]
    evals = d + 1
    it = 0
    while True:
        order = sorted(range(d + 1), key=lambda i: vals[i])
        pts = [pts[i] for i in order]
        vals = [vals[i] for i in order]
        if vals[-1] - vals[0] <= reltol * (abs(vals[0]) + reltol) or it >= max_iter:
            break
        it += 1
        c = np.mean(pts[:-1], axis=0)
        xr = c + (c - pts[-1])
        fr = f(xr)
        evals += 1
        if vals[0] <= fr < vals[-2]:
            pts[-1], vals[-1] = xr, fr
            continue
        if fr < vals[0]:
            xe = c + 2.0 * (xr - c)
            fe = f(xe)
            evals += 1
            if fe < fr:
                pts[-1], vals[-1] = xe, fe
            else:
                pts[-1], vals[-1] = xr, fr
            continue
        if fr < vals[-1]:
            xc = c + 0.5 * (xr - c)
            fc = f(xc)
            evals += 1
            if fc <= fr:
                pts[-1], vals[-1] = xc, fc
                continue
        else:
            xcc = c - 0.5 * (c - pts[-1])
            fcc = f(xcc)
            evals += 1
            if fcc < vals[-1]:
                pts[-1], vals[-1] = xcc, fcc
                continue
        for i in range(1, d + 1):
            pts[i] = pts[0] + 0.5 * (pts[i] - pts[0])
            vals[i] = f(pts[i])
            evals += 1
    return dict(x=pts[0], fx=vals[0], iters=it, evals=evals)


def matern_nll(locs, z, nu, nugget):
    """The negative log-likelihood as a function of p = (log range, log
    variance), evaluated by the plain FP64 definition; +inf where Sigma is not
    numerically positive definite."""
    z = np.asarray(z, dtype=np.float64).reshape(-1, 1)

    def nll(p):
        a, s2 = math.exp(p[0]), math.exp(p[1])
        try:
            r = loglik_fp64(cov.covariance(locs, s2, a, nu, nugget), z)
        except NotPositiveDefinite:
            return math.inf
        return -float(r["loglik"][0])
    return nll
