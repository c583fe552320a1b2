"""Laplace approximation of a latent Gaussian model with Bernoulli
observations (oracle side): the paper's "Integrated Nested Multi-Precision
Arithmetic Laplace Approximation" section, written out in the section's steps
and notation.

Model: latent field x ~ N(0, Sigma(alpha)) with the exponential (Matern)
covariance sigma^2 m_nu(d / alpha), observations y_i in {0, 1} with
P(y_i = 1) = 1 / (1 + exp(-beta x_i)).  For each alpha:
* Q = Sigma^{-1} (the section forms the dense precision matrix by inversion);
* Newton iterations from x0 = 0:
      g1 = beta y - beta e^{beta x0} / (1 + e^{beta x0})     (gradient of log p(y|x))
      g2 = -beta^2 e^{beta x0} / (1 + e^{beta x0})^2          (its diagonal Hessian)
      x  = (Q - diag(g2))^{-1} (g1 - x0 g2)
  until mean((x - x0)^2) < tol, else x0 <- x; the mode is the last x;
* H = Q + diag(beta^2 e^{beta x0} / (1 + e^{beta x0})^2) at the mode;
* log posterior (up to a constant)
      sum(beta x0 y - log(1 + e^{beta x0})) + log|Q|/2 - x0^T Q x0 / 2 - log|H|/2,
  the log-determinants from Cholesky factors;
* over an equally spaced alpha grid: subtract the mean of the values,
  exponentiate and normalise with Simpson's rule (weights 1, 4, 2, ..., 4, 1).
"""
from __future__ import annotations

import numpy as np

from . import covariance as cov
from .dense import cholesky_lower, logdet_from_cholesky


def laplace_logpost(locs, y, sigma2, alpha, nu, beta, tol=1e-12, max_newton=100):
    """Returns dict(lpost, mode, iters)."""
    y = np.asarray(y, dtype=np.float64)
    n = y.size
    Q = np.linalg.inv(cov.covariance(locs, sigma2, alpha, nu, 0.0))
    x0 = np.zeros(n)
    it = 0
    while True:
        it += 1
        e = np.exp(beta * x0)
        g1 = beta * y - beta * e / (1.0 + e)
        g2 = -beta ** 2 * e / (1.0 + e) ** 2
        x = np.linalg.solve(Q - np.diag(g2), g1 - x0 * g2)
        if np.mean((x - x0) ** 2) < tol:
            break
        if it >= max_newton:
            raise RuntimeError("Newton iteration did not converge")
        x0 = x
    x0 = x
    e = np.exp(beta * x0)
    H = Q + np.diag(beta ** 2 * e / (1.0 + e) ** 2)
    Qs = 0.5 * (Q + Q.T)   # the inverse is symmetric up to rounding; the factor reads the lower triangle
    logdet_Q = logdet_from_cholesky(cholesky_lower(Qs))
    logdet_H = logdet_from_cholesky(cholesky_lower(0.5 * (H + H.T)))
    quad = float(x0 @ Q @ x0)
    lpost = float(np.sum(beta * x0 * y - np.log1p(np.exp(beta * x0)))) + 0.5 * logdet_Q - 0.5 * quad - 0.5 * logdet_H
    return dict(lpost=lpost, mode=x0, iters=it)


def posterior(alphas, lposts):
    """exp(l - mean l) normalised by Simpson's rule on the equally spaced grid."""
    lp = np.asarray(lposts, dtype=np.float64)
    lp = lp - lp.mean()
    h = alphas[1] - alphas[0]
    m = len(alphas)
    w = np.array([1.0] + [4.0 if i % 2 == 1 else 2.0 for i in range(1, m - 1)] + [1.0])
    z = np.sum(w * np.exp(lp)) * h / 3.0
    return np.exp(lp) / z
