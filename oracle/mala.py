"""Metropolis-adjusted Langevin sampler (oracle side): the paper's section
"Metropolis-Hastings Algorithm in High Dimensions", in its steps and notation.

Target N(mu, Sigma) with mu = 0; preconditioner M; step h.  The section forms
sig.inv = Sigma^{-1}, L = t(chol(h M)) and pre_M_inv = (h M)^{-1}, and with
    grad(x) = Sigma^{-1} x,   step(x, t) = x - t M grad(x)
iterates
    z_prop = step(z, h/2) + L eps
    p_prop = -1/2 z_prop^T Sigma^{-1} z_prop,    p_curr = -1/2 z^T Sigma^{-1} z
    q_curr = -1/2 (z - step(z_prop, h/2))^T (h M)^{-1} (z - step(z_prop, h/2))
    q_prop = -1/2 (z_prop - step(z, h/2))^T (h M)^{-1} (z_prop - step(z, h/2))
    accept z_prop when u < exp(min(0, p_prop - p_curr + q_curr - q_prop)).
The normal draws eps (one column per iteration) and the uniforms u are
inputs.
"""
from __future__ import annotations

import numpy as np

from .dense import cholesky_lower


def mala(Sigma, Mpre, h, z0, eps, unif):
    """Returns dict(z, trace (n x iters), accepted, log_ratio)."""
    sig_inv = np.linalg.inv(Sigma)
    L = cholesky_lower(h * Mpre)
    pre_inv = np.linalg.inv(h * Mpre)
    grad = lambda x: sig_inv @ x
    step = lambda x, t: x - t * (Mpre @ grad(x))
    z = np.array(z0, dtype=np.float64)
    iters = eps.shape[1]
    trace = np.zeros((z.size, iters))
    acc = np.zeros(iters, dtype=bool)
    logr = np.zeros(iters)
    for i in range(iters):
        z_prop = step(z, 0.5 * h) + L @ eps[:, i]
        p_prop = -0.5 * z_prop @ sig_inv @ z_prop
        p_curr = -0.5 * z @ sig_inv @ z
        dc = z - step(z_prop, 0.5 * h)
        dp = z_prop - step(z, 0.5 * h)
        q_curr = -0.5 * dc @ pre_inv @ dc
        q_prop = -0.5 * dp @ pre_inv @ dp
        logr[i] = p_prop - p_curr + q_curr - q_prop
        if unif[i] < np.exp(min(0.0, logr[i])):
            z = z_prop
            acc[i] = True
        trace[:, i] = z
    return dict(z=z, trace=trace, accepted=acc, log_ratio=logr)
