"""Pins for the MALA oracle (oracle/mala.py).

* the log acceptance ratio of every iteration equals the one assembled from
  scipy's multivariate normal log-densities of the target and of the two
  proposal distributions N(step(., h/2), h M) (normalising constants cancel);
* the proposal noise is L eps with L L^T = h M (LAPACK Cholesky);
* h -> 0: proposals stay at the current state and are always accepted;
* u = 1 never accepts (exp(min(0, .)) <= 1 and equality needs log r >= 0,
  which the case below avoids), u = 0 always accepts.
"""
import numpy as np
from scipy.stats import multivariate_normal as mvn

import synth
from oracle import covariance as cov
from oracle import mala


def setup(m=6, seed=3, iters=12, h=0.01):
    locs = synth.grid_2d(m)
    n = m * m
    S = cov.covariance(locs, 1.0, 0.5, 0.5, 0.0)
    M = cov.covariance(locs, 1.0, 0.05, 0.5, 0.0)
    g = synth.rng(seed)
    z0 = g.random(n)
    eps = g.standard_normal((n, iters))
    unif = g.random(iters)
    return S, M, h, z0, eps, unif


def test_log_ratio_matches_scipy_densities():
    S, M, h, z0, eps, unif = setup()
    r = mala.mala(S, M, h, z0, eps, unif)
    Sinv = np.linalg.inv(S)
    step = lambda x: x - 0.5 * h * (M @ (Sinv @ x))
    L = np.linalg.cholesky(h * M)
    z = z0.copy()
    for i in range(eps.shape[1]):
        zp = step(z) + L @ eps[:, i]
        ref = (mvn.logpdf(zp, np.zeros(z.size), S) - mvn.logpdf(z, np.zeros(z.size), S)
               + mvn.logpdf(z, step(zp), h * M) - mvn.logpdf(zp, step(z), h * M))
        assert abs(r["log_ratio"][i] - ref) <= 1e-8 * max(1.0, abs(ref)), (i, r["log_ratio"][i], ref)
        if r["accepted"][i]:
            z = zp
        np.testing.assert_allclose(r["trace"][:, i], z, rtol=0, atol=1e-12)


def test_tiny_step_always_accepts():
    S, M, _, z0, eps, unif = setup(h=1e-14)
    r = mala.mala(S, M, 1e-14, z0, eps, unif)
    assert r["accepted"].all()
    np.testing.assert_allclose(r["z"], z0, atol=1e-5)


def test_uniform_extremes():
    S, M, h, z0, eps, _ = setup()
    iters = eps.shape[1]
    r0 = mala.mala(S, M, h, z0, eps, np.zeros(iters))
    assert r0["accepted"].all() or np.all(r0["log_ratio"][~r0["accepted"]] == -np.inf)
    r1 = mala.mala(S, M, h, z0, eps, np.ones(iters))
    assert not np.any(r1["accepted"] & (r1["log_ratio"] < 0))
