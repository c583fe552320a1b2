"""Pins for the Laplace-approximation oracle (oracle/laplace.py).

* the mode is a stationary point of log p(y|x) + log N(x; 0, Sigma):
  g1(x0) = Q x0;
* on the exponential covariance of a regular 1-D grid (the KMS matrix) the
  pieces have closed forms: log|Q| = -(n log sigma^2 + (n-1) log(1-rho^2)),
  Q tridiagonal, and log|H| from LAPACK: the returned value is their sum;
* beta -> 0: the observations carry no information, the mode goes to 0 and
  the value to n log(1/2);
* one site: the mode solves x / sigma^2 = beta (y - pi(x)) (found by a root
  finder) and the value is the scalar formula.
* Simpson's rule integrates exp of a quadratic exactly to the grid's accuracy.
"""
import math

import numpy as np
import pytest

import synth
from oracle import laplace
from tests.test_oracle_dense import kms


def line(n, spacing=1.0):
    return synth.grid_1d(n, spacing)


def data(n, seed):
    g = np.random.default_rng(seed)
    return (g.random(n) < 0.5).astype(np.float64)


def test_mode_is_stationary():
    n = 40
    locs = line(n)
    y = data(n, 1)
    r = laplace.laplace_logpost(locs, y, 0.1, 0.6, 0.5, 10.0, tol=1e-24)
    x0 = r["mode"]
    rho = math.exp(-1.0 / 0.6)
    Q = np.linalg.inv(0.1 * kms(n, rho))
    pi = 1.0 / (1.0 + np.exp(-10.0 * x0))
    np.testing.assert_allclose(10.0 * (y - pi), Q @ x0, rtol=0, atol=1e-9)


@pytest.mark.parametrize("alpha", [0.2, 0.6, 0.95])
def test_pieces_on_the_kms_grid(alpha):
    n, s2, beta = 30, 0.1, 10.0
    locs = line(n)
    y = data(n, 2)
    r = laplace.laplace_logpost(locs, y, s2, alpha, 0.5, beta, tol=1e-24)
    x0 = r["mode"]
    rho = math.exp(-1.0 / alpha)
    logdet_Q = -(n * math.log(s2) + (n - 1) * math.log(1 - rho * rho))
    # tridiagonal precision of the KMS matrix
    Q = np.zeros((n, n))
    i = np.arange(n)
    Q[i, i] = 1 + rho * rho
    Q[0, 0] = Q[-1, -1] = 1.0
    Q[i[:-1], i[1:]] = Q[i[1:], i[:-1]] = -rho
    Q /= s2 * (1 - rho * rho)
    pi = 1.0 / (1.0 + np.exp(-beta * x0))
    _, logdet_H = np.linalg.slogdet(Q + np.diag(beta ** 2 * pi * (1 - pi)))
    lik = np.sum(beta * x0 * y - np.log1p(np.exp(beta * x0)))
    ref = lik + 0.5 * logdet_Q - 0.5 * x0 @ Q @ x0 - 0.5 * logdet_H
    assert abs(r["lpost"] - ref) <= 1e-10 * abs(ref)


def test_uninformative_observations():
    n = 25
    r = laplace.laplace_logpost(line(n), data(n, 3), 0.1, 0.5, 0.5, 1e-7, tol=1e-30)
    assert np.max(np.abs(r["mode"])) < 1e-6
    assert abs(r["lpost"] - n * math.log(0.5)) < 1e-9


@pytest.mark.parametrize("y", [0.0, 1.0])
def test_one_site_by_a_root_finder(y):
    from scipy.optimize import brentq
    s2, beta = 0.3, 4.0
    r = laplace.laplace_logpost(np.zeros((1, 2)), np.array([y]), s2, 0.5, 0.5, beta, tol=1e-30)
    f = lambda x: x / s2 - beta * (y - 1.0 / (1.0 + math.exp(-beta * x)))
    x = brentq(f, -10, 10, xtol=1e-15)
    assert abs(r["mode"][0] - x) < 1e-12
    pi = 1.0 / (1.0 + math.exp(-beta * x))
    w = beta * beta * pi * (1 - pi)
    ref = beta * x * y - math.log1p(math.exp(beta * x)) - 0.5 * math.log(s2) - 0.5 * x * x / s2 \
        - 0.5 * math.log(1 / s2 + w)
    assert abs(r["lpost"] - ref) < 1e-12


def test_simpson_posterior_normalises():
    a = np.linspace(0.05, 0.95, 21)
    lp = -0.5 * ((a - 0.4) / 0.1) ** 2
    post = laplace.posterior(a, lp)
    exact = np.exp(-0.5 * ((a - 0.4) / 0.1) ** 2) / (0.1 * math.sqrt(2 * math.pi))
    np.testing.assert_allclose(post, exact, rtol=2e-3)
