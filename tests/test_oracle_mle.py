"""Pins for the Nelder-Mead MLE driver of the oracle (oracle/mle.py).

* one iteration traced by hand on f(x) = x0^2 + 2 x1^2 from (1, 1): the first
  simplex, the reflection and the accepted expansion;
* convergence to the minimiser of a quadratic, and to the Rosenbrock
  minimiser where scipy's Nelder-Mead also ends;
* the negative log-likelihood's parametrisation (range = exp(p0), variance =
  exp(p1)) against the closed form of the exponential covariance on a 1-D
  grid (the KMS matrix).
"""
import math

import numpy as np
import pytest

import synth
from oracle import mle
from tests.test_oracle_dense import kms_loglik_closed_form


def test_first_iteration_by_hand():
    f = lambda x: x[0] ** 2 + 2 * x[1] ** 2
    # simplex (1,1):3, (1.1,1):3.21, (1,1.1):3.42; centroid of the best two
    # (1.05, 1); reflection (1.1, 0.9): 2.83 < 3 -> expansion (1.15, 0.8): 2.6025
    r = mle.nelder_mead(f, [1.0, 1.0], max_iter=1)
    assert r["iters"] == 1 and r["evals"] == 5
    np.testing.assert_allclose(r["x"], [1.15, 0.8], rtol=0, atol=1e-15)
    assert abs(r["fx"] - 2.6025) <= 1e-14


def test_converges_on_a_quadratic():
    a = np.array([0.3, -1.2])
    H = np.array([[2.0, 0.5], [0.5, 1.0]])
    f = lambda x: float((x - a) @ H @ (x - a)) + 7.0
    r = mle.nelder_mead(f, [2.0, 2.0], max_iter=2000, reltol=1e-14)
    np.testing.assert_allclose(r["x"], a, atol=1e-5)
    assert abs(r["fx"] - 7.0) <= 1e-9


def test_rosenbrock_agrees_with_scipy():
    from scipy.optimize import minimize
    f = lambda x: 100.0 * (x[1] - x[0] ** 2) ** 2 + (1 - x[0]) ** 2
    r = mle.nelder_mead(f, [-1.2, 1.0], max_iter=5000, reltol=1e-16)
    s = minimize(f, [-1.2, 1.0], method="Nelder-Mead", options=dict(xatol=1e-10, fatol=1e-14, maxiter=5000))
    np.testing.assert_allclose(r["x"], [1.0, 1.0], atol=1e-4)
    np.testing.assert_allclose(r["x"], s.x, atol=1e-4)


@pytest.mark.parametrize("a,s2", [(8.0 / 300, 1.0), (0.05, 2.5)])
def test_nll_parametrisation_on_the_kms_grid(a, s2):
    n = 300
    h = 1.0 / n
    locs = synth.grid_1d(n, h)
    z = synth.normal_rhs(n, 1, 12)[:, 0]
    nll = mle.matern_nll(locs, z, 0.5, 0.0)
    _, _, ref = kms_loglik_closed_form(z, s2, math.exp(-h / a))
    assert abs(nll([math.log(a), math.log(s2)]) + ref) <= 1e-10 * abs(ref)
