"""Pins for the covariance and ordering oracle (oracle/covariance.py).

* the half-integer closed forms equal x^nu K_nu(x) / (2^(nu-1) Gamma(nu)) with
  K_nu from scipy.special.kv (the Matérn form of the paper's MLE section, read
  with M_nu(x) = x^nu K_nu(x));
* nu = 1/2 is the exponential covariance sigma^2 exp(-d / a) stated there;
* the Morton code equals a bit-string interleave computed independently, and
  the order is stable on ties.
"""
import math

import numpy as np
import pytest
from scipy.special import gamma, kv

from oracle import covariance as cov


@pytest.mark.parametrize("nu", [0.5, 1.5, 2.5])
def test_matern_closed_form_matches_bessel(nu):
    x = np.random.default_rng(1).uniform(1e-3, 30.0, 2000)
    ref = x ** nu * kv(nu, x) / (2.0 ** (nu - 1) * gamma(nu))
    np.testing.assert_allclose(cov.matern_correlation(x, nu), ref, rtol=1e-12, atol=1e-300)


def test_matern_zero_distance_and_exponential():
    for nu in (0.5, 1.5, 2.5):
        assert cov.matern_correlation(0.0, nu) == 1.0
    locs = np.random.default_rng(2).random((50, 2))
    S = cov.covariance(locs, 2.0, 0.3, 0.5, 0.0)
    d = np.array([[math.dist(p, q) for q in locs] for p in locs])
    np.testing.assert_allclose(S, 2.0 * np.exp(-d / 0.3), rtol=1e-14)


def test_covariance_symmetric_with_nugget():
    locs = np.random.default_rng(3).random((64, 2))
    S = cov.covariance(locs, 1.5, 0.1, 1.5, 1e-6)
    assert np.array_equal(S, S.T)
    np.testing.assert_array_equal(np.diag(S), np.full(64, 1.5 + 1e-6))
    blk = cov.covariance_block(locs[16:32], locs[0:16], 1.5, 0.1, 1.5, 1e-6, diag_offset=16)
    assert np.array_equal(blk, S[16:32, 0:16])


def _morton_by_strings(locs):
    out = []
    for x, y in locs:
        qx = min(int(math.floor(x * 65536.0)), 65535)
        qy = min(int(math.floor(y * 65536.0)), 65535)
        bx = format(qx, "016b")
        by = format(qy, "016b")
        s = "".join(b + a for a, b in zip(bx, by))   # y bit above x bit, MSB first
        out.append(int(s, 2))
    return np.array(out, dtype=np.uint64)


def test_morton_codes_bit_interleave():
    locs = np.random.default_rng(4).random((3000, 2))
    locs[:5] = [[0.0, 0.0], [0.999999999, 0.999999999], [0.5, 0.25], [0.25, 0.5], [1.0 - 2 ** -17, 0.0]]
    assert np.array_equal(cov.morton_codes(locs), _morton_by_strings(locs))


def test_morton_order_stable_on_ties():
    locs = np.array([[0.5, 0.5], [0.1, 0.1], [0.5, 0.5], [0.1, 0.1000001], [0.5, 0.5]])
    perm = cov.morton_order(locs)
    codes = cov.morton_codes(locs)[perm]
    assert np.all(np.diff(codes.astype(np.int64)) >= 0)
    ties = [p for p in perm if tuple(locs[p]) == (0.5, 0.5)]
    assert ties == [0, 2, 4]
