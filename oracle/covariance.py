"""Matérn covariance and spatial ordering (oracle side).

The paper (section "Maximum Likelihood Estimation of Matérn Covariance
Function") writes the covariance of two sites as
    sigma^2 / (2^(nu-1) Gamma(nu)) * M_nu(||s_i - s_j|| / a)
without defining M_nu.  Reading: M_nu(x) = x^nu K_nu(x) (K_nu the modified
Bessel function of the second kind), which makes C(0) = sigma^2 and reduces
for nu = 1/2 to the exponential covariance sigma^2 exp(-||s_i - s_j|| / a)
that the same section states.  For half-integer nu the Bessel function has a
closed form, which gives
    nu = 1/2 : exp(-x)
    nu = 3/2 : (1 + x) exp(-x)
    nu = 5/2 : (1 + x + x^2/3) exp(-x)
for the normalised correlation m_nu(x).  A nugget tau^2 is added to the
diagonal in FP64 (the section's R code adds 1e-6 to the diagonal for single
precision).

Ordering: the band map of the mixed-precision factor only makes sense when
nearby sites get nearby indices.  Reading: sort the sites by a Morton
(Z-order) code built from 16 bits per axis, stably.  The log-likelihood is
invariant under a joint permutation of the sites and the observations.
"""
from __future__ import annotations

import numpy as np

SUPPORTED_NU = (0.5, 1.5, 2.5)


def matern_correlation(x, nu: float) -> np.ndarray:
    """m_nu(x) for nu in {1/2, 3/2, 5/2}, x = distance / range >= 0."""
    x = np.asarray(x, dtype=np.float64)
    e = np.exp(-x)
    if nu == 0.5:
        return e
    if nu == 1.5:
        return (1.0 + x) * e
    if nu == 2.5:
        return (1.0 + x + x * x / 3.0) * e
    raise ValueError(f"nu must be one of {SUPPORTED_NU}")


def distances(locs_a: np.ndarray, locs_b: np.ndarray) -> np.ndarray:
    """Euclidean distances between the rows of two point arrays (na x 2, nb x 2)."""
    dx = locs_a[:, 0][:, None] - locs_b[:, 0][None, :]
    dy = locs_a[:, 1][:, None] - locs_b[:, 1][None, :]
    return np.sqrt(dx * dx + dy * dy)


def covariance_block(locs_r, locs_c, sigma2, range_, nu, nugget=0.0, diag_offset=None):
    """Block of Sigma with rows at ``locs_r`` and columns at ``locs_c``.
    ``diag_offset`` = (first row index - first column index) when the block
    touches the diagonal; the nugget goes on entries whose global row and column
    coincide."""
    cov = sigma2 * matern_correlation(distances(locs_r, locs_c) / range_, nu)
    if nugget and diag_offset is not None:
        r = np.arange(locs_r.shape[0])[:, None] + diag_offset
        c = np.arange(locs_c.shape[0])[None, :]
        cov = cov + np.where(r == c, nugget, 0.0)
    return cov


def covariance(locs, sigma2, range_, nu, nugget=0.0) -> np.ndarray:
    """Dense n x n covariance matrix Sigma(theta) + nugget * I (float64)."""
    return covariance_block(locs, locs, sigma2, range_, nu, nugget, diag_offset=0)


def morton_codes(locs: np.ndarray) -> np.ndarray:
    """32-bit Z-order code of each site: each coordinate in [0,1) is quantised to
    16 bits (q = min(floor(65536 x), 65535)) and the bits are interleaved with
    bit b of x at position 2b and bit b of y at position 2b+1."""
    q = np.minimum(np.floor(np.clip(locs, 0.0, None) * 65536.0), 65535).astype(np.uint64)
    qx, qy = q[:, 0], q[:, 1]
    code = np.zeros(locs.shape[0], dtype=np.uint64)
    for b in range(16):
        code |= ((qx >> np.uint64(b)) & np.uint64(1)) << np.uint64(2 * b)
        code |= ((qy >> np.uint64(b)) & np.uint64(1)) << np.uint64(2 * b + 1)
    return code


def morton_order(locs: np.ndarray) -> np.ndarray:
    """Permutation that sorts the sites by Morton code, ties kept in input order."""
    return np.argsort(morton_codes(locs), kind="stable")
