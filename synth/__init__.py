"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This module only draws random numbers and shapes them; it holds none of the
method's arithmetic (no covariance, ordering, rounding or factorisation).  The
workloads follow the paper's spatial experiments (points in the unit square,
Gaussian observations z ~ N(0, 1), Matérn parameters) and its GEMM example
(uniform matrix entries), with the sizes of the workloads listed below.
All draws use numpy's PCG64 generator so that every side sees the same arrays.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "rng", "locations", "normal_rhs", "uniform_matrix", "integer_matrix",
    "grid_1d", "grid_2d", "serving_requests", "WORKLOADS",
]


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def locations(n: int, seed: int) -> np.ndarray:
    """n points drawn uniformly from [0,1)^2, returned as an n x 2 float64
    array (column 0 = x, column 1 = y)."""
    return rng(seed).random((n, 2))


def normal_rhs(n: int, nrhs: int, seed: int) -> np.ndarray:
    """n x nrhs standard normal observations, Fortran (column-major) order."""
    return np.asfortranarray(rng(seed).standard_normal((n, nrhs)))


def uniform_matrix(m: int, n: int, seed: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    """m x n matrix with U(lo, hi) entries, column-major."""
    return np.asfortranarray(rng(seed).uniform(lo, hi, size=(m, n)))


def integer_matrix(m: int, n: int, seed: int, lo: int = -4, hi: int = 4) -> np.ndarray:
    """m x n matrix of integers in [lo, hi] stored as float64, column-major."""
    return np.asfortranarray(rng(seed).integers(lo, hi + 1, size=(m, n)).astype(np.float64))


def grid_1d(n: int, spacing: float) -> np.ndarray:
    """n points on a regular 1-D grid along the x axis (y = 0), n x 2."""
    out = np.zeros((n, 2))
    out[:, 0] = np.arange(n, dtype=np.float64) * spacing
    return out


def grid_2d(m: int) -> np.ndarray:
    """The m x m regular grid on the unit square, points (i/(m-1), j/(m-1)),
    x varying fastest (the layout of R's expand.grid), as an m^2 x 2 array."""
    t = np.arange(m, dtype=np.float64) / (m - 1)
    out = np.empty((m * m, 2))
    out[:, 0] = np.tile(t, m)
    out[:, 1] = np.repeat(t, m)
    return out


def serving_requests(count: int, seed: int, n_lo: int = 256, n_hi: int = 8192):
    """A stream of likelihood requests: n log-uniform in [n_lo, n_hi], each with
    its own parameters (variance U(0.5,2), range U(0.02,0.3), smoothness drawn
    from {0.5, 1.5, 2.5}, nugget 1e-6), its own points and one N(0,1) response.
    Returns a list of dicts; the per-request arrays are drawn lazily from a
    per-request seed so that a long stream costs little memory."""
    g = rng(seed)
    ns = np.rint(np.exp(g.uniform(np.log(n_lo), np.log(n_hi), size=count))).astype(np.int64)
    sig = g.uniform(0.5, 2.0, size=count)
    rng_ = g.uniform(0.02, 0.3, size=count)
    nu = np.array([0.5, 1.5, 2.5])[g.integers(0, 3, size=count)]
    sub = g.integers(0, 2**62, size=count)
    reqs = []
    for i in range(count):
        reqs.append(dict(id=i, n=int(ns[i]), sigma2=float(sig[i]), range=float(rng_[i]),
                         nu=float(nu[i]), nugget=1e-6, seed=int(sub[i])))
    return reqs


def request_arrays(req: dict):
    """Points and response of one serving request."""
    g = rng(req["seed"])
    locs = g.random((req["n"], 2))
    z = np.asfortranarray(g.standard_normal((req["n"], 1)))
    return locs, z


# The workloads: sizes, parameters and seeds.  Each is a small dict; the
# arrays are drawn from the seeds above on demand.
WORKLOADS = {
    # Plain FP64 path: exponential covariance, 1024 points, one response.
    "fp64_n1024": dict(n=1024, nb=256, nrhs=1, nu=0.5, sigma2=1.0, range=0.1,
                       nugget=1e-8, seed_locs=1, seed_z=2, map="fp64"),
    # Multi-precision GEMM sweep, m = n = k = 8192, U(-1, 1) entries.
    "gemm_8192": dict(m=8192, n=8192, k=8192, seed=3),
    # Mixed-precision tile Cholesky, n = 32768, nb = 512, Matérn 3/2.
    "mixed_n32768": dict(n=32768, nb=512, nrhs=16, nu=1.5, sigma2=1.0, range=0.05,
                         nugget=1e-6, seed_locs=4, seed_z=5,
                         map="band", bands=((2, "fp64"), (8, "fp32"), (None, "bf16"))),
    # Serving stream.
    "serve_4096": dict(count=4096, seed=6, n_lo=256, n_hi=8192, nb=256),
    # Maximum likelihood fit on a regular grid (the MLE example's 120 x 120
    # grid, exponential covariance, variance 1, range 0.03, nu fixed at 1/2,
    # optimiser started from p = (log range, log variance) = (1.5, -0.3)).
    "mle_grid120": dict(m=120, nu=0.5, sigma2=1.0, range=0.03, nugget=0.0, seed_z=1234, x0=(1.5, -0.3),
                        max_iter=1000, reltol=1e-8),
    # Large mixed factor, n = 65536, nb = 1024, Matérn 5/2.
    "mixed_n65536": dict(n=65536, nb=1024, nrhs=256, nu=2.5, sigma2=1.0, range=0.05,
                         nugget=1e-6, seed_locs=7, seed_z=8,
                         map="band", bands=((1, "fp64"), (4, "fp32"), (15, "fp16"), (None, "fp8"))),
}
