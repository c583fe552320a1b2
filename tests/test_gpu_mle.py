"""GPU parity of the maximum likelihood driver (mpcr_mle_fit, Nelder-Mead over
p = (log range, log variance), nu fixed) against the oracle's Nelder-Mead on
the oracle's plain FP64 negative log-likelihood.

The data are a Gaussian field on a regular grid drawn with the oracle's
covariance (z = L_true e, e ~ N(0, 1)).  Both sides run the same simplex
rules from the same start; their objective values agree to ~1e-12, so the
simplex paths coincide unless two vertices tie to that level.  Gates: the
oracle's objective at the GPU's optimum is within the stopping tolerance of
its value at its own optimum, the optima agree to the simplex's resolution,
and when the iteration counts agree the optima agree to rounding.  A mixed
map with FP32 far tiles ends at the same estimate (the MLE section's
observation that single precision gives the same estimates on such data).
"""
import ctypes
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import synth  # noqa: E402
from oracle import covariance as cov  # noqa: E402
from oracle import mle  # noqa: E402
from oracle import tiled  # noqa: E402


@pytest.fixture(scope="module")
def g():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from tests import gpu_util
    ctx = gpu_util.Ctx()
    yield gpu_util, ctx
    ctx.close()


def field(m, s2, a, nu, nugget, seed):
    locs = synth.grid_2d(m)
    S = cov.covariance(locs, s2, a, nu, nugget)
    e = synth.normal_rhs(m * m, 1, seed)[:, 0]
    return locs, np.linalg.cholesky(S) @ e


def fit(gu, ctx, locs, z, nu, nugget, x0, m=None, nb=256, refine=None, max_iter=500, reltol=1e-8):
    from paper_2406_02701_amd import mpcr
    n = locs.shape[0]
    dl, dz = gu.dev(locs), gu.dev(z)
    x = np.zeros(2)
    f = ctypes.c_double()
    it, ev = ctypes.c_int(), ctypes.c_int()
    hm = None if m is None else gu.u8map(m)
    tm = None if m is None else ctypes.byref(mpcr.tilemap(n, nb, hm))
    x0a = np.asarray(x0, dtype=np.float64)
    ctx.check(mpcr.mpcr_mle_fit(ctx.ptr, n, dl.data_ptr(), dz.data_ptr(), nu, nugget, tm,
                                None if refine is None else ctypes.byref(refine), mpcr.f64p(x0a), max_iter, reltol,
                                mpcr.f64p(x), ctypes.byref(f), ctypes.byref(it), ctypes.byref(ev)))
    return x, f.value, it.value, ev.value


def test_mle_fp64_matches_oracle(g):
    gu, ctx = g
    locs, z = field(24, 1.0, 0.1, 0.5, 1e-6, 31)
    x0 = (math.log(0.05), math.log(0.5))
    x, f, it, ev = fit(gu, ctx, locs, z, 0.5, 1e-6, x0)
    # the oracle works in the same (Morton) order as the library's evaluations
    perm = cov.morton_order(locs)
    nll = mle.matern_nll(locs[perm], z[perm], 0.5, 1e-6)
    ref = mle.nelder_mead(nll, x0, max_iter=500, reltol=1e-8)
    print(f"GPU x {x} nll {f!r} iters {it} evals {ev}; oracle x {ref['x']} nll {ref['fx']!r} "
          f"iters {ref['iters']} evals {ref['evals']}", flush=True)
    assert abs(f - ref["fx"]) <= 1e-9 * abs(ref["fx"]) + 1e-8 * (abs(ref["fx"]) + 1e-8)
    assert abs(nll(x) - ref["fx"]) <= 2e-8 * (abs(ref["fx"]) + 1e-8)
    np.testing.assert_allclose(x, ref["x"], atol=5e-3)
    if it == ref["iters"] and ev == ref["evals"]:
        np.testing.assert_allclose(x, ref["x"], rtol=0, atol=1e-9)


def test_mle_mixed_map_same_estimate(g):
    from paper_2406_02701_amd import mpcr
    gu, ctx = g
    m_ = 48
    locs, z = field(m_, 1.0, 0.03, 0.5, 1e-6, 32)
    n, nb = m_ * m_, 256
    x0 = (math.log(0.05), math.log(0.5))
    x64, f64, _, _ = fit(gu, ctx, locs, z, 0.5, 1e-6, x0, m=tiled.tilemap_uniform(n, nb), nb=nb)
    mixed = tiled.tilemap_banded(n, nb, ((1, "fp64"), (None, "fp32")))
    ref = mpcr.mpcr_refine_opts_t(1e-13, 100, 0, 20, 0, 1)
    xm, fm, _, _ = fit(gu, ctx, locs, z, 0.5, 1e-6, x0, m=mixed, nb=nb, refine=ref)
    print(f"fp64 x {x64} nll {f64!r}; mixed x {xm} nll {fm!r}", flush=True)
    np.testing.assert_allclose(xm, x64, atol=5e-3)
    assert abs(fm - f64) <= 1e-6 * abs(f64)
