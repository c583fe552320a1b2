"""GPU parity of the MALA sampler (mpcr_mala_run) against the oracle's literal
evaluation of the paper's MALA example (which inverts Sigma and h M).

Grid of m x m sites in the unit square, target N(0, exp(-d/0.5)),
preconditioner M = exp(-d/0.05), h = 0.01 (the section's parameters), initial
state U(0,1), normal draws and uniforms passed in.  Both sides make the same
accept decisions (every decision's margin |log r - log u| is far above the
two sides' rounding differences, checked on the oracle), the log acceptance
ratios agree to 1e-9 relative and the states along the chain to 1e-9.
"""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import synth  # noqa: E402
from oracle import covariance as cov  # noqa: E402
from oracle import mala  # noqa: E402
from oracle import tiled  # noqa: E402


@pytest.fixture(scope="module")
def g():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from tests import gpu_util
    ctx = gpu_util.Ctx()
    yield gpu_util, ctx
    ctx.close()


def inputs(m, iters, seed):
    locs = synth.grid_2d(m)
    n = m * m
    gen = synth.rng(seed)
    z0 = gen.random(n)
    eps = np.asfortranarray(gen.standard_normal((n, iters)))
    unif = gen.random(iters)
    return locs, z0, eps, unif


def run(gu, ctx, locs, z0, eps, unif, h, m=None, nb=256):
    from paper_2406_02701_amd import mpcr
    n, iters = eps.shape
    dl, dz0, de = gu.dev(locs), gu.dev(z0), gu.dev(eps)
    zout = torch.zeros(n, dtype=torch.float64, device="cuda")
    trace = gu.empty(n, iters)
    acc = (ctypes.c_int * iters)()
    lr = np.zeros(iters)
    ts = gu.theta(1.0, 0.5, 0.5, 0.0)
    tm_ = gu.theta(1.0, 0.05, 0.5, 0.0)
    hm = None if m is None else gu.u8map(m)
    tm = None if m is None else ctypes.byref(mpcr.tilemap(n, nb, hm))
    u = np.ascontiguousarray(unif)
    ctx.check(mpcr.mpcr_mala_run(ctx.ptr, n, dl.data_ptr(), ctypes.byref(ts), ctypes.byref(tm_), h, dz0.data_ptr(),
                                 iters, de.data_ptr(), mpcr.f64p(u), tm, zout.data_ptr(), trace.data_ptr(), acc,
                                 mpcr.f64p(lr)))
    torch.cuda.synchronize()
    return zout.cpu().numpy(), gu.host(trace, (n, iters)), np.array(list(acc), bool), lr


def test_mala_matches_oracle(g):
    gu, ctx = g
    m, iters, h = 20, 60, 0.01
    locs, z0, eps, unif = inputs(m, iters, 51)
    S = cov.covariance(locs, 1.0, 0.5, 0.5, 0.0)
    M = cov.covariance(locs, 1.0, 0.05, 0.5, 0.0)
    ref = mala.mala(S, M, h, z0, eps, unif)
    margin = np.abs(np.minimum(ref["log_ratio"], 0.0) - np.log(unif))
    assert margin.min() > 1e-6        # no decision is near a tie
    z, trace, acc, lr = run(gu, ctx, locs, z0, eps, unif, h)
    print(f"MALA m={m}: accepted {acc.sum()}/{iters}; max |dlogr| {np.max(np.abs(lr - ref['log_ratio'])):.2e}; "
          f"max |dz| {np.max(np.abs(trace - ref['trace'])):.2e}", flush=True)
    assert np.array_equal(acc, ref["accepted"])
    np.testing.assert_allclose(lr, ref["log_ratio"], rtol=1e-9, atol=1e-9)
    np.testing.assert_allclose(trace, ref["trace"], rtol=0, atol=1e-9)
    np.testing.assert_allclose(z, ref["z"], rtol=0, atol=1e-9)
