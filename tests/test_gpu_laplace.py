"""GPU parity of the Laplace-approximation driver (mpcr_inla_posterior) against
the oracle's literal evaluation of the paper's INLA analogue.

Workload of the section: n sites on a line (spacing n / (n - 1)), latent field
x ~ N(0, 0.1 exp(-d / 0.6)), Bernoulli observations with logit link and
beta = 10, and the log posterior of the range on 21 equally spaced values in
[0.05, 0.95].  The oracle inverts Sigma and solves with Q - diag(g2) as the
section does; the library never forms Q (it factors I + W^1/2 Sigma W^1/2 in
the tile store).  Gates: the log-posterior values to 1e-9 relative, the
normalised posterior to 1e-8 absolute, equal Newton step counts, and the mode.
"""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import synth  # noqa: E402
from oracle import covariance as cov  # noqa: E402
from oracle import laplace  # noqa: E402
from oracle import tiled  # noqa: E402


@pytest.fixture(scope="module")
def g():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from tests import gpu_util
    ctx = gpu_util.Ctx()
    yield gpu_util, ctx
    ctx.close()


def inla_data(n, seed):
    locs = synth.grid_1d(n, n / (n - 1))
    S = cov.covariance(locs, 0.1, 0.6, 0.5, 0.0)
    e = synth.normal_rhs(n, 1, seed)[:, 0]
    x = np.linalg.cholesky(S) @ e
    u = synth.rng(seed + 1).random(n)
    y = (u < 1.0 / (1.0 + np.exp(-10.0 * x))).astype(np.float64)
    return locs, y


def run(gu, ctx, locs, y, alphas, m=None, nb=256):
    from paper_2406_02701_amd import mpcr
    n = y.size
    dl, dy = gu.dev(locs), gu.dev(y)
    lp = np.zeros(alphas.size)
    post = np.zeros(alphas.size)
    its = (ctypes.c_int * alphas.size)()
    mode = torch.zeros(n, dtype=torch.float64, device="cuda")
    hm = None if m is None else gu.u8map(m)
    tm = None if m is None else ctypes.byref(mpcr.tilemap(n, nb, hm))
    a = np.ascontiguousarray(alphas)
    ctx.check(mpcr.mpcr_inla_posterior(ctx.ptr, n, dl.data_ptr(), dy.data_ptr(), 0.1, 0.5, 10.0, mpcr.f64p(a),
                                       a.size, 1e-12, 100, tm, mpcr.f64p(lp), mpcr.f64p(post), its,
                                       mode.data_ptr()))
    torch.cuda.synchronize()
    return lp, post, list(its), mode.cpu().numpy()


def test_inla_posterior_matches_oracle(g):
    gu, ctx = g
    n = 900
    locs, y = inla_data(n, 41)
    alphas = np.linspace(0.05, 0.95, 21)
    lp, post, its, mode = run(gu, ctx, locs, y, alphas)
    ref = [laplace.laplace_logpost(locs, y, 0.1, a, 0.5, 10.0) for a in alphas]
    lref = np.array([r["lpost"] for r in ref])
    print("INLA n=900: max rel dl", np.max(np.abs(lp - lref) / np.abs(lref)),
          "newton", its, [r["iters"] for r in ref], flush=True)
    np.testing.assert_allclose(lp, lref, rtol=1e-9)
    np.testing.assert_allclose(post, laplace.posterior(alphas, lref), rtol=0, atol=1e-8)
    assert its == [r["iters"] for r in ref]
    np.testing.assert_allclose(mode, ref[-1]["mode"], rtol=0, atol=1e-8)


def test_inla_mixed_b_tiles(g):
    """B = I + W^1/2 Sigma W^1/2 has eigenvalues >= 1: with FP32 off-diagonal
    tiles (unrefined solves) the Newton iteration still converges and the
    posterior of the range agrees with the FP64 one to FP32's level."""
    gu, ctx = g
    n, nb = 2500, 256
    locs, y = inla_data(n, 42)
    alphas = np.linspace(0.05, 0.95, 21)
    lp64, post64, _, _ = run(gu, ctx, locs, y, alphas)
    m = tiled.tilemap_banded(n, nb, ((0, "fp64"), (None, "fp32")))
    lp32, post32, _, _ = run(gu, ctx, locs, y, alphas, m=m, nb=nb)
    print("INLA n=2500 FP32 B tiles: max |dl|", np.max(np.abs(lp32 - lp64)),
          "max |dpost|", np.max(np.abs(post32 - post64)), flush=True)
    assert np.max(np.abs(lp32 - lp64)) <= 1e-4 * np.max(np.abs(lp64))
    assert np.max(np.abs(post32 - post64)) <= 1e-3 * np.max(post64)
