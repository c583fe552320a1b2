"""GPU tests at the largest configuration (n = 65536 sites, nb = 1024,
256 right-hand sides), through the C-ABI.

* Exponential covariance on a regular 1-D grid is the KMS matrix, whose
  log-likelihood has an O(n) closed form at any n: the FP64 map and the
  65536-site band map (FP64 for d <= 1, FP32 for 2 <= d <= 4, FP16 beyond)
  are checked against it for all 256 right-hand sides.
* The Matern 5/2 recipe of the 65536-site workload: its band map (FP16 from
  distance 5, FP8 with per-tile scales from 16) makes the stored matrix
  indefinite (NOT_SPD), like the BF16 band at 32768 sites.  The norm-guarded map with the 32768-site guard (0.01 nugget)
  breaks down on this smoother, larger covariance (NOT_SPD: the FP32-stored
  tiles' perturbation summed over a row of Sigma exceeds its smallest
  eigenvalue), which is checked; with 1e-4 nugget (1651 FP64 / 429 FP32
  tiles) it factors, refines to eta <= 1e-13 and agrees with the all-FP64
  path (log-likelihood 1e-8, log-determinant 1e-6: the mixed factor's
  log-determinant is not refinable).
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import synth  # noqa: E402
from oracle import tiled  # noqa: E402
from tests.test_oracle_dense import kms_loglik_closed_form  # noqa: E402
from tests.test_gpu_tile import _loglik  # noqa: E402

W = synth.WORKLOADS["mixed_n65536"]


@pytest.fixture(scope="module")
def g():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from tests import gpu_util
    ctx = gpu_util.Ctx()
    yield gpu_util, ctx
    ctx.close()


@pytest.mark.parametrize("bands", [None, ((1, "fp64"), (4, "fp32"), (None, "fp16")),
                                   ((1, "fp64"), (4, "fp32"), (15, "fp16"), (None, "fp8_e4m3"))])
def test_kms_closed_form_n65536(g, bands):
    gu, ctx = g
    from paper_2406_02701_amd import mpcr
    n, nb, nrhs = W["n"], W["nb"], W["nrhs"]
    h, a = 1.0 / n, 8.0 / n
    locs = synth.grid_1d(n, h)
    z = synth.normal_rhs(n, nrhs, W["seed_z"])
    th = gu.theta(1.0, a, 0.5, 0.0)
    m = tiled.tilemap_uniform(n, nb) if bands is None else tiled.tilemap_banded(n, nb, bands)
    opts = None if bands is None else mpcr.mpcr_refine_opts_t(1e-14, 100, 0, 20, 0)
    st, ll, diag = _loglik(gu, ctx, locs, z, th, nb, m, order=0, opts=opts)
    ctx.check(st)
    rho = math.exp(-h / a)
    tol = 1e-11 if bands is None else 1e-6
    for c in range(nrhs):
        logdet, q, ref = kms_loglik_closed_form(z[:, c], 1.0, rho)
        assert abs(ll[c] - ref) <= tol * abs(ref), (c, ll[c], ref)
    if bands is None:
        assert abs(diag.logdet - logdet) <= 1e-11 * abs(logdet)


def test_matern52_n65536_guarded_matches_fp64(g):
    gu, ctx = g
    from paper_2406_02701_amd import mpcr
    n, nb, nrhs = W["n"], W["nb"], W["nrhs"]
    locs = synth.locations(n, W["seed_locs"])
    z = synth.normal_rhs(n, nrhs, W["seed_z"])
    th = gu.theta(W["sigma2"], W["range"], W["nu"], W["nugget"])
    lit = tiled.tilemap_banded(n, nb, ((1, "fp64"), (4, "fp32"), (15, "fp16"), (None, "fp8_e4m3")))
    opts = mpcr.mpcr_refine_opts_t(1e-13, 100, 0, 20, 1)
    st, _, d = _loglik(gu, ctx, locs, z, th, nb, lit, order=1, opts=opts)
    print("literal band map:", st, mpcr.mpcr_last_error(ctx.ptr), d.info, flush=True)
    assert st == mpcr.MPCR_ERR_NOT_SPD and d.info > 0
    # guarded: the band map with FP16 where it had FP8, promoted by the guard
    start = tiled.tilemap_banded(n, nb, ((1, "fp64"), (4, "fp32"), (None, "fp16")))
    loose = gu.guarded_map(ctx, locs, th, n, nb, start, 0.01 * W["nugget"])
    st, _, d = _loglik(gu, ctx, locs, z, th, nb, loose, order=1, opts=opts)
    assert st == mpcr.MPCR_ERR_NOT_SPD and d.info > 0
    guarded = gu.guarded_map(ctx, locs, th, n, nb, start, 1e-4 * W["nugget"])
    tri = guarded[np.tril_indices(guarded.shape[0])]
    print("guarded map tiles by format:", {f: int(np.sum(tri == f)) for f in range(5)}, flush=True)
    assert not np.any(tri == 4)
    st, ll, d = _loglik(gu, ctx, locs, z, th, nb, guarded, order=1, opts=opts)
    ctx.check(st)
    assert d.converged == 1 and d.eta <= 1e-13
    st, ll64, d64 = _loglik(gu, ctx, locs, z, th, nb, tiled.tilemap_uniform(n, nb), order=1)
    ctx.check(st)
    assert np.max(np.abs(ll - ll64) / np.abs(ll64)) <= 1e-8
    assert abs(d.logdet - d64.logdet) <= 1e-6 * abs(d64.logdet)
