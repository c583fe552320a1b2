"""GPU tests at the full sizes of the 32768-site and 65536-site workloads,
through the C-ABI.

* The 32768-site workload (Matern 3/2, 512 x 512 tiles, 16 responses) against
  oracle-written expected values (tests/golden/mixed_n32768.json): the FP64
  path's log-likelihoods, log-determinant and sampled factor entries; the band
  map's breakdown step; the norm-guarded map (bit-exact, decided from the
  library's own tile maxima); the mixed path's refined quadratic forms and the
  log-determinant of its factor against the emulated mixed factor's.
* Exponential covariance on a regular 1-D grid is the KMS matrix, whose
  log-likelihood has an O(n) closed form at any n: the FP64 map and the
  65536-site band map (FP64 for d <= 1, FP32 for 2 <= d <= 4, FP16 beyond)
  are checked against it for all 256 right-hand sides.  With the range of 8
  grid steps the tiles beyond the first band hold values below every low
  format's range (this pins the FP64 path and the schedule at n = 65536; the
  low-precision kernels at nb = 1024 are compared elementwise with the
  emulation in test_gpu_parity_tiles.py).
* The Matern 5/2 recipe of the 65536-site workload: its band map (FP16 from
  distance 5, FP8 with per-tile scales from 16) makes the stored matrix
  indefinite (NOT_SPD), like the BF16 band at 32768 sites.  The norm-guarded map with the 32768-site guard (0.01 nugget)
  is not usable on this smoother, larger covariance: the FP32-stored tiles'
  perturbation summed over a row of Sigma reaches its smallest eigenvalue, so
  the factorisation breaks down, or its refinement stalls, or it moves the
  log-determinant by more than 1e-6 (which one depends on rounding details); with 1e-4 nugget (1651 FP64 / 429 FP32
  tiles) it factors, refines to eta <= 1e-13 and agrees with the all-FP64
  path (log-likelihood 1e-8, log-determinant 1e-6: the mixed factor's
  log-determinant is not refinable).
"""
import ctypes
import json
import math
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import synth  # noqa: E402
from oracle import covariance as cov  # noqa: E402
from oracle import tiled  # noqa: E402
from tests.test_oracle_dense import kms_loglik_closed_form  # noqa: E402
from tests.test_gpu_tile import _loglik  # noqa: E402

W = synth.WORKLOADS["mixed_n65536"]
W3 = synth.WORKLOADS["mixed_n32768"]
GOLD32768 = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "mixed_n32768.json")


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
    st_loose, _, d_loose = _loglik(gu, ctx, locs, z, th, nb, loose, order=1, opts=opts)
    print("loose guard:", st_loose, d_loose.info, d_loose.logdet, flush=True)
    assert st_loose in (mpcr.MPCR_OK, mpcr.MPCR_ERR_NOT_SPD, mpcr.MPCR_ERR_NOT_CONVERGED)
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
    # the loose guard is not usable here: its stored FP32 tiles either make the
    # matrix indefinite (a pivot fails, which rounding details decide) or move
    # the log-determinant far beyond the tight guard's
    if st_loose == mpcr.MPCR_ERR_NOT_SPD:
        assert d_loose.info > 0
    elif st_loose == mpcr.MPCR_OK:
        assert abs(d_loose.logdet - d64.logdet) > 1e-6 * abs(d64.logdet)


def _map_string(m):
    nt = m.shape[0]
    return "".join(str(int(m[i, j])) for i in range(nt) for j in range(i + 1))


def _gold32768():
    assert os.path.exists(GOLD32768), "tests/golden/mixed_n32768.json is missing (make_golden.py n32768)"
    return json.load(open(GOLD32768))


def _inputs32768(gu):
    n, nrhs = W3["n"], W3["nrhs"]
    locs = synth.locations(n, W3["seed_locs"])
    z = synth.normal_rhs(n, nrhs, W3["seed_z"])
    th = gu.theta(W3["sigma2"], W3["range"], W3["nu"], W3["nugget"])
    return locs, z, th


def test_n32768_fp64_path_matches_oracle_golden(g):
    """FP64 map: l, log|Sigma| and z^T Sigma^-1 z of all 16 responses against
    the oracle's FP64 tile factor, and 460 sampled factor entries.  Sigma's
    eigenvalues lie in [nugget, ||Sigma||_inf], so cond(L) <= sqrt(||Sigma||_inf
    / nugget) (about 4e4 here): factor entries agree to 4 n u cond(L); the
    log-likelihood, whose error is the quadratic form's forward error cond(L) n u
    relative, to 1e-9."""
    from paper_2406_02701_amd import mpcr
    gu, ctx = g
    gold = _gold32768()
    n, nb = W3["n"], W3["nb"]
    locs, z, th = _inputs32768(gu)
    perm = cov.morton_order(locs)
    assert perm[:32].tolist() == gold["perm_head"]
    m = tiled.tilemap_uniform(n, nb)
    st, ll, d = _loglik(gu, ctx, locs, z, th, nb, m, order=1)
    ctx.check(st)
    ref = np.array(gold["fp64"]["loglik"])
    assert np.max(np.abs(ll - ref) / np.abs(ref)) <= 1e-9
    assert abs(d.logdet - gold["fp64"]["logdet"]) <= 1e-9 * abs(gold["fp64"]["logdet"])
    assert abs(d.quad0 - gold["fp64"]["quad"][0]) <= 1e-9 * abs(gold["fp64"]["quad"][0])
    # sampled factor entries of the same factorisation
    dls = gu.dev(locs[perm])
    hm = gu.u8map(m)
    tm = mpcr.tilemap(n, nb, hm)
    f = ctypes.c_void_p()
    info = ctypes.c_int64(-1)
    ctx.check(mpcr.mpcr_potrf_tiled_covariance(ctx.ptr, n, dls.data_ptr(), ctypes.byref(th), ctypes.byref(tm),
                                               ctypes.byref(f), ctypes.byref(info)))
    dL = gu.empty(n, n)
    ctx.check(mpcr.mpcr_factor_to_dense(ctx.ptr, f, dL.data_ptr(), n))
    smp = np.array(gold["fp64"]["L_samples"])
    ii = torch.from_numpy(smp[:, 0].astype(np.int64)).cuda()
    jj = torch.from_numpy(smp[:, 1].astype(np.int64)).cuda()
    got = dL[jj, ii].cpu().numpy()       # column-major buffer: element (i, j) at [j][i]
    torch.cuda.synchronize()
    del dL
    mpcr.mpcr_factor_destroy(f)
    cond_l = math.sqrt(gold["sigma_inf"] / W3["nugget"])
    tol = 4 * n * 2.0 ** -53 * cond_l
    err = np.max(np.abs(got - smp[:, 2]))
    print(f"n32768 FP64: max |dl|/|l| {np.max(np.abs(ll - ref) / np.abs(ref)):.2e}, max |dL| {err:.2e} "
          f"(gate {tol:.2e})", flush=True)
    assert err <= tol


def test_n32768_guarded_mixed_path_matches_oracle_golden(g):
    """The band map breaks down in the oracle's tile step; the norm-guarded map
    is the oracle's, bit for bit; the mixed path refines every quadratic form
    to the FP64 one (eta <= 1e-13: 1e-9 relative at this conditioning).  The
    log-determinant is not refinable: the emulated mixed factor (tile
    roundings, exact accumulation) moves it by d_emu from the FP64 value; the
    GPU's FP32 tiles also accumulate their 512-term updates in FP32 (about
    sqrt(512) u32 per update where the emulation has u32), so its shift is
    gated at 10 |d_emu|, and both shifts at 1e-6 of the log-determinant."""
    from paper_2406_02701_amd import mpcr
    gu, ctx = g
    gold = _gold32768()
    n, nb = W3["n"], W3["nb"]
    locs, z, th = _inputs32768(gu)
    banded = tiled.tilemap_banded(n, nb, W3["bands"])
    opts = mpcr.mpcr_refine_opts_t(1e-13, 100, 0, 20, 0)
    st, _, d = _loglik(gu, ctx, locs, z, th, nb, banded, order=1, opts=opts)
    assert st == mpcr.MPCR_ERR_NOT_SPD
    print(f"n32768 band map: info {d.info} (oracle {gold['band_map_info']})", flush=True)
    assert (d.info - 1) // nb == (gold["band_map_info"] - 1) // nb
    gm = gu.guarded_map(ctx, locs, th, n, nb, banded, 0.01 * W3["nugget"])
    assert _map_string(gm) == gold["guarded"]["map"]
    st, ll, d = _loglik(gu, ctx, locs, z, th, nb, gm, order=1, opts=opts)
    ctx.check(st)
    assert d.converged == 1 and d.eta <= 1e-13
    q64 = gold["fp64"]["quad"][0]
    assert abs(d.quad0 - q64) <= 1e-9 * abs(q64)
    ld_emu, ld64 = gold["guarded"]["logdet"], gold["fp64"]["logdet"]
    print(f"n32768 mixed: logdet {d.logdet!r} emulated {ld_emu!r} fp64 {ld64!r}; "
          f"l vs fp64 {np.max(np.abs(ll - np.array(gold['fp64']['loglik'])) / np.abs(ll)):.2e}", flush=True)
    assert abs(d.logdet - ld64) <= 10 * abs(ld_emu - ld64)
    assert max(abs(d.logdet - ld64), abs(ld_emu - ld64)) <= 1e-6 * abs(ld64)
