"""GPU parity of the refinement solvers (PCG, GMRES-based iterative
refinement, block PCG) against the oracle's refine module, through the C-ABI.

Preconditioner and matrix are chosen so that both sides apply the same
operators up to FP64 rounding: Sigma is a Matern 3/2 covariance (range 0.05,
nugget 1e-4) on 1500 sites (tile size 256, a ragged last tile) and the
preconditioner is the all-FP64 tile factor of the covariance with range 0.045,
so that the solvers need several iterations (about 9 for PCG).  Gates: every
column reaches eta <= 1e-13 (recomputed on the host), the solution equals the
oracle's to 1e-9 of its largest entry, and the iteration counts agree to one
(a column's eta can land on either side of the tolerance through rounding).
Block PCG runs with one group of 20 columns and with groups of 8, 8 and 4.
A mixed-precision log-likelihood refined by each solver matches the plain
FP64 oracle.
"""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import synth  # noqa: E402
from oracle import covariance as cov  # noqa: E402
from oracle import dense, loglik, refine, tiled  # noqa: E402
from tests.test_gpu_tile import _factor_dense, _loglik  # noqa: E402


@pytest.fixture(scope="module")
def g():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from tests import gpu_util
    ctx = gpu_util.Ctx()
    yield gpu_util, ctx
    ctx.close()


N, NB, NRHS = 1500, 256, 20


@pytest.fixture(scope="module")
def problem():
    locs = synth.locations(N, 95)
    locs = locs[cov.morton_order(locs)]
    S = np.asfortranarray(cov.covariance(locs, 1.0, 0.05, 1.5, 1e-4))
    M = np.asfortranarray(cov.covariance(locs, 1.0, 0.045, 1.5, 1e-4))
    B = synth.normal_rhs(N, NRHS, 96)
    L = dense.cholesky_lower(M)
    return locs, S, M, B, L


CASES = {"pcg": (0, {}), "ir_gmres": (2, {}), "ir_gmres_m4": (2, dict(gmres_m=4)),
         "block_pcg": (3, {}), "block_pcg_8": (3, dict(block_size=8))}


@pytest.mark.parametrize("case", list(CASES))
def test_refinement_solvers_match_oracle(g, problem, case):
    from paper_2406_02701_amd import mpcr
    gu, ctx = g
    locs, S, M, B, L = problem
    solver, extra = CASES[case]
    f, _ = _factor_dense(gu, ctx, M, NB, tiled.tilemap_uniform(N, NB))
    opts = mpcr.mpcr_refine_opts_t(1e-13, 200, solver, 20, 0)
    for k, v in extra.items():
        setattr(opts, k, v)
    dS, dB, dX = gu.dev(S), gu.dev(B), gu.empty(N, NRHS)
    diag = mpcr.mpcr_diag_t()
    ctx.check(mpcr.mpcr_potrs(ctx.ptr, f, NRHS, dB.data_ptr(), N, dX.data_ptr(), N, dS.data_ptr(), N,
                              ctypes.byref(opts), ctypes.byref(diag)))
    X = gu.host(dX, (N, NRHS))
    mpcr.mpcr_factor_destroy(f)
    sig_inf = np.max(np.sum(np.abs(S), axis=1))
    pre = lambda R: dense.cholesky_solve(L, R)
    mv = lambda Y: S @ Y
    if solver == 0:
        ref = refine.pcg(mv, B, pre, sig_inf, tol=1e-13, max_iter=200)
    elif solver == 2:
        ref = refine.gmres_ir(mv, B, pre, sig_inf, tol=1e-13, max_iter=200, m=extra.get("gmres_m", 20))
    else:
        ref = refine.block_pcg(mv, B, pre, sig_inf, tol=1e-13, max_iter=200, block=extra.get("block_size", 32))
        assert not ref["fallback"]
    R = B - S @ X
    eta = np.max(np.abs(R), axis=0) / (sig_inf * np.max(np.abs(X), axis=0) + np.max(np.abs(B), axis=0))
    print(f"{case}: GPU iters {diag.iters} eta {diag.eta:.2e} (host {eta.max():.2e}); oracle iters {ref['iters']}; "
          f"max |dX| {np.abs(X - ref['X']).max():.2e}", flush=True)
    assert diag.converged == 1 and diag.eta <= 1e-13 and eta.max() <= 2e-13
    assert abs(diag.iters - ref["iters"]) <= 1
    np.testing.assert_allclose(X, ref["X"], rtol=0, atol=1e-9 * np.abs(ref["X"]).max())


@pytest.mark.parametrize("solver", [2, 3])
def test_mixed_loglik_with_krylov_solvers(g, solver):
    """The refined quadratic forms equal the FP64 ones; the log-likelihood
    differs from the FP64 one only by the log-determinant of the mixed factor
    (not refinable)."""
    from paper_2406_02701_amd import mpcr
    gu, ctx = g
    n, nb = 2000, 256
    locs = synth.locations(n, 97)
    z = synth.normal_rhs(n, 3, 98)
    th = gu.theta(1.0, 0.05, 1.5, 1e-4)
    m = tiled.tilemap_banded(n, nb, ((1, "fp64"), (None, "fp32")))
    opts = mpcr.mpcr_refine_opts_t(1e-13, 100, solver, 20, 0)
    st, ll, d = _loglik(gu, ctx, locs, z, th, nb, m, opts=opts)
    ctx.check(st)
    lo, zo, _ = loglik.order_sites(locs, z)
    ref = loglik.loglik_plain(lo, zo, 1.0, 0.05, 1.5, 1e-4)
    quad = -2.0 * (ll + 0.5 * n * np.log(2 * np.pi) + 0.5 * d.logdet)
    print(f"solver {solver}: iters {d.iters} eta {d.eta:.2e} max rel dquad "
          f"{np.max(np.abs(quad - ref['quad']) / ref['quad']):.2e}", flush=True)
    assert d.converged == 1 and d.eta <= 1e-13
    assert abs(d.quad0 - ref["quad"][0]) <= 1e-9 * ref["quad"][0]
    np.testing.assert_allclose(quad, ref["quad"], rtol=1e-9)
    assert abs(d.logdet - ref["logdet"]) <= 1e-5 * abs(ref["logdet"])


def test_bad_solver_options_are_rejected(g):
    from paper_2406_02701_amd import mpcr
    gu, ctx = g
    n, nb = 300, 128
    locs = synth.locations(n, 99)
    z = synth.normal_rhs(n, 1, 100)
    th = gu.theta(1.0, 0.1, 0.5, 1e-6)
    for bad in (dict(solver=4), dict(solver=2, gmres_m=65), dict(solver=3, block_size=33),
                dict(solver=2, gmres_inner_tol=1.5)):
        opts = mpcr.mpcr_refine_opts_t(1e-12, 10, 0, 20, 0)
        for k, v in bad.items():
            setattr(opts, k, v)
        st, _, _ = _loglik(gu, ctx, locs, z, th, nb, None, opts=opts)
        assert st == mpcr.MPCR_ERR_ARG, bad
