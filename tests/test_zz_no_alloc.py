"""GPU test of the allocation-free ordering entry point (mpcr_morton_order_noalloc):
its permutation equals mpcr_morton_order's (and the oracle's) on two calls in
a row, the second with fewer sites, and sizes above its static key array are
rejected."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import synth  # noqa: E402
from oracle import covariance as cov  # noqa: E402


@pytest.fixture(scope="module")
def g():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from tests import gpu_util
    ctx = gpu_util.Ctx()
    yield gpu_util, ctx
    ctx.close()


def test_noalloc_order_matches_allocating_entry_point(g):
    from paper_2406_02701_amd import mpcr
    gu, ctx = g
    for n, seed in ((70000, 301), (3000, 302)):
        print(f"noalloc order: n {n}", flush=True)
        locs = synth.locations(n, seed)
        locs[10:20] = locs[5]        # ties keep input order
        dl = gu.dev(locs)
        p_alloc = torch.zeros(n, dtype=torch.int64, device="cuda")
        p_free = torch.full((n,), -1, dtype=torch.int64, device="cuda")
        ctx.check(mpcr.mpcr_morton_order(ctx.ptr, n, dl.data_ptr(), p_alloc.data_ptr()))
        ctx.check(mpcr.mpcr_morton_order_noalloc(ctx.ptr, n, dl.data_ptr(), p_free.data_ptr()))
        torch.cuda.synchronize()
        a, b = p_alloc.cpu().numpy(), p_free.cpu().numpy()
        assert np.array_equal(a, b)
        assert np.array_equal(b, cov.morton_order(locs))


def test_noalloc_order_rejects_sizes_above_its_array(g):
    from paper_2406_02701_amd import mpcr
    gu, ctx = g
    n = (1 << 20) + 1
    dl = torch.zeros((2, n), dtype=torch.float64, device="cuda")
    perm = torch.zeros(n, dtype=torch.int64, device="cuda")
    assert mpcr.mpcr_morton_order_noalloc(ctx.ptr, n, dl.data_ptr(), perm.data_ptr()) == mpcr.MPCR_ERR_ARG
