"""GPU tests of the serving engine (continuous batching of log-likelihood requests).

* Alone vs mix: every request's log-likelihood computed with the server running
  one request at a time equals, bitwise, the value computed while many requests
  of different n share the device (the arithmetic of a request does not depend
  on its co-runners).
* Admission: a request larger than the whole HBM budget is rejected at submit;
  with a budget that holds only a few requests at once, all requests still
  complete (they wait in the queue).
* Results agree with the FP64 oracle log-likelihood (mixed map refined to
  eta <= 1e-13; the factor's log-determinant carries the low tiles' error).
* Requests of 1600-3000 sites whose norm-guarded maps keep BF16 tiles at
  nb = 256: the quadratic form is the FP64 one and the served
  log-determinant lies within the emulated mixed factor's shift from the FP64
  log-determinant of the emulated value.
* Options the footprint estimate does not cover (the stored FP64 residual)
  are rejected at create.
"""
import ctypes
import time

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import synth  # noqa: E402
from oracle import covariance as cov  # noqa: E402
from oracle import loglik as olog  # noqa: E402
from oracle import tiled  # noqa: E402


@pytest.fixture(scope="module")
def mp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2406_02701_amd import mpcr
    return mpcr


def opts(mp, nb=256):
    return mp.mpcr_serve_opts_t(nb, 1, 4, mp.MPCR_BF16, 0.01, mp.mpcr_refine_opts_t(1e-13, 100, 0, 20, 0, 1), 1)


def requests(count, seed, n_lo, n_hi):
    reqs = synth.serving_requests(count, seed, n_lo, n_hi)
    out = []
    for r in reqs:
        locs, z = synth.request_arrays(r)
        out.append((r, np.asfortranarray(locs), np.ascontiguousarray(z[:, 0])))
    return out


def submit(mp, srv, rid, r, locs, z):
    th = mp.mpcr_theta_t(r["sigma2"], r["range"], r["nu"], r["nugget"])
    return mp.mpcr_serve_submit(srv, rid, r["n"], mp.f64p(locs), mp.f64p(z), ctypes.byref(th))


def drain(mp, srv, count, timeout=240.0):
    out = {}
    t0 = time.time()
    while len(out) < count:
        rid, ll, st, fb = ctypes.c_uint64(), ctypes.c_double(), ctypes.c_int(), ctypes.c_int()
        ts, td = ctypes.c_double(), ctypes.c_double()
        diag = mp.mpcr_diag_t()
        got = mp.mpcr_serve_poll(srv, ctypes.byref(rid), ctypes.byref(ll), ctypes.byref(diag), ctypes.byref(ts),
                                 ctypes.byref(td), ctypes.byref(st), ctypes.byref(fb))
        if got == 1:
            out[rid.value] = dict(ll=ll.value, status=st.value, fallback=fb.value, eta=diag.eta,
                                  t=(ts.value, td.value))
        else:
            assert time.time() - t0 < timeout, "serving drain timed out"
            time.sleep(0.002)
    return out


def make_server(mp, budget, slots):
    srv = ctypes.c_void_p()
    o = opts(mp)
    assert mp.mpcr_serve_create(0, budget, slots, ctypes.byref(o), ctypes.byref(srv)) == 0
    return srv


def test_alone_vs_mix_bitwise(mp):
    reqs = requests(24, 61, 256, 1500)
    srv = make_server(mp, 8 << 30, 1)
    alone = {}
    for i, (r, locs, z) in enumerate(reqs):
        assert submit(mp, srv, i, r, locs, z) == 0
        alone.update(drain(mp, srv, 1))
    mp.mpcr_serve_destroy(srv)
    srv = make_server(mp, 8 << 30, 6)
    for i, (r, locs, z) in enumerate(reqs):
        assert submit(mp, srv, i, r, locs, z) == 0
    mix = drain(mp, srv, len(reqs))
    mp.mpcr_serve_destroy(srv)
    for i in range(len(reqs)):
        assert alone[i]["status"] == 0 and mix[i]["status"] == 0, (alone[i], mix[i])
        assert alone[i]["ll"] == mix[i]["ll"], (i, alone[i]["ll"], mix[i]["ll"])
        assert alone[i]["fallback"] == mix[i]["fallback"]


def test_admission_and_rejection(mp):
    fp = mp.mpcr_serve_footprint(4096, 256)
    budget = int(2.5 * fp)
    srv = make_server(mp, budget, 4)
    big = requests(1, 62, 8000, 8192)[0]
    big[0]["n"] = 8192
    locs, z = synth.request_arrays(big[0])
    assert mp.mpcr_serve_submit is not None
    th = mp.mpcr_theta_t(1.0, 0.1, 1.5, 1e-6)
    locs = np.asfortranarray(locs)
    zz = np.ascontiguousarray(z[:, 0])
    assert mp.mpcr_serve_footprint(8192, 256) > budget
    assert mp.mpcr_serve_submit(srv, 999, 8192, mp.f64p(locs), mp.f64p(zz), ctypes.byref(th)) == mp.MPCR_ERR_REJECTED
    reqs = requests(10, 63, 2048, 4096)
    for i, (r, lo, zr) in enumerate(reqs):
        assert submit(mp, srv, i, r, lo, zr) == 0
    res = drain(mp, srv, len(reqs))
    q, run, fin, rej, byt = (ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64(),
                             ctypes.c_size_t())
    mp.mpcr_serve_stats(srv, ctypes.byref(q), ctypes.byref(run), ctypes.byref(fin), ctypes.byref(rej),
                        ctypes.byref(byt))
    mp.mpcr_serve_destroy(srv)
    assert rej.value == 1 and q.value == 0 and run.value == 0 and byt.value == 0
    assert all(v["status"] == 0 for v in res.values())


def test_serving_matches_oracle(mp):
    reqs = requests(6, 64, 256, 900)
    srv = make_server(mp, 4 << 30, 3)
    for i, (r, locs, z) in enumerate(reqs):
        assert submit(mp, srv, i, r, locs, z) == 0
    res = drain(mp, srv, len(reqs))
    mp.mpcr_serve_destroy(srv)
    for i, (r, locs, z) in enumerate(reqs):
        lo, zo, _ = olog.order_sites(locs, z[:, None])
        ref = olog.loglik_plain(lo, zo, r["sigma2"], r["range"], r["nu"], r["nugget"])["loglik"][0]
        assert res[i]["status"] == 0
        assert abs(res[i]["ll"] - ref) <= 1e-6 * abs(ref), (i, res[i]["ll"], ref, r)


def test_serving_bf16_tiles_match_emulation(mp):
    cases = [(2048, 0.02, 0.5, 701), (2048, 0.03, 1.5, 702), (3000, 0.02, 2.5, 703), (1600, 0.02, 0.5, 704)]
    srv = make_server(mp, 8 << 30, 4)
    data = []
    for i, (n, rng_, nu, seed) in enumerate(cases):
        locs = np.asfortranarray(synth.locations(n, seed))
        z = np.ascontiguousarray(synth.normal_rhs(n, 1, seed + 1000)[:, 0])
        r = dict(n=n, sigma2=1.0, range=rng_, nu=nu, nugget=1e-6)
        assert submit(mp, srv, i, r, locs, z) == 0
        data.append((r, locs, z))
    got = {}
    for _ in cases:
        rid, ll, st, fb = ctypes.c_uint64(), ctypes.c_double(), ctypes.c_int(), ctypes.c_int()
        diag = mp.mpcr_diag_t()
        t0 = time.time()
        while mp.mpcr_serve_poll(srv, ctypes.byref(rid), ctypes.byref(ll), ctypes.byref(diag), None, None,
                                 ctypes.byref(st), ctypes.byref(fb)) != 1:
            assert time.time() - t0 < 240
            time.sleep(0.002)
        got[rid.value] = (ll.value, st.value, fb.value, diag.logdet, diag.quad0, diag.promotions)
    mp.mpcr_serve_destroy(srv)
    for i, (r, locs, z) in enumerate(data):
        ll, st, fb, ld, q, promos = got[i]
        assert st == 0 and fb == 0 and promos == 0, got[i]
        lo, zo, _ = olog.order_sites(locs, z[:, None])
        S = cov.covariance(lo, 1.0, r["range"], r["nu"], 1e-6)
        banded = tiled.tilemap_banded(r["n"], 256, ((1, "fp64"), (4, "fp32"), (None, "bf16")))
        gm = tiled.tilemap_guarded(banded, tiled.tile_amax(S, 256), 0.01 * 1e-6)
        assert np.any(gm == mp.MPCR_BF16)
        emu = olog.loglik_mixed(lo, zo, 1.0, r["range"], r["nu"], 1e-6, 256, gm, tol=1e-13)
        plain = olog.loglik_plain(lo, zo, 1.0, r["range"], r["nu"], 1e-6)
        assert abs(q - plain["quad"][0]) <= 1e-9 * abs(plain["quad"][0])
        shift = abs(emu["logdet"] - plain["logdet"])
        print(f"request {i}: logdet {ld!r} emulated {emu['logdet']!r} fp64 {plain['logdet']!r}", flush=True)
        assert abs(ld - emu["logdet"]) <= max(shift, 1e-9 * abs(plain["logdet"]))


def test_serving_rejects_stored_residual(mp):
    srv = ctypes.c_void_p()
    o = opts(mp)
    o.refine.residual = 1
    assert mp.mpcr_serve_create(0, 1 << 30, 2, ctypes.byref(o), ctypes.byref(srv)) == mp.MPCR_ERR_ARG
