"""Benchmark: mixed-precision tile Cholesky + solve + Gaussian log-likelihood.

Workload (the mixed-precision tile Cholesky configuration): n = 32768 sites
drawn uniformly in the unit square, Matern nu = 3/2 covariance (variance 1,
range 0.05, nugget 1e-6), tiles nb = 512, 16 N(0,1) observation vectors,
FP64 refinement (PCG, GMRES-IR or block PCG) to a normwise backward error
below the 1e-9 bar (default 1e-13, so that the quadratic forms match the FP64
path), and the log-likelihood.

One step = one mpcr_gauss_loglik call: Morton ordering, covariance
generation into the tile formats, the tile factorisation, log-determinant,
refined solve and the log-likelihood, all on the GPU with inputs resident in
HBM.  `value` is the algorithmic rate (n^3/3 + 2 n^2 nrhs) / step time of the
mixed path; the all-FP64 path (the paper's evaluation: forward solve and
||L^-1 z||^2, no refinement) is timed the same way for the speed-up.

Precision map: the band map (FP64 for tile distance d <= 2, FP32 for
3 <= d <= 8, BF16 beyond) breaks down on this covariance (the BF16-stored
far tiles make the matrix indefinite); the library reports NOT_SPD for it
and the bench records that outcome.  The map study promotes the same band
map tile by tile by norm guards u_p * max|Sigma_tile| <= g * nugget for
several g and reports, per guard and refinement solver, the time, the
log-determinant and log-likelihood errors against the FP64 path, and the
same with refinement (PCG) stopped at the bar alone.  The headline is the
fastest (guard, solver) pair whose log-likelihoods match the FP64 path to
1e-6; the fastest guard that only holds the bar is reported beside it.

Further lines: the 1024-site FP64 workload and the 65536-site workload
(256 RHS), the multi-format GEMM sweep, the serving loop (capacity and a
Poisson load sweep) and the oracle's FP64 tile path on a bounded sample of
the workload on the host's cores.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import synth  # noqa: E402

PEAK_TFLOPS = {0: 78.6, 1: 157.3, 2: 2516.6, 3: 2516.6, 4: 5033.2}
FMT_NAME = {0: "fp64", 1: "fp32", 2: "fp16", 3: "bf16", 4: "fp8_e4m3"}
KIND_NAME = {0: "tile_update_fp64", 1: "tile_update_fp32", 2: "tile_update_fp16", 3: "tile_update_bf16",
             4: "tile_update_fp8", 5: "potrf_fp64", 6: "trsm_fp64", 7: "trtri_diag_fp64", 8: "tile_solve_sweeps",
             9: "residual_fp64", 10: "syrk_next_diag_fp64"}
NKIND = 11


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=None, help="override the order (smaller runs)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-n", type=int, default=4096)
    ap.add_argument("--no-gemm", action="store_true", help="skip the multi-format GEMM sweep")
    ap.add_argument("--gemm-only", action="store_true",
                    help="run only the multi-format GEMM sweep (for counter collection) and print its results")
    ap.add_argument("--no-other", action="store_true", help="skip the 1024- and 65536-site workloads")
    ap.add_argument("--no-n65536", action="store_true", help="skip the 65536-site workload")
    ap.add_argument("--guard-n65536", type=float, default=1e-4,
                    help="norm guard of the 65536-site map, as a multiple of the nugget")
    ap.add_argument("--serve-count", type=int, default=4096, help="serving requests (0 = skip the serving leg)")
    ap.add_argument("--serve-only", action="store_true", help="run only the serving leg and print its results")
    ap.add_argument("--serve-slots", type=int, default=16)
    ap.add_argument("--serve-queues", type=int, default=16,
                    help="HIP hardware queues of the serving process (GPU_MAX_HW_QUEUES; the serving leg runs in a "
                         "child process with this setting so that every slot's streams get queues of their own; "
                         "0 = run it in this process)")
    ap.add_argument("--serve-budget-gb", type=float, default=64.0)
    ap.add_argument("--guard", type=float, default=0.01,
                    help="fallback guard of the headline map (used if no map of the study matches), as a multiple "
                         "of the nugget: a tile keeps its band format p only if u_p max|Sigma_tile| <= guard * nugget")
    ap.add_argument("--study-guards", type=float, nargs="*", default=[0.003, 0.01, 0.02, 0.03, 0.1, 0.3, 1.0],
                    help="guards (multiples of the nugget) of the map study")
    ap.add_argument("--study-solvers", nargs="*", default=["pcg", "gmres", "bpcg"],
                    choices=["pcg", "ir", "gmres", "bpcg"],
                    help="refinement solvers timed for every map of the study (PCG, classical IR, GMRES-IR, "
                         "block PCG)")
    ap.add_argument("--loglik-match", type=float, default=1e-6,
                    help="headline map: the fastest of the study whose log-likelihoods match the FP64 path to this "
                         "relative error")
    ap.add_argument("--residual", type=int, default=1,
                    help="refinement residual: 0 = regenerate Sigma from the sites, 1 = stream a stored FP64 copy")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="copy a buffer of this many MiB once before the timed steps (a plain copy of known size "
                         "that scales hardware byte counters)")
    ap.add_argument("--fp32-split", type=int, default=1, choices=[0, 1],
                    help="FP32 tile updates: 1 = products from a three-way BF16 split on the BF16 MFMA, 0 = FP32 MFMA")
    ap.add_argument("--tol", type=float, default=1e-13,
                    help="refinement stopping rule: normwise backward error per column (the metric's bar is 1e-9; "
                         "the tighter default makes the quadratic forms match the FP64 path on this covariance)")
    return ap.parse_args()


class Lib:
    def __init__(self, torch):
        from paper_2406_02701_amd import mpcr
        self.m = mpcr
        self.torch = torch

    def ctx(self, fp32_split=1):
        c = ctypes.c_void_p()
        s = self.torch.cuda.current_stream().cuda_stream
        self.m.check(self.m.mpcr_ctx_create(0, ctypes.c_void_p(s), ctypes.byref(c)))
        self.m.check(self.m.mpcr_ctx_set_fp32_split(c, fp32_split), c)
        return c

    def loglik(self, ctx, n, dl, dz, nrhs, th, hmap, nb, opts):
        out = np.zeros(nrhs)
        diag = self.m.mpcr_diag_t()
        tm = self.m.tilemap(n, nb, hmap)
        st = self.m.mpcr_gauss_loglik(ctx, n, dl.data_ptr(), dz.data_ptr(), nrhs, ctypes.byref(th),
                                      ctypes.byref(tm), 1, None if opts is None else ctypes.byref(opts),
                                      self.m.f64p(out), ctypes.byref(diag))
        return st, out, diag

    def stats(self, ctx, kind):
        ms, n, fl = ctypes.c_double(), ctypes.c_int64(), ctypes.c_double()
        self.m.check(self.m.mpcr_ctx_kernel_stats(ctx, kind, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(fl)))
        return ms.value, n.value, fl.value


SOLVER_CODE = {"pcg": 0, "ir": 1, "gmres": 2, "bpcg": 3}
SOLVER_NAME = {"pcg": "pcg", "ir": "iterative refinement", "gmres": "GMRES-IR", "bpcg": "block pcg"}


def serving_leg(lib, args):
    """The serving results, from a child process started with
    GPU_MAX_HW_QUEUES = args.serve_queues (HIP reads it at start-up; with its
    default of 4 queues the slots' streams share in-order queues and wait on
    each other), or from this process when args.serve_queues is 0."""
    if args.serve_queues <= 0:
        return serving_bench(lib, args.serve_count, args.serve_slots, args.serve_budget_gb)
    import subprocess
    env = dict(os.environ, GPU_MAX_HW_QUEUES=str(args.serve_queues))
    cmd = [sys.executable, os.path.abspath(__file__), "--serve-only", "--serve-count", str(args.serve_count),
           "--serve-slots", str(args.serve_slots), "--serve-budget-gb", str(args.serve_budget_gb)]
    r = subprocess.run(cmd, env=env, capture_output=True, text=True)
    if r.returncode != 0:
        return {"error": f"serving child exited with {r.returncode}", "stderr_tail": r.stderr[-2000:]}
    out = json.loads(r.stdout.strip().splitlines()[-1])["serving"]
    out["hw_queues"] = args.serve_queues
    return out


def measured_traffic(kind, guard):
    """HBM bytes per launch of `kind` under the nugget guard `guard` from the
    committed counter summary (scaled FETCH_SIZE + WRITE_SIZE), or None when
    the summary has no such entry or the kernel source has changed since the
    counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "tile_update_n32768_traffic.md")
    if not os.path.exists(path):
        return None
    rec = dict(l.split(": ", 1) for l in open(path).read().splitlines() if ": " in l and not l.startswith(("|", "#")))
    src = os.path.join(ROOT, "paper_2406_02701_amd", "csrc", "factor.hip")
    if hashlib.sha256(open(src, "rb").read()).hexdigest() != rec.get("kernel_source_sha256", "").strip():
        return None
    v = rec.get(f"traffic_bytes_per_launch[{kind}@{guard:g}]")
    return None if v is None else float(v)


def banded(mp, n, nb, dmax, precs):
    nt = (n + nb - 1) // nb
    out = np.zeros((nt, nt), np.uint8)
    st = mp.mpcr_tilemap_banded(n, nb, (ctypes.c_int * len(dmax))(*dmax), (ctypes.c_int * len(precs))(*precs),
                                len(dmax), out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)))
    mp.check(st)
    return out


def timed_steps(lib, ctx, args, call):
    torch = lib.torch
    for _ in range(args.warmup):
        st, out, diag = call()
        lib.m.check(st, ctx)
    lib.m.mpcr_ctx_reset_stats(ctx)
    lib.m.mpcr_ctx_set_profiling(ctx, 1)
    torch.cuda.synchronize()
    region = [time.monotonic_ns(), 0]
    t0 = time.perf_counter()
    for _ in range(args.steps):
        st, out, diag = call()
        lib.m.check(st, ctx)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    region[1] = time.monotonic_ns()
    lib.m.mpcr_ctx_set_profiling(ctx, 0)
    timed_steps.last_region = region  # CLOCK_MONOTONIC ns (to match kernel traces)
    return dt, out, diag


def cpu_baseline(w, n_cpu):
    """The oracle's FP64 tile path (the tile Cholesky with all tiles FP64 at the
    workload's tile size, forward solve and log-likelihood of all responses) on
    the first n_cpu sites of the same recipe: a bounded sample of the
    workload, reported at the same algorithmic rate (n^3/3 + 2 n^2 nrhs)/time."""
    from threadpoolctl import threadpool_info

    from oracle import covariance as cov
    from oracle import dense, loglik, tiled
    locs = synth.locations(w["n"], w["seed_locs"])[:n_cpu]
    z = synth.normal_rhs(w["n"], w["nrhs"], w["seed_z"])[:n_cpu]
    lo, zo, _ = loglik.order_sites(locs, z)
    nb = w["nb"]
    t0 = time.perf_counter()
    S = cov.covariance(lo, w["sigma2"], w["range"], w["nu"], w["nugget"])
    L = tiled.tile_cholesky_emulated(S, nb, tiled.tilemap_uniform(n_cpu, nb))["L"][:n_cpu, :n_cpu]
    W = dense.forward_substitution(L, zo)
    logdet = dense.logdet_from_cholesky(L)
    dense.gaussian_loglik(n_cpu, logdet, np.sum(W * W, axis=0))
    dt = time.perf_counter() - t0
    flops = n_cpu ** 3 / 3 + 2 * n_cpu ** 2 * w["nrhs"]
    threads = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    return {"value": flops / dt / 1e12, "unit": "TFLOP/s", "cores": threads, "kind": "oracle",
            "sample": f"oracle FP64 tile path (tiles {nb} x {nb}, covariance, tile Cholesky, forward solve, "
                      f"log-likelihood) on the first {n_cpu} sites of the workload ({w['nrhs']} RHS), {dt:.1f} s"}


def gemm_sweep(lib, torch, steps):
    """C = A B with m = n = k = 8192, U(-1,1) entries, in every format; rate and
    error against the FP64 product of the same inputs."""
    mp = lib.m
    w = synth.WORKLOADS["gemm_8192"]
    N = w["m"]
    ctx = lib.ctx()
    A = synth.uniform_matrix(N, N, w["seed"])
    B = synth.uniform_matrix(N, N, w["seed"] + 1000)
    dA = torch.from_numpy(np.ascontiguousarray(A.T)).cuda()
    dB = torch.from_numpy(np.ascontiguousarray(B.T)).cuda()
    del A, B
    tdt = {0: torch.float64, 1: torch.float32, 2: torch.int16, 3: torch.int16, 4: torch.uint8}
    out, ref = {}, None
    for p in (0, 1, 2, 3, 4):
        qa = torch.empty((N, N), dtype=tdt[p], device="cuda")
        qb = torch.empty((N, N), dtype=tdt[p], device="cuda")
        sa = sb = None
        if p == 4:
            sa = torch.zeros((N // 128, N // 128), dtype=torch.int8, device="cuda")
            sb = torch.zeros((N // 128, N // 128), dtype=torch.int8, device="cuda")
        mp.check(mp.mpcr_convert(ctx, p, N, N, dA.data_ptr(), N, qa.data_ptr(), N,
                                 None if sa is None else sa.data_ptr()), ctx)
        mp.check(mp.mpcr_convert(ctx, p, N, N, dB.data_ptr(), N, qb.data_ptr(), N,
                                 None if sb is None else sb.data_ptr()), ctx)
        cp = 0 if p == 0 else 1
        C = torch.empty((N, N), dtype=torch.float64 if cp == 0 else torch.float32, device="cuda")

        def call():
            mp.check(mp.mpcr_gemm(ctx, p, 0, 0, N, N, N, 1.0, qa.data_ptr(), N, None if sa is None else sa.data_ptr(),
                                  qb.data_ptr(), N, None if sb is None else sb.data_ptr(), 0.0, C.data_ptr(), N, cp),
                     ctx)
        call()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            call()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        Cd = C.to(torch.float64)
        if p == 0:
            ref = Cd.clone()
        rel_f = (torch.linalg.norm(Cd - ref) / torch.linalg.norm(ref)).item()
        rel_max = (torch.max(torch.abs(Cd - ref)) / torch.max(torch.abs(ref))).item()
        out[FMT_NAME[p]] = {"ms": ms, "tflops": 2.0 * N ** 3 / (ms * 1e-3) / 1e12,
                            "frac_of_peak": 2.0 * N ** 3 / (ms * 1e-3) / 1e12 / PEAK_TFLOPS[p],
                            "rel_frobenius_err_vs_fp64": rel_f, "max_abs_err_over_max_vs_fp64": rel_max}
        del qa, qb, C, Cd
    mp.mpcr_ctx_destroy(ctx)
    return out


def serving_bench(lib, count, slots, budget_gb, seed=6):
    """Log-likelihood requests with n log-uniform in [256, 8192] and their own
    parameters (variance U(0.5,2), range U(0.02,0.3), nu in {1/2, 3/2, 5/2},
    nugget 1e-6), one observation vector each.  The closed-loop capacity
    (solves/s) is the median of three runs that submit all requests at once;
    Poisson arrivals are then replayed at 0.5, 0.8 and 1.0 x that capacity,
    each reporting the latency (done - arrival) percentiles and whether the
    served rate kept up with the offered one."""
    mp = lib.m
    w = synth.WORKLOADS["serve_4096"]
    reqs = synth.serving_requests(count, seed, w["n_lo"], w["n_hi"])
    arrays = []
    for r in reqs:
        locs, z = synth.request_arrays(r)
        arrays.append((np.asfortranarray(locs), np.ascontiguousarray(z[:, 0]),
                       mp.mpcr_theta_t(r["sigma2"], r["range"], r["nu"], r["nugget"])))
    opts = mp.mpcr_serve_opts_t(w["nb"], 1, 4, mp.MPCR_BF16, 0.01, mp.mpcr_refine_opts_t(1e-13, 100, 0, 20, 0, 1), 1)

    def run(arrival):
        srv = ctypes.c_void_p()
        mp.check(mp.mpcr_serve_create(0, int(budget_gb * (1 << 30)), slots, ctypes.byref(opts), ctypes.byref(srv)))
        t_base = mp.mpcr_serve_clock(srv)
        res, nsub, rejected = {}, 0, 0
        rid, ll, st, fb = ctypes.c_uint64(), ctypes.c_double(), ctypes.c_int(), ctypes.c_int()
        ts, td = ctypes.c_double(), ctypes.c_double()
        dg = mp.mpcr_diag_t()

        def poll_all():
            while mp.mpcr_serve_poll(srv, ctypes.byref(rid), ctypes.byref(ll), ctypes.byref(dg), ctypes.byref(ts),
                                     ctypes.byref(td), ctypes.byref(st), ctypes.byref(fb)) == 1:
                res[rid.value] = (ts.value, td.value, st.value, fb.value, ll.value, dg.promotions)
        while nsub < count:
            now = mp.mpcr_serve_clock(srv) - t_base
            while nsub < count and arrival[nsub] <= now:
                locs, z, th = arrays[nsub]
                rc = mp.mpcr_serve_submit(srv, nsub, reqs[nsub]["n"], mp.f64p(locs), mp.f64p(z), ctypes.byref(th))
                rejected += rc == mp.MPCR_ERR_REJECTED
                nsub += 1
            poll_all()
            time.sleep(0.0002)
        while len(res) + rejected < count:
            poll_all()
            time.sleep(0.0005)
        t_end = max(v[1] for v in res.values()) - t_base
        mp.mpcr_serve_destroy(srv)
        lat = np.array([v[1] - (t_base + arrival[k]) for k, v in res.items()])
        ok = sum(1 for v in res.values() if v[2] == 0)
        return dict(wall_s=t_end, solves_per_s=ok / t_end, completed_ok=ok, rejected=rejected,
                    failed=len(res) - ok, fallback_fp64=sum(v[3] for v in res.values()),
                    promoted=sum(1 for v in res.values() if v[5] > 0),
                    p50_ms=float(np.percentile(lat, 50) * 1e3), p99_ms=float(np.percentile(lat, 99) * 1e3),
                    mean_ms=float(lat.mean() * 1e3))

    # capacity: median of three closed-loop runs (all requests submitted at once)
    cap_runs = [run(np.zeros(count)) for _ in range(3)]
    caps = sorted(r["solves_per_s"] for r in cap_runs)
    capacity = caps[1]
    legs = []
    for frac in (0.5, 0.8, 1.0):
        qps = frac * capacity
        gaps = synth.rng(seed + 100).exponential(1.0 / qps, size=count)
        leg = run(np.cumsum(gaps) - gaps[0])
        leg.update(offered_fraction_of_capacity=frac, offered_qps=qps,
                   sustained=bool(leg["solves_per_s"] >= 0.97 * qps))
        legs.append(leg)
    flops = sum(r["n"] ** 3 / 3 + 2 * r["n"] ** 2 for r in reqs)
    return {"requests": count, "slots": slots, "hbm_budget_gb": budget_gb, "nb": w["nb"],
            "map": "band d<=1 fp64 / 2-4 fp32 / rest bf16, norm-guarded 0.01 nugget, promote on breakdown, "
                   "fp64 fallback",
            "capacity_solves_per_s": capacity, "closed_loop_runs_solves_per_s": caps,
            "closed_loop": cap_runs[[r["solves_per_s"] for r in cap_runs].index(capacity)],
            "closed_loop_tflops": flops / (count / capacity) / 1e12,
            "poisson_legs": legs}


def other_configs(lib, torch, args):
    """The FP64 1024-site workload and the 65536-site workload, timed as extra
    lines beside the headline (same step definition: one mpcr_gauss_loglik
    call with inputs resident in HBM)."""
    mp = lib.m
    out = {}
    sub = argparse.Namespace(warmup=2, steps=20)
    w = synth.WORKLOADS["fp64_n1024"]
    n, nb = w["n"], w["nb"]
    locs = synth.locations(n, w["seed_locs"])
    z = synth.normal_rhs(n, w["nrhs"], w["seed_z"])
    dl = torch.from_numpy(np.ascontiguousarray(locs.T)).cuda()
    dz = torch.from_numpy(np.ascontiguousarray(z.T)).cuda()
    th = mp.mpcr_theta_t(w["sigma2"], w["range"], w["nu"], w["nugget"])
    ctx = lib.ctx()
    fmap = banded(mp, n, nb, [-1], [0])
    opts64 = mp.mpcr_refine_opts_t(1e-9, 0, 0, 20, 0, 0, 0)
    t, ll, d = timed_steps(lib, ctx, sub, lambda: lib.loglik(ctx, n, dl, dz, 1, th, fmap, nb, opts64))
    fl = n ** 3 / 3 + 2 * n ** 2
    out["fp64_n1024"] = {"ms_per_step": t * 1e3, "tflops": fl / t / 1e12, "loglik": float(ll[0]),
                         "steps": sub.steps}
    mp.mpcr_ctx_destroy(ctx)
    if args.no_n65536:
        return out
    w = synth.WORKLOADS["mixed_n65536"]
    n, nb, nrhs = w["n"], w["nb"], w["nrhs"]
    sub = argparse.Namespace(warmup=1, steps=1)
    locs = synth.locations(n, w["seed_locs"])
    z = synth.normal_rhs(n, nrhs, w["seed_z"])
    dl = torch.from_numpy(np.ascontiguousarray(locs.T)).cuda()
    dz = torch.from_numpy(np.ascontiguousarray(z.T)).cuda()
    th = mp.mpcr_theta_t(w["sigma2"], w["range"], w["nu"], w["nugget"])
    ctx = lib.ctx()
    perm = torch.zeros(n, dtype=torch.int64, device="cuda")
    mp.check(mp.mpcr_morton_order(ctx, n, dl.data_ptr(), perm.data_ptr()), ctx)
    dls = torch.from_numpy(np.ascontiguousarray(locs[perm.cpu().numpy()].T)).cuda()
    start = banded(mp, n, nb, [1, 4, -1], [0, 1, 2])
    nt = start.shape[0]
    amax = np.zeros((nt, nt))
    mp.check(mp.mpcr_covariance_tile_amax(ctx, n, nb, dls.data_ptr(), ctypes.byref(th), mp.f64p(amax)), ctx)
    guard = args.guard_n65536 * w["nugget"]
    gmap = np.zeros_like(start)
    mp.check(mp.mpcr_tilemap_guarded(n, nb, start.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), mp.f64p(amax),
                                     guard, gmap.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))))
    fmap = banded(mp, n, nb, [-1], [0])
    opts = mp.mpcr_refine_opts_t(args.tol, 100, 0, 20, args.residual, 1, 0)
    t_mix, ll_mix, d_mix = timed_steps(lib, ctx, sub, lambda: lib.loglik(ctx, n, dl, dz, nrhs, th, gmap, nb, opts))
    ctx64 = lib.ctx()
    opts64 = mp.mpcr_refine_opts_t(1e-9, 0, 0, 20, 0, 0, 0)
    t_64, ll_64, d_64 = timed_steps(lib, ctx64, sub, lambda: lib.loglik(ctx64, n, dl, dz, nrhs, th, fmap, nb,
                                                                         opts64))
    fl = n ** 3 / 3 + 2 * n ** 2 * nrhs
    tri = gmap[np.tril_indices(nt)]
    out["mixed_n65536"] = {
        "mixed": {"ms_per_step": t_mix * 1e3, "tflops": fl / t_mix / 1e12, "iters": d_mix.iters,
                  "eta": d_mix.eta, "promotions": d_mix.promotions, "t_factor_ms": d_mix.t_factor_ms,
                  "t_solve_refine_ms": d_mix.t_solve_ms + d_mix.t_refine_ms,
                  "tiles_by_format": {FMT_NAME[p]: int(np.sum(tri == p)) for p in range(5) if np.any(tri == p)},
                  "map": f"band d<=1 fp64 / 2-4 fp32 / rest fp16, norm-guarded {args.guard_n65536:g} nugget",
                  "logdet_rel_err_vs_fp64": abs(d_mix.logdet - d_64.logdet) / abs(d_64.logdet),
                  "loglik_rel_err_vs_fp64": float(np.max(np.abs(ll_mix - ll_64) / np.abs(ll_64)))},
        "fp64_path": {"ms_per_step": t_64 * 1e3, "tflops": fl / t_64 / 1e12, "t_factor_ms": d_64.t_factor_ms,
                      "t_solve_ms": d_64.t_solve_ms},
        "speedup_vs_fp64": t_64 / t_mix, "nrhs": nrhs, "steps": sub.steps}
    mp.mpcr_ctx_destroy(ctx)
    mp.mpcr_ctx_destroy(ctx64)
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 "
                                   "(the multi-GPU sharding is described, not built)"}))
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench needs a GPU"
    torch.cuda.set_device(0)
    lib = Lib(torch)
    mp = lib.m
    if args.gemm_only:
        print(json.dumps({"gemm_sweep_8192": gemm_sweep(lib, torch, args.steps)}), flush=True)
        return
    if args.serve_only:
        print(json.dumps({"serving": serving_bench(lib, args.serve_count, args.serve_slots, args.serve_budget_gb)}),
              flush=True)
        return
    w = dict(synth.WORKLOADS["mixed_n32768"])
    if args.n:
        w["n"] = args.n
    n, nb, nrhs = w["n"], w["nb"], w["nrhs"]
    locs = synth.locations(n, w["seed_locs"])
    z = synth.normal_rhs(n, nrhs, w["seed_z"])
    dl = torch.from_numpy(np.ascontiguousarray(locs.T)).cuda()
    dz = torch.from_numpy(np.ascontiguousarray(z.T)).cuda()
    th = mp.mpcr_theta_t(w["sigma2"], w["range"], w["nu"], w["nugget"])
    opts = mp.mpcr_refine_opts_t(args.tol, 100, 0, 20, args.residual)
    flops = n ** 3 / 3 + 2 * n ** 2 * nrhs

    if args.calib_copy_mib > 0:
        src = torch.empty(args.calib_copy_mib << 20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # maps: literal band map, its norm-guarded version, and all-FP64
    lit = banded(mp, n, nb, [2, 8, -1], [0, 1, 3])
    ctx_m = lib.ctx(args.fp32_split)
    # the guard needs max|Sigma| per tile of the Morton-ordered covariance
    perm = torch.zeros(n, dtype=torch.int64, device="cuda")
    mp.check(mp.mpcr_morton_order(ctx_m, n, dl.data_ptr(), perm.data_ptr()), ctx_m)
    dl_sorted = torch.from_numpy(np.ascontiguousarray(locs[perm.cpu().numpy()].T)).cuda()
    nt = lit.shape[0]
    amax = np.zeros((nt, nt))
    mp.check(mp.mpcr_covariance_tile_amax(ctx_m, n, nb, dl_sorted.data_ptr(), ctypes.byref(th), mp.f64p(amax)), ctx_m)
    guarded = np.zeros_like(lit)
    mp.check(mp.mpcr_tilemap_guarded(n, nb, lit.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), mp.f64p(amax),
                                     args.guard * w["nugget"], guarded.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))))
    fp64map = banded(mp, n, nb, [-1], [0])

    # literal band map outcome (untimed)
    st, _, dlit = lib.loglik(ctx_m, n, dl, dz, nrhs, th, lit, nb, opts)
    literal = {"status": mp.STATUS_NAMES.get(st, st), "info": int(dlit.info)}

    # all-FP64 path (paper's evaluation: forward solve quad), timed on its own
    # context (opts max_iter = 0: no refinement; direct_eta = 0: the backward
    # error of the direct solve, an extra FP64 residual pass, is taken once
    # untimed)
    ctx_d = lib.ctx()
    opts64 = mp.mpcr_refine_opts_t(1e-9, 0, 0, 20, 0, 0, 0)
    t_64, ll_64, d_64 = timed_steps(lib, ctx_d, args, lambda: lib.loglik(ctx_d, n, dl, dz, nrhs, th, fp64map, nb,
                                                                         opts64))
    region64 = timed_steps.last_region
    kstats64 = {k: lib.stats(ctx_d, k) for k in range(NKIND)}
    st, _, d_64eta = lib.loglik(ctx_d, n, dl, dz, nrhs, th, fp64map, nb, None)
    mp.check(st, ctx_d)
    ideal64 = sum(d_64.flops_by_prec) / (PEAK_TFLOPS[0] * 1e12)

    def fmt_peak(p):
        """MFMA ceiling of the algorithmic rate of updates in format p (FP32
        tiles with the BF16 split: the BF16 peak over its six products)."""
        return PEAK_TFLOPS[3] / 6 if (p == 1 and args.fp32_split) else PEAK_TFLOPS[p]

    def guarded_map(gmul):
        out = np.zeros_like(lit)
        mp.check(mp.mpcr_tilemap_guarded(n, nb, lit.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), mp.f64p(amax),
                                         gmul * w["nugget"], out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))))
        return out

    def tiles_of(m):
        tri = m[np.tril_indices(nt)]
        return {FMT_NAME[p]: int(np.sum(tri == p)) for p in range(5) if np.any(tri == p)}

    # map study: the band map under norm guards of increasing size, each
    # refined to eta <= tol (1e-13: the quadratic forms then carry FP64
    # accuracy) and once to the bar alone (eta <= 1e-9), whose quadratic forms
    # are far from the FP64 ones on this covariance (cond ~ 1e8)
    study = []
    opts_bar = mp.mpcr_refine_opts_t(1e-9, 100, 0, 20, args.residual)

    def solver_opts(name):
        o = mp.mpcr_refine_opts_t(args.tol, 100, SOLVER_CODE[name], 20, args.residual)
        return o

    for gmul in args.study_guards:
        gm_ = guarded_map(gmul)
        st, ll, d = lib.loglik(ctx_m, n, dl, dz, nrhs, th, gm_, nb, opts)
        rec = {"guard_x_nugget": gmul, "tiles": tiles_of(gm_), "status": mp.STATUS_NAMES.get(st, st),
               "info": int(d.info)}
        if st == mp.MPCR_OK and d.converged:
            fl_by = list(d.flops_by_prec)
            ideal = sum(fl_by[p] / (fmt_peak(p) * 1e12) for p in range(5))
            rec.update(ideal_ms_at_mfma_peak=ideal * 1e3, ideal_speedup=ideal64 / ideal,
                       logdet_err_vs_fp64=d.logdet - d_64.logdet, by_solver={})
            for sname in args.study_solvers:
                so = solver_opts(sname)
                st, ll, d = lib.loglik(ctx_m, n, dl, dz, nrhs, th, gm_, nb, so)      # untimed first call
                if st != mp.MPCR_OK or not d.converged:
                    rec["by_solver"][sname] = {"status": mp.STATUS_NAMES.get(st, st), "converged": bool(d.converged)}
                    continue
                t, ll, d = timed_steps(lib, ctx_m, argparse.Namespace(warmup=0, steps=2),
                                       lambda: lib.loglik(ctx_m, n, dl, dz, nrhs, th, gm_, nb, so))
                rec["by_solver"][sname] = {
                    "ms_per_step": t * 1e3, "speedup_vs_fp64": t_64 / t, "iters": d.iters, "eta": d.eta,
                    "t_solve_ms": d.t_solve_ms,
                    "loglik_rel_err_vs_fp64": float(np.max(np.abs(ll - ll_64) / np.abs(ll_64)))}
            done = {k: v for k, v in rec["by_solver"].items() if "ms_per_step" in v}
            if done:
                best = min(done, key=lambda k: done[k]["ms_per_step"])
                rec.update(solver=best, **{k: done[best][k] for k in ("ms_per_step", "speedup_vs_fp64", "iters",
                                                                      "eta", "loglik_rel_err_vs_fp64")})
            t9, ll9, d9 = timed_steps(lib, ctx_m, argparse.Namespace(warmup=0, steps=2),
                                      lambda: lib.loglik(ctx_m, n, dl, dz, nrhs, th, gm_, nb, opts_bar))
            rec["bar_only"] = {"tol": 1e-9, "ms_per_step": t9 * 1e3, "speedup_vs_fp64": t_64 / t9,
                               "iters": d9.iters, "eta": d9.eta, "rel_resid2": d9.rel_resid2,
                               "loglik_rel_err_vs_fp64": float(np.max(np.abs(ll9 - ll_64) / np.abs(ll_64)))}
        study.append(rec)
    # headline: the fastest (map, solver) pair of the study whose log-
    # likelihoods match the FP64 path to 1e-6 (the log-determinant is the part
    # refinement cannot fix)
    cands = [(r["guard_x_nugget"], sname, v["ms_per_step"]) for r in study for sname, v in r.get("by_solver", {}).items()
             if v.get("loglik_rel_err_vs_fp64", 1.0) <= args.loglik_match]
    head = min(cands, key=lambda c: c[2]) if cands else None
    head_gmul = head[0] if head else args.guard
    head_solver = head[1] if head else "pcg"
    head_map = guarded_map(head_gmul)
    opts = solver_opts(head_solver)
    guarded = guarded_map(args.guard)

    # headline, timed with kernel profiling
    t_mix, ll_mix, d_mix = timed_steps(lib, ctx_m, args, lambda: lib.loglik(ctx_m, n, dl, dz, nrhs, th, head_map,
                                                                          nb, opts))
    region_mix = timed_steps.last_region
    kstats = {k: lib.stats(ctx_m, k) for k in range(NKIND)}
    # the fastest map of the study that holds the bar alone (eta <= 1e-9),
    # whatever its log-likelihood error
    fast = min((r for r in study if "bar_only" in r), key=lambda r: r["bar_only"]["ms_per_step"], default=None)

    # dominant kernel of the mixed step (largest total time) and its roofline;
    # the tile updates, POTRF and TRSM are MFMA contractions (FP64 MFMA for the
    # latter two); the other kinds are reported against FP64 as well
    def roof(stats, kind, traffic):
        ms, launches, kfl = stats[kind]
        avg_ms = ms / max(launches, 1)
        fl_per_launch = kfl / max(launches, 1)
        achieved = fl_per_launch / (avg_ms * 1e-3) / 1e12 if avg_ms > 0 else 0.0
        peak = PEAK_TFLOPS[kind] if kind <= 4 else PEAK_TFLOPS[0]
        note = None
        if kind == 1 and args.fp32_split:
            # FP32 tiles updated on the BF16 MFMA with six products per FP32
            # product: the ceiling of the algorithmic FP32 rate is the BF16 peak / 6
            peak = PEAK_TFLOPS[3] / 6
            note = "FP32 products from a three-way BF16 split: BF16 MFMA peak 2516.6 / 6 products"
        bound = "mfma" if kind <= 7 or kind == 10 else "alu"
        out = {"bound": bound, "kernel": KIND_NAME[kind], "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
               "frac": achieved / peak, "traffic": traffic, "traffic_unit": "bytes per launch",
               "launches": launches, "avg_launch_ms": avg_ms, "flops_per_launch": fl_per_launch}
        if note:
            out["peak_note"] = note
        return out

    dom = max(range(NKIND), key=lambda k: kstats[k][0])
    roofline = roof(kstats, dom, measured_traffic(KIND_NAME[dom], head_gmul) if n == 32768 else None)
    # the trailing updates share the GPU with the next-column and POTRF/TRSM
    # streams, so a launch's duration includes some sharing; the FP64 path's
    # figure is given beside it
    roofline["overlap"] = ("launches share the GPU: FP64 and lower-format updates run on two concurrent streams, "
                           "beside the next-column update and POTRF/TRSM streams; a launch's duration includes that "
                           "sharing (profiles/mfma_utilisation_n32768.md has each kernel alone)")
    roofline_fp64_path = roof(kstats64, 0, None)

    fl_by = list(d_mix.flops_by_prec)
    tot = sum(fl_by)
    share = {FMT_NAME[p]: fl_by[p] / tot for p in range(5) if fl_by[p] > 0}
    ideal_s = sum(fl_by[p] / (fmt_peak(p) * 1e12) for p in range(5))

    line = {
        "metric": "tile-Cholesky+solve TFLOP/s mixed vs FP64 at <=1e-9 residual",
        "value": flops / t_mix / 1e12,
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_mix * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "mixed-f64/f32/bf16",
        "data": "synthetic",
        "config": {"workload": "mixed_n32768" if n == 32768 else f"mixed_n{n}", "n": n, "nb": nb, "nrhs": nrhs,
                   "nu": w["nu"], "sigma2": w["sigma2"], "range": w["range"], "nugget": w["nugget"],
                   "map": f"band d<=2 fp64 / 3-8 fp32 / >=9 bf16, norm-guarded (u_p max|tile| <= {head_gmul:g} "
                          f"nugget): the fastest guard of the map study whose log-likelihoods match the FP64 path "
                          f"to {args.loglik_match:g}",
                   "refine": f"{SOLVER_NAME[head_solver]}, normwise backward error <= {args.tol:g} (bar: 1e-9), "
                             f"{'stored FP64 tiles' if args.residual else 'matrix-free'} residual"},
        "fp64_path": {"value": flops / t_64 / 1e12, "ms_per_step": t_64 * 1e3,
                      "eta_untimed_check": d_64eta.eta, "rel_resid2_untimed_check": d_64eta.rel_resid2,
                      "logdet": d_64.logdet,
                      "t_factor_ms": d_64.t_factor_ms, "t_solve_ms": d_64.t_solve_ms,
                      "ideal_ms_at_mfma_peak": ideal64 * 1e3},
        "speedup_vs_fp64": t_64 / t_mix,
        "mixed": {"guard_x_nugget": head_gmul, "solver": head_solver, "eta": d_mix.eta, "rel_resid2": d_mix.rel_resid2,
                  "iters": d_mix.iters, "converged": bool(d_mix.converged), "logdet": d_mix.logdet,
                  "logdet_err_vs_fp64": d_mix.logdet - d_64.logdet,
                  "logdet_rel_err_vs_fp64": abs(d_mix.logdet - d_64.logdet) / abs(d_64.logdet),
                  "loglik_rel_err_vs_fp64": float(np.max(np.abs(ll_mix - ll_64) / np.abs(ll_64))),
                  "t_gen_ms": d_mix.t_gen_ms, "t_factor_ms": d_mix.t_factor_ms, "t_solve_ms": d_mix.t_solve_ms,
                  "t_refine_ms": d_mix.t_refine_ms, "flop_share": share, "ideal_ms_at_mfma_peak": ideal_s * 1e3,
                  "ideal_speedup_vs_fp64_ideal": ideal64 / ideal_s, "tiles_by_format": tiles_of(head_map)},
        "fastest_holding_bar_only": None if fast is None else
        {"guard_x_nugget": fast["guard_x_nugget"], **fast["bar_only"],
         "value": flops / (fast["bar_only"]["ms_per_step"] * 1e-3) / 1e12,
         "ideal_speedup": fast["ideal_speedup"], "logdet_err_vs_fp64": fast["logdet_err_vs_fp64"]},
        "map_study": study,
        "literal_band_map": literal,
        "kernels_mixed": {KIND_NAME[k]: {"ms_per_step": v[0] / args.steps, "launches_per_step": v[1] / args.steps,
                                         "tflops": (v[2] / (v[0] * 1e-3) / 1e12) if v[0] > 0 else 0.0}
                          for k, v in kstats.items() if v[1]},
        "kernels_fp64": {KIND_NAME[k]: {"ms_per_step": v[0] / args.steps, "launches_per_step": v[1] / args.steps,
                                        "tflops": (v[2] / (v[0] * 1e-3) / 1e12) if v[0] > 0 else 0.0}
                         for k, v in kstats64.items() if v[1]},
        "roofline": roofline,
        "roofline_fp64_path": roofline_fp64_path,
        "cpu_baseline": None,
        "timed_region_ns": {"mixed": region_mix, "fp64": region64},
    }
    mp.mpcr_ctx_destroy(ctx_m)
    mp.mpcr_ctx_destroy(ctx_d)
    if not args.no_other:
        line["other_configs"] = other_configs(lib, torch, args)
    if not args.no_gemm:
        line["gemm_sweep_8192"] = gemm_sweep(lib, torch, 3)
    if args.serve_count > 0:
        line["serving"] = serving_leg(lib, args)
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(w, min(args.cpu_n, n))
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
