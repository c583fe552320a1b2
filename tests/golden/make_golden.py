"""Writes the stored expected values under tests/golden/ from the oracle only.

    python tests/golden/make_golden.py            # fp64_n1024.json (seconds)
    python tests/golden/make_golden.py n32768     # mixed_n32768.json (about an hour, ~30 GB RAM)

fp64_n1024.json: the plain FP64 log-likelihood of the 1024-site exponential
workload (variance 1, range 0.1, nugget 1e-8, sites in Morton order, one N(0,1)
response), with a sample of factor entries and solution values.

mixed_n32768.json: the 32768-site Matern 3/2 workload (variance 1, range 0.05,
nugget 1e-6, sites in Morton order, 16 N(0,1) responses, 512 x 512 tiles):
* ||Sigma||_inf (with the nugget as a lower bound of Sigma's eigenvalues it
  bounds the condition number);
* the FP64 tile factor's log-determinant, the quadratic forms ||L^{-1} z||^2
  and log-likelihoods of all 16 responses, and a sample of factor entries;
* the band map (d <= 2 FP64, 3..8 FP32, beyond BF16) as given, with the
  column at which its emulated factorisation breaks down;
* the same map under the norm guard (a tile keeps its band format only if
  rounding it costs at most 0.01 * nugget), its tile counts, and the
  log-determinant of its emulated mixed factor.
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import synth  # noqa: E402
from oracle import covariance as cov  # noqa: E402
from oracle import dense, loglik, tiled  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def fp64_n1024():
    w = synth.WORKLOADS["fp64_n1024"]
    locs = synth.locations(w["n"], w["seed_locs"])
    z = synth.normal_rhs(w["n"], w["nrhs"], w["seed_z"])
    lo, zo, perm = loglik.order_sites(locs, z)
    r = loglik.loglik_plain(lo, zo, w["sigma2"], w["range"], w["nu"], w["nugget"])
    g = np.random.default_rng(99)
    idx = sorted({(int(i), int(j)) for i, j in g.integers(0, w["n"], (200, 2)) if i >= j})
    return dict(workload="fp64_n1024", perm_head=perm[:32].tolist(),
                logdet=r["logdet"], quad=r["quad"].tolist(), loglik=r["loglik"].tolist(),
                L_samples=[[i, j, r["L"][i, j]] for i, j in idx],
                x_head=r["X"][:32, 0].tolist())


def _log(msg, t0):
    print(f"[{time.time() - t0:8.1f} s] {msg}", flush=True)


def map_string(m: np.ndarray) -> str:
    """Lower triangle of a tile map, row by row, one digit (the format code) per tile."""
    nt = m.shape[0]
    return "".join(str(int(m[i, j])) for i in range(nt) for j in range(i + 1))


def mixed_n32768():
    t0 = time.time()
    w = synth.WORKLOADS["mixed_n32768"]
    n, nb, nrhs = w["n"], w["nb"], w["nrhs"]
    th = (w["sigma2"], w["range"], w["nu"], w["nugget"])
    locs = synth.locations(n, w["seed_locs"])
    z = synth.normal_rhs(n, nrhs, w["seed_z"])
    lo, zo, perm = loglik.order_sites(locs, z)
    # Sigma by blocks of rows (the oracle's covariance_block; the full-matrix
    # distance temporaries would need ~40 GB)
    S = np.empty((n, n))
    for r0 in range(0, n, 2048):
        S[r0:r0 + 2048] = cov.covariance_block(lo[r0:r0 + 2048], lo, *th, diag_offset=r0)
    _log("covariance", t0)
    out = dict(workload="mixed_n32768", n=n, nb=nb, nrhs=nrhs, perm_head=perm[:32].tolist(),
               sigma_inf=float(np.max(np.sum(np.abs(S), axis=1))))

    # FP64 tile path
    fac = tiled.tile_cholesky_emulated(S, nb, tiled.tilemap_uniform(n, nb))
    assert fac["info"] == 0
    L = fac["L"]
    del fac
    _log("fp64 tile factor", t0)
    logdet = dense.logdet_from_cholesky(L)
    W = dense.forward_substitution(L, zo)
    quad = np.array([dense.neumaier_sum(W[:, c] * W[:, c]) for c in range(nrhs)])
    _log("fp64 forward solve", t0)
    g = np.random.default_rng(2024)
    idx = sorted({(int(i), int(j)) for i, j in g.integers(0, n, (400, 2)) if i >= j})
    diag_idx = sorted({int(i) for i in g.integers(0, n, 64)})
    out.update(fp64=dict(logdet=logdet, quad=quad.tolist(), loglik=dense.gaussian_loglik(n, logdet, quad).tolist(),
                         L_samples=[[i, j, float(L[i, j])] for i, j in idx] +
                                   [[i, i, float(L[i, i])] for i in diag_idx]))
    del L, W

    # band map as given, then under the norm guard
    banded = tiled.tilemap_banded(n, nb, w["bands"])
    lit = tiled.tile_cholesky_emulated(S, nb, banded)
    out["band_map_info"] = int(lit["info"])
    del lit
    _log(f"band map: info {out['band_map_info']}", t0)
    amax = tiled.tile_amax(S, nb)
    guard = 0.01 * w["nugget"]
    gm = tiled.tilemap_guarded(banded, amax, guard)
    low = gm[np.tril_indices(gm.shape[0])]
    mix = tiled.tile_cholesky_emulated(S, nb, gm)
    assert mix["info"] == 0
    ld_mix = dense.logdet_from_cholesky(mix["L"][:n, :n])
    _log("guarded mixed factor", t0)
    out.update(guarded=dict(guard=guard, map=map_string(gm),
                            tiles={str(c): int(np.sum(low == c)) for c in range(5) if np.any(low == c)},
                            logdet=ld_mix))
    return out


if __name__ == "__main__":
    which = sys.argv[1] if len(sys.argv) > 1 else "n1024"
    name, fn = {"n1024": ("fp64_n1024.json", fp64_n1024), "n32768": ("mixed_n32768.json", mixed_n32768)}[which]
    data = fn()
    path = os.path.join(HERE, name)
    with open(path, "w") as f:
        json.dump(data, f, indent=1)
    print("wrote", path)
