"""Writes the stored expected values under tests/golden/ from the oracle only.

    python tests/golden/make_golden.py

fp64_n1024.json: the plain FP64 log-likelihood of the 1024-site exponential
workload (variance 1, range 0.1, nugget 1e-8, sites in Morton order, one N(0,1)
response), with a sample of factor entries and solution values.
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import synth  # noqa: E402
from oracle import loglik  # noqa: E402


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


if __name__ == "__main__":
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "fp64_n1024.json")
    with open(out, "w") as f:
        json.dump(fp64_n1024(), f, indent=1)
    print("wrote", out)
