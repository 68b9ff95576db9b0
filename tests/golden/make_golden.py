"""Writes the stored expected values under tests/golden/.

Every value here comes from the FP64 oracle package (``oracle/``) or its
brute-force module on seeded inputs from ``workloads``; nothing is taken from
the GPU library.

  tiny_optima.json   exact optima of problem nsw (Section 2) for three tiny
                     instances, found by brute force with a Frank-Wolfe
                     certificate (oracle/brute.py).
  c2_trajectory.json Algorithm 1 on the 2000 x 100 x 10 low-rank workload
                     (eps 0.02, T 200, N 100, Adam lr 0.1 eps) run by the
                     FP64 oracle: F_0..F_N and the final impacts.  Takes a
                     few minutes on 8 cores.

Usage:  python tests/golden/make_golden.py [tiny] [c2]
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import workloads as W  # noqa: E402
from oracle import brute  # noqa: E402


def tiny():
    out = []
    rng = np.random.default_rng(2024)
    # T1: U=2, I=2, m=2
    r = rng.uniform(0.1, 1.0, (2, 2))
    e = np.array([1.0])
    F, X = brute.optimum_t1(r, e)
    F2, X2, gap = brute.optimum_vertex_weights(r, e, 2, lam0=X[:, :, 0])
    out.append(dict(name="T1", U=2, I=2, m=2, r=r.tolist(), e=e.tolist(), F_star=max(F, F2),
                    F_grid=F, fw_gap=gap, tol_gap=1e-4))
    # T2: U=2, I=3, m=2
    r = rng.uniform(0.1, 1.0, (2, 3))
    F, X = brute.optimum_t2(r, e)
    F2, X2, gap = brute.optimum_vertex_weights(r, e, 2, lam0=X[:, :, 0])
    out.append(dict(name="T2", U=2, I=3, m=2, r=r.tolist(), e=e.tolist(), F_star=max(F, F2),
                    F_grid=F, fw_gap=gap, tol_gap=1e-3))
    # T3: U=2, I=3, m=3 (Birkhoff polytope)
    r = rng.uniform(0.1, 1.0, (2, 3))
    e3 = W.exposure(3).astype(np.float64)
    F, X, gap = brute.optimum_birkhoff(r, e3)
    out.append(dict(name="T3", U=2, I=3, m=3, r=r.tolist(), e=e3.tolist(), F_star=F,
                    F_grid=None, fw_gap=gap, tol_gap=1e-4))
    doc = {"source": "oracle/brute.py: grid search and exponentiated-gradient ascent over the "
                     "vertices of the feasible set of problem nsw (Section 2, Eqs. dsm1-dsm4, "
                     "Imp, objF); certified by the Frank-Wolfe gap (F concave in X).",
           "instances": out}
    with open(os.path.join(HERE, "tiny_optima.json"), "w") as fh:
        json.dump(doc, fh, indent=1)
    for o in out:
        print(o["name"], o["F_star"], o["fw_gap"])


def c2():
    inst = W.config("C2")
    t0 = time.time()
    res = oracle.solve(inst.r, inst.e, float(inst.eps), inst.T, inst.N, lr=float(inst.lr))
    dt = time.time() - t0
    doc = {"source": "oracle.solve (FP64 Algorithm 1, Adam lr = 0.1 eps, C0 = 0) on "
                     "workloads.config('C2'): U=2000, I=100, m=10, low-rank-16 sigmoid "
                     "relevance, seed 2, eps=0.02 (float32-rounded), T=200, N=100.",
           "seconds": dt, "threads": oracle.num_threads(),
           "F_hist": res["F_hist"].tolist(), "imp_final": res["imp"].tolist(),
           "C_final_sample_idx": [], "C_final_sample": []}
    rng = np.random.default_rng(77)
    idx = [int(x) for x in rng.choice(res["C"].size, 64, replace=False)]
    doc["C_final_sample_idx"] = idx
    doc["C_final_sample"] = [float(res["C"].ravel()[j]) for j in idx]
    with open(os.path.join(HERE, "c2_trajectory.json"), "w") as fh:
        json.dump(doc, fh, indent=1)
    print("c2", dt, res["F_hist"][0], res["F_hist"][-1])


if __name__ == "__main__":
    which = sys.argv[1:] or ["tiny"]
    if "tiny" in which:
        tiny()
    if "c2" in which:
        c2()
