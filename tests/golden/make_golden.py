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
  c3_grad.npz        the 10000 x 300 x 20 gradient workload (eps 0.02, T 300)
                     at C = 0 and at C ~ N(0, (2 eps)^2): the oracle's
                     impacts and F, its reverse-mode dF/dC and dF/dr for 8
                     sampled consumers, and FP64 central differences
                     (h = 1e-4) at 64 cost and 64 relevance coordinates.

  c5_sub.npz         1000 consumers sampled (seed 55) from the 100000 x 1000 x 50
                     workload (eps 0.01, T 300): at C ~ N(0, (2 eps)^2) (seed 56)
                     the oracle's impacts and F of the sub-instance and the
                     plans of two of its consumers; and Algorithm 1 (Adam,
                     lr 0.1 eps) for 3 steps from C = 0: F_0..F_3.
  c5_traj.npz        the same sub-instance solved by Algorithm 1 for all 50
                     outer steps (Adam, lr 0.1 eps, T 300, C0 = 0): F_0..F_50
                     and the final impacts.  About an hour on 8 cores.
  c4_full.npz        eight instances of the 128-instance batched workload (the
                     four with the fewest plan cells and four drawn with seed
                     44 from the rest of those with at most 1e7 plan cells)
                     solved by Algorithm 1 at the configured
                     size (eps 0.03, T 200, N 50, Adam lr 0.1 eps): F_0..F_50
                     and the final impacts of each.

Usage:  python tests/golden/make_golden.py [tiny] [c2] [c3] [c5] [c5traj]
        python tests/golden/make_golden.py c4 [instance ...] [--out DIR]
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


def _consumer_y(r_u, e, C_u, eps, T):
    """y_i = r_ui sum_{k<m} e_k x_uik for one consumer (oracle forward)."""
    X = oracle.forward(C_u[None], eps, T)[0]
    m = X.shape[1]
    return r_u * (X[:, : m - 1] @ e)


def c3():
    inst = W.config("C3")
    U, I, m, T = inst.U, inst.I, inst.m, inst.T
    eps = float(inst.eps)
    r = inst.r.astype(np.float64)
    e = inst.e.astype(np.float64)
    rng = np.random.default_rng(34)
    users = np.sort(rng.choice(U, size=8, replace=False))
    cu = users[rng.integers(0, 8, 64)]
    ci = rng.integers(0, I, 64)
    ck = rng.integers(0, m, 64)
    ru = users[rng.integers(0, 8, 64)]
    ri = rng.integers(0, I, 64)
    h = 1e-4
    out = {"users": users, "c_u": cu, "c_i": ci, "c_k": ck, "r_u": ru, "r_i": ri, "h": h}
    for tag, C in (("zero", np.zeros((U, I, m), dtype=np.float32)),
                   ("rand", W.random_costs(U, I, m, 2 * eps, seed=33))):
        t0 = time.time()
        X = oracle.forward(C, eps, T)
        imp = oracle.impact(r, e, X)
        del X
        F = oracle.nsw(imp)
        gC, gr = oracle.grad(r[users], e, eps, T, C[users], imp=imp)
        fdC = np.empty(64)
        for j in range(64):
            u, i, k = int(cu[j]), int(ci[j]), int(ck[j])
            base = _consumer_y(r[u], e, C[u].astype(np.float64), eps, T)
            Cp = C[u].astype(np.float64)
            Cp[i, k] += h
            Cm = C[u].astype(np.float64)
            Cm[i, k] -= h
            dp = _consumer_y(r[u], e, Cp, eps, T) - base
            dm = _consumer_y(r[u], e, Cm, eps, T) - base
            fdC[j] = (np.sum(np.log1p(dp / imp)) - np.sum(np.log1p(dm / imp))) / (2 * h)
        fdr = np.empty(64)
        for j in range(64):
            u, i = int(ru[j]), int(ri[j])
            Xu = oracle.forward(C[u][None].astype(np.float64), eps, T)[0]
            s = float(Xu[i, : m - 1] @ e)
            fdr[j] = (np.log1p(h * s / imp[i]) - np.log1p(-h * s / imp[i])) / (2 * h)
        out[f"{tag}_imp"] = imp
        out[f"{tag}_F"] = np.array([F])
        out[f"{tag}_dC"] = gC.astype(np.float32)
        out[f"{tag}_dr"] = gr.astype(np.float32)
        out[f"{tag}_fdC"] = fdC
        out[f"{tag}_fdr"] = fdr
        print("c3", tag, time.time() - t0, F)
    np.savez_compressed(os.path.join(HERE, "c3_grad.npz"), **out)


def c5_subsample():
    """The 1000-consumer sub-instance of the precision-at-scale workload."""
    inst = W.config("C5")
    users = W.subsample_users(inst.U, 1000, seed=55)
    return inst, users, inst.r[users]


def c5():
    inst, users, r = c5_subsample()
    I, m, T = inst.I, inst.m, inst.T
    eps = float(inst.eps)
    rs = r.astype(np.float64)
    e = inst.e.astype(np.float64)
    t0 = time.time()
    C = W.random_costs(1000, I, m, 2 * eps, seed=56)
    X = oracle.forward(C, eps, T)
    imp = oracle.impact(rs, e, X)
    F = oracle.nsw(imp)
    X2 = X[[0, 777]].astype(np.float32)
    del X
    print("c5 forward", time.time() - t0, F, flush=True)
    res = oracle.solve(rs, e, eps, T, 3, lr=float(inst.lr))
    print("c5 solve", time.time() - t0, res["F_hist"], flush=True)
    np.savez_compressed(os.path.join(HERE, "c5_sub.npz"), users=users, rand_imp=imp,
                        rand_F=np.array([F]), rand_X_sel=X2, sel=np.array([0, 777]),
                        adam_F_hist=res["F_hist"], adam_imp=res["imp"])


def c5traj():
    inst, users, r = c5_subsample()
    eps = float(inst.eps)
    t0 = time.time()
    res = oracle.solve(r.astype(np.float64), inst.e.astype(np.float64), eps, inst.T, inst.N,
                       lr=float(inst.lr))
    dt = time.time() - t0
    print("c5traj", dt, res["F_hist"][0], res["F_hist"][-1], flush=True)
    np.savez_compressed(os.path.join(HERE, "c5_traj.npz"), users=users, F_hist=res["F_hist"],
                        imp_final=res["imp"], seconds=np.array([dt]),
                        threads=np.array([oracle.num_threads()]))


def _solve_in_chunks(r, e, eps, T, N, lr, tag, chunk=5):
    """oracle.solve for N outer steps, resumed every `chunk` steps (the
    oracle's resume is bitwise) so that progress is printed as it goes."""
    res = None
    F = []
    done = 0
    while done < N:
        n = min(chunk, N - done)
        if res is None:
            res = oracle.solve(r, e, eps, T, n, lr=lr)
        else:
            res = oracle.solve(r, e, eps, T, n, C0=res["C"], lr=lr, mom=res["mom"],
                               vel=res["vel"], start_step=done)
        F.extend(res["F_hist"][(0 if done == 0 else 1):].tolist())
        done += n
        print(f"  {tag}: {done}/{N} outer steps", flush=True)
    res["F_hist"] = np.array(F)
    return res


def c4_golden_instances():
    """Indices of the batched workload's instances with stored oracle solves:
    the four with the fewest plan cells and four drawn (seed 44) from the rest
    of those with at most 1e7 plan cells (an FP64 oracle solve of 50 outer
    steps of a larger one takes longer than a run may)."""
    shapes = W.batched_shapes(128, seed=4)
    cells = np.array([a * b * c for a, b, c in shapes])
    order = np.argsort(cells, kind="stable")
    small = [int(j) for j in order[:4]]
    rest = [int(j) for j in order[4:] if cells[j] <= 10_000_000]
    rng = np.random.default_rng(44)
    pick = sorted(int(j) for j in rng.choice(rest, 4, replace=False))
    return shapes, small + pick


def c4(only=None, out_dir=HERE):
    """Oracle solves of the stored batched instances; with ``only`` (instance
    indices) just those, merged into the file's existing entries.  The file is
    rewritten after every instance, so a cut-off run keeps what it finished."""
    shapes, idx = c4_golden_instances()
    path = os.path.join(out_dir, "c4_full.npz")
    out = {"idx": np.array(idx)}
    if os.path.exists(path):
        old = np.load(path)
        out.update({k: old[k] for k in old.files if k != "idx"})
    todo = [j for j in idx if only is None or j in only]
    for j in todo:
        x = W.batched_instance(j, shapes[j])
        t0 = time.time()
        res = _solve_in_chunks(x.r.astype(np.float64), x.e.astype(np.float64), float(x.eps),
                               x.T, x.N, float(x.lr), f"c4 instance {j} {shapes[j]}")
        dt = time.time() - t0
        print("c4", j, shapes[j], dt, res["F_hist"][-1], flush=True)
        out[f"F_hist_{j}"] = res["F_hist"]
        out[f"imp_{j}"] = res["imp"]
        out[f"seconds_{j}"] = np.array([dt])
        out[f"threads_{j}"] = np.array([oracle.num_threads()])
        np.savez_compressed(path, **out)


if __name__ == "__main__":
    which = sys.argv[1:] or ["tiny"]
    if "tiny" in which:
        tiny()
    if "c2" in which:
        c2()
    if "c3" in which:
        c3()
    if "c5" in which:
        c5()
    if "c5traj" in which:
        c5traj()
    if "c4" in which:
        # optional: c4 <j> <j> ... [--out DIR]
        rest = which[which.index("c4") + 1:]
        out_dir = HERE
        if "--out" in rest:
            out_dir = rest[rest.index("--out") + 1]
            rest = rest[:rest.index("--out")]
        only = [int(a) for a in rest if a.isdigit()] or None
        c4(only, out_dir)
