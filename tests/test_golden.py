"""Consistency of the stored expected values (all written by
tests/golden/make_golden.py from the oracle alone)."""
import json
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_c3_oracle_gradient_matches_its_central_differences():
    """At the 10000 x 300 x 20 workload the oracle's reverse-mode gradient
    agrees with FP64 central differences of F (h = 1e-4) on 64 cost and 64
    relevance coordinates, at C = 0 and at random C."""
    d = np.load(os.path.join(GOLDEN, "c3_grad.npz"))
    users = list(d["users"])
    for tag in ("zero", "rand"):
        dC = d[tag + "_dC"].astype(np.float64)
        dr = d[tag + "_dr"].astype(np.float64)
        g = np.array([dC[users.index(u), i, k] for u, i, k in zip(d["c_u"], d["c_i"], d["c_k"])])
        gr = np.array([dr[users.index(u), i] for u, i in zip(d["r_u"], d["r_i"])])
        assert np.max(np.abs(g - d[tag + "_fdC"])) <= 1e-5 * np.max(np.abs(dC))
        assert np.max(np.abs(gr - d[tag + "_fdr"])) <= 1e-5 * np.max(np.abs(dr))
        assert np.all(d[tag + "_imp"] > 0)


def test_c3_zero_cost_impacts_are_the_uniform_closed_form():
    """At C = 0 every plan is the uniform policy b_k / I."""
    import workloads as W
    from oracle import brute
    d = np.load(os.path.join(GOLDEN, "c3_grad.npz"))
    inst = W.config("C3")
    ref = brute.uniform_impacts(inst.r.astype(np.float64), inst.e.astype(np.float64), inst.I)
    assert np.max(np.abs(d["zero_imp"] / ref - 1)) < 1e-12


def test_c2_trajectory_is_an_ascent_from_the_uniform_policy():
    import workloads as W
    from oracle import brute
    with open(os.path.join(GOLDEN, "c2_trajectory.json")) as fh:
        g = json.load(fh)
    inst = W.config("C2")
    F0 = np.sum(np.log(brute.uniform_impacts(inst.r.astype(np.float64),
                                             inst.e.astype(np.float64), inst.I)))
    Fh = np.array(g["F_hist"])
    assert abs(Fh[0] - F0) < 1e-9 * abs(F0)
    assert len(Fh) == inst.N + 1 and Fh[-1] > Fh[0]


def test_c5_subsample_golden_is_an_ascent():
    d = np.load(os.path.join(GOLDEN, "c5_sub.npz"))
    Fh = d["adam_F_hist"]
    assert len(Fh) == 4 and np.all(np.diff(Fh) > 0)
    assert d["users"].shape == (1000,) and np.all(np.diff(d["users"]) > 0)
    X = d["rand_X_sel"].astype(np.float64)
    b = np.ones(50)
    b[-1] = 1000 - 50 + 1
    assert np.max(np.abs(X.sum(1) - b[None]) / b[None]) < 1e-6   # float32-stored columns
