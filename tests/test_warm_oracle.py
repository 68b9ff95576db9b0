"""Pins of the converged-map oracle (oracle/warm.py): warm-started Sinkhorn
and the implicit-function gradient."""
import numpy as np

import oracle
import workloads as W
from oracle import warm


def _inst(U=6, I=12, m=4, seed=3):
    inst = W.small_instance(U, I, m, seed=seed, eps=0.1, T=50)
    C = W.random_costs(U, I, m, 0.3, seed=seed + 1).astype(np.float64)
    return inst, C


def test_cold_start_without_tolerance_is_the_fixed_t_forward():
    inst, C = _inst()
    U, I, m = C.shape
    X, g, it = oracle.forward_warm(C, float(inst.eps), np.zeros((U, m)), 0.0, 37)
    assert np.all(it == 37)
    assert np.array_equal(X, oracle.forward(C, float(inst.eps), 37))


def test_converged_plan_does_not_depend_on_the_start():
    inst, C = _inst()
    U, I, m = C.shape
    rng = np.random.default_rng(9)
    X0, _, _ = oracle.forward_warm(C, float(inst.eps), np.zeros((U, m)), 1e-13, 20000)
    X1, _, it1 = oracle.forward_warm(C, float(inst.eps), rng.normal(0, 1.0, (U, m)), 1e-13, 20000)
    assert np.max(np.abs(X0 - X1)) < 1e-10
    assert np.all(it1 < 20000)
    b = np.ones(m)
    b[-1] = I - m + 1
    assert np.max(np.abs(X0.sum(2) - 1)) < 1e-10
    assert np.max(np.abs(X0.sum(1) - b)) < 1e-10


def test_implicit_gradient_matches_differences_of_the_converged_map():
    inst, C = _inst(U=3, I=7, m=3, seed=5)
    U, I, m = C.shape
    eps = float(inst.eps)
    r, e = inst.r.astype(np.float64), inst.e.astype(np.float64)

    def F(Cx):
        X, _, _ = oracle.forward_warm(Cx, eps, np.zeros((U, m)), 1e-14, 100000)
        return oracle.nsw(oracle.impact(r, e, X))

    X, _, _ = oracle.forward_warm(C, eps, np.zeros((U, m)), 1e-14, 100000)
    grad = warm.grad_implicit(r, e, eps, X, oracle.impact(r, e, X))
    rng = np.random.default_rng(2)
    h = 1e-5
    for _ in range(8):
        u, i, k = rng.integers(0, U), rng.integers(0, I), rng.integers(0, m)
        Cp, Cm = C.copy(), C.copy()
        Cp[u, i, k] += h
        Cm[u, i, k] -= h
        fd = (F(Cp) - F(Cm)) / (2 * h)
        assert abs(fd - grad[u, i, k]) <= 1e-6 * max(1.0, np.max(np.abs(grad)))
    # row shifts do not change the converged plan
    assert np.max(np.abs(grad.sum(2))) < 1e-9


def test_warm_starts_cut_the_iterations():
    inst = W.config("C1")
    eps = float(inst.eps)
    res = warm.solve_warm(inst.r, inst.e, eps, 5000, 1e-7, 4, rule="gd", lr=0.2)
    assert np.all(np.diff(res["F_hist"]) > 0)
    # one more small change of the costs: restarting from the last potentials
    # converges in far fewer iterations than a cold start
    C = res["C"] + W.random_costs(*res["C"].shape, 0.01 * eps, seed=8)
    U, I, m = C.shape
    _, _, cold = oracle.forward_warm(C, eps, np.zeros((U, m)), 1e-7, 5000)
    Xw, _, hot = oracle.forward_warm(C, eps, res["g"], 1e-7, 5000)
    Xc, _, _ = oracle.forward_warm(C, eps, np.zeros((U, m)), 1e-7, 5000)
    assert hot.mean() < 0.75 * cold.mean()
    assert np.max(np.abs(Xw - Xc)) < 1e-6
