"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these tests retypes the oracle's own formula: each checks a closed
form, an invariant, an independent library routine, central finite
differences, or a brute-force optimum (``oracle.brute`` never runs Sinkhorn).
"""
import json
import os

import numpy as np
import pytest

import oracle
import workloads as W
from oracle import brute

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rand_problem(U, I, m, seed, scale=0.2):
    rng = np.random.default_rng(seed)
    r = rng.uniform(0.1, 1.0, (U, I))
    e = W.exposure(m).astype(np.float64)
    C = rng.normal(0.0, scale, (U, I, m))
    return r, e, C


def _F(r, e, eps, T, C):
    return oracle.nsw(oracle.impact(r, e, oracle.forward(C, eps, T)))


# ---------------------------------------------------------------- forward
@pytest.mark.parametrize("T", [1, 3, 17])
def test_column_marginals_exact_at_any_T(T):
    """Eq. dsm2 and the dummy mass I-m+1 hold after every column half-step."""
    r, e, C = _rand_problem(4, 9, 4, seed=T, scale=0.5)
    X = oracle.forward(C, 0.1, T)
    b = brute.column_masses(9, 4)
    assert np.abs(X.sum(1) - b[None, :]).max() < 1e-12
    assert (X > 0).all()


def test_row_marginals_at_convergence():
    """Eq. dsm1 holds once Sinkhorn has converged."""
    r, e, C = _rand_problem(3, 7, 3, seed=5, scale=0.3)
    X, f, g, its = oracle.forward_converge(C, 0.1, tol=1e-13, cap=100000)
    assert np.abs(X.sum(2) - 1).max() < 1e-12
    assert np.abs(X.sum(1) - brute.column_masses(7, 3)[None, :]).max() < 1e-12


@pytest.mark.parametrize("T", [1, 4])
def test_rank_one_cost_gives_product_plan(T):
    """Separable cost c_ik = alpha_i + beta_k: plan = b_k / I after >= 1 iteration."""
    rng = np.random.default_rng(7)
    U, I, m = 3, 11, 5
    C = rng.normal(0, 1, (U, I, 1)) + rng.normal(0, 1, (U, 1, m))
    X = oracle.forward(C, 0.07, T)
    assert np.abs(X - brute.plan_rank_one(I, m)[None]).max() < 1e-13


def test_theorem1_round_trip():
    """Theorem 1: for a strictly positive feasible X, C = -eps log X gives
    Sinkhorn(C) = X (already after one iteration)."""
    rng = np.random.default_rng(3)
    I, m = 4, 3
    V = brute.vertices(I, m)
    lam = rng.dirichlet(np.ones(V.shape[0]), size=2)
    X = np.einsum("up,pik->uik", lam, V)            # feasible, strictly positive
    assert (X > 0).all()
    eps = 0.05
    C = -eps * np.log(X)
    for T in (1, 5):
        assert np.abs(oracle.forward(C, eps, T) - X).max() < 1e-13


@pytest.mark.parametrize("eps", [0.05, 0.3])
def test_2x2_closed_form(eps):
    rng = np.random.default_rng(int(eps * 100))
    C = rng.normal(0, 0.2, (1, 2, 2))
    X, _, _, _ = oracle.forward_converge(C, eps, tol=1e-14, cap=100000)
    assert np.abs(X[0] - brute.plan_2x2(C[0], eps)).max() < 1e-12


def test_primal_equals_dual_at_convergence():
    r, e, C = _rand_problem(2, 6, 4, seed=9, scale=0.3)
    eps = 0.1
    X, f, g, _ = oracle.forward_converge(C, eps, tol=1e-14, cap=100000)
    b = brute.column_masses(6, 4)
    for u in range(2):
        p = brute.entropic_primal(C[u], X[u], eps)
        d = brute.entropic_dual(f[u], g[u], b, eps)
        assert abs(p - d) < 1e-12


def test_row_shift_invariance_exact_at_finite_T():
    """Adding a per-row constant to C leaves every Sinkhorn iterate's plan
    unchanged (it is absorbed by f); adding a per-column constant does not at
    finite T."""
    r, e, C = _rand_problem(2, 8, 4, seed=2, scale=0.3)
    eps, T = 0.05, 5
    X0 = oracle.forward(C, eps, T)
    alpha = np.random.default_rng(1).normal(0, 1, (2, 8, 1))
    assert np.abs(oracle.forward(C + alpha, eps, T) - X0).max() < 1e-13
    beta = np.random.default_rng(2).normal(0, 1, (2, 1, 4))
    assert np.abs(oracle.forward(C + beta, eps, T) - X0).max() > 1e-6


def test_entropic_plan_minimises_otp():
    """The converged plan beats random feasible plans on problem otp."""
    rng = np.random.default_rng(4)
    I, m, eps = 4, 3, 0.2
    C = rng.normal(0, 0.5, (1, I, m))
    X, _, _, _ = oracle.forward_converge(C, eps, tol=1e-14, cap=100000)
    best = brute.entropic_primal(C[0], X[0], eps)
    V = brute.vertices(I, m)
    for _ in range(200):
        lam = rng.dirichlet(np.ones(V.shape[0]))
        Y = np.einsum("p,pik->ik", lam, V)
        assert brute.entropic_primal(C[0], Y, eps) >= best - 1e-12


# ---------------------------------------------------------------- impact / F
def test_uniform_policy_impacts():
    """At C = 0 the plan is the uniform policy x = b_k / I, so
    Imp_i = (sum_u r_ui)(sum_{k<m} e_k) / I; F = sum_i log of that."""
    inst = W.config("C1")
    r = inst.r.astype(np.float64)
    e = inst.e.astype(np.float64)
    X = oracle.forward(np.zeros((inst.U, inst.I, inst.m)), float(inst.eps), 3)
    imp = oracle.impact(r, e, X)
    ref = brute.uniform_impacts(r, e, inst.I)
    assert np.abs(imp / ref - 1).max() < 1e-14
    assert abs(oracle.nsw(imp) - np.sum(np.log(ref))) < 1e-12


def test_impact_matches_einsum_and_ignores_dummy():
    r, e, C = _rand_problem(5, 7, 4, seed=12)
    X = oracle.forward(C, 0.1, 6)
    assert np.abs(oracle.impact(r, e, X) - brute.impacts(r, e, X)).max() < 1e-13
    X2 = X.copy()
    X2[:, :, -1] += 3.0   # mass on the dummy carries no impact
    assert np.abs(oracle.impact(r, e, X2) - oracle.impact(r, e, X)).max() == 0.0


# ---------------------------------------------------------------- gradient
def test_grad_matches_central_differences():
    r, e, C = _rand_problem(3, 6, 4, seed=21, scale=0.3)
    eps, T = 0.1, 15
    gC, gr = oracle.grad(r, e, eps, T, C)
    scale = np.abs(gC).max()
    rng = np.random.default_rng(0)
    h = 1e-5
    for _ in range(25):
        idx = tuple(rng.integers(0, s) for s in C.shape)
        Cp, Cm = C.copy(), C.copy()
        Cp[idx] += h
        Cm[idx] -= h
        fd = (_F(r, e, eps, T, Cp) - _F(r, e, eps, T, Cm)) / (2 * h)
        assert abs(fd - gC[idx]) <= 1e-7 * scale + 1e-6 * abs(gC[idx]), (idx, fd, gC[idx])
    for _ in range(10):
        idx = tuple(rng.integers(0, s) for s in r.shape)
        rp, rm = r.copy(), r.copy()
        rp[idx] += h
        rm[idx] -= h
        fd = (_F(rp, e, eps, T, C) - _F(rm, e, eps, T, C)) / (2 * h)
        assert abs(fd - gr[idx]) <= 1e-8 + 1e-6 * abs(gr[idx])


def test_grad_rows_sum_to_zero():
    """Row shifts leave X unchanged (see above), so every row of dF/dC sums to 0."""
    r, e, C = _rand_problem(3, 8, 5, seed=22, scale=0.3)
    gC, _ = oracle.grad(r, e, 0.05, 20, C)
    assert np.abs(gC.sum(2)).max() < 1e-12 * max(1.0, np.abs(gC).max())


def test_grad_equals_implicit_gradient_at_convergence():
    """For T large the unrolled gradient tends to the implicit-function
    gradient of the exact entropic solution."""
    r, e, C = _rand_problem(2, 5, 3, seed=23, scale=0.3)
    eps = 0.2
    X, f, g, its = oracle.forward_converge(C, eps, tol=1e-15, cap=100000)
    T = int(its.max()) * 3 + 50
    imp = oracle.impact(r, e, X)
    gC, _ = oracle.grad(r, e, eps, T, C, imp=imp)
    for u in range(2):
        G = np.zeros((5, 3))
        G[:, :2] = r[u][:, None] * e[None, :] / imp[:, None]
        ref = brute.implicit_grad(X[u], G, eps)
        assert np.abs(gC[u] - ref).max() < 1e-10 * max(1.0, np.abs(ref).max())


def test_grad_2x2_analytic():
    """One consumer, I = m = 2 at convergence: x11 = p = sigmoid(-d/(2 eps)),
    d = c11 + c22 - c12 - c21; F = log(r1 e1 p) + log(r2 e1 (1 - p)), so
    dF/dc11 = dF/dc22 = -(1-2p)/(2 eps) ... written out via dp/dd."""
    eps = 0.3
    r = np.array([[0.7, 0.4]])
    e = np.array([1.0])
    C = np.array([[[0.1, -0.2], [0.05, 0.3]]])
    X, _, _, its = oracle.forward_converge(C, eps, tol=1e-15, cap=100000)
    gC, _ = oracle.grad(r, e, eps, int(its.max()) * 3 + 50, C)
    p = X[0, 0, 0]
    dF_dp = 1.0 / p - 1.0 / (1.0 - p)
    dp_dd = -p * (1 - p) / (2 * eps)
    sign = np.array([[1.0, -1.0], [-1.0, 1.0]])
    ref = dF_dp * dp_dd * sign
    assert np.abs(gC[0] - ref).max() < 1e-10


# ---------------------------------------------------------------- update
def test_adam_matches_torch_adam_maximize():
    """Adam on -F equals torch.optim.Adam(maximize=True) in float64."""
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(5)
    n = 37
    C = rng.normal(0, 1, n)
    mom = np.zeros(n)
    vel = np.zeros(n)
    p = torch.tensor(C.copy(), dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([p], lr=0.01, betas=(0.9, 0.999), eps=1e-8, maximize=True)
    for step in range(1, 8):
        g = rng.normal(0, 1, n) * (10.0 ** rng.integers(-6, 1, n))
        oracle.adam(C, mom, vel, g, 0.01, 0.9, 0.999, 1e-8, step)
        p.grad = torch.tensor(g, dtype=torch.float64)
        opt.step()
        assert np.abs(C - p.detach().numpy()).max() < 1e-14


def test_adam_first_step_closed_form():
    """First Adam step: bias-corrected moments are g and g^2, so the move is
    lr * g / (|g| + eps_adam)."""
    g = np.array([0.5, -2.0, 1e-9, 0.0])
    C = np.zeros(4)
    oracle.adam(C, np.zeros(4), np.zeros(4), g, 0.1, 0.9, 0.999, 1e-8, 1)
    assert np.abs(C - 0.1 * g / (np.abs(g) + 1e-8)).max() < 1e-15


# ---------------------------------------------------------------- Algorithm 1
def test_gradient_ascent_with_armijo_is_monotone():
    r, e, C = _rand_problem(3, 6, 3, seed=31, scale=0.1)
    eps, T = 0.1, 30
    Fv = _F(r, e, eps, T, C)
    for _ in range(15):
        gC, _ = oracle.grad(r, e, eps, T, C)
        eta = 1.0
        g2 = float(np.sum(gC * gC))
        while True:
            Cn = C + eta * gC
            Fn = _F(r, e, eps, T, Cn)
            if Fn >= Fv + 1e-4 * eta * g2 or eta < 1e-12:
                break
            eta *= 0.5
        assert Fn >= Fv - 1e-15
        C, Fv = Cn, Fn


def _golden_tiny():
    with open(os.path.join(GOLDEN, "tiny_optima.json")) as fh:
        return json.load(fh)["instances"]


@pytest.mark.parametrize("case", ["T1", "T2", "T3"])
def test_ascent_approaches_brute_force_optimum(case):
    g = [c for c in _golden_tiny() if c["name"] == case][0]
    r = np.array(g["r"])
    e = np.array(g["e"])
    Fstar = g["F_star"]
    res = oracle.solve(r, e, 0.05, 300, 1500, lr=0.05)
    Fh = res["F_hist"]
    # X^(T) has exact columns but rows off by delta.  X/(1+delta) plus a
    # nonnegative transport of the deficits is feasible and dominates
    # X/(1+delta), hence F(X) <= F* + I log(1 + delta).
    delta = np.abs(res["X"].sum(2) - 1).max()
    assert Fh[-1] <= Fstar + r.shape[1] * np.log1p(delta) + 1e-12
    assert (Fh <= Fstar + 1e-5).all()
    assert Fstar - Fh[-1] < g["tol_gap"]
    assert Fh[-1] > Fh[0]


def test_brute_force_golden_values_are_certified():
    """The stored optima carry Frank-Wolfe certificates below 1e-9."""
    for g in _golden_tiny():
        assert g["fw_gap"] < 1e-9


def test_solve_resume_is_bitwise():
    inst = W.small_instance(4, 7, 3, seed=8, eps=0.05, T=20)
    r, e = inst.r.astype(np.float64), inst.e.astype(np.float64)
    full = oracle.solve(r, e, float(inst.eps), 20, 6)
    a = oracle.solve(r, e, float(inst.eps), 20, 2)
    b = oracle.solve(r, e, float(inst.eps), 20, 4, C0=a["C"], mom=a["mom"], vel=a["vel"],
                     start_step=2)
    assert np.array_equal(b["C"], full["C"])
    assert np.array_equal(b["F_hist"], full["F_hist"][2:])


def test_solve_is_the_plain_loop():
    """solve() equals forward / impact / grad / Adam called one by one."""
    inst = W.small_instance(3, 6, 4, seed=9, eps=0.05, T=15)
    r, e, eps = inst.r.astype(np.float64), inst.e.astype(np.float64), float(inst.eps)
    N, lr = 4, 0.005
    res = oracle.solve(r, e, eps, 15, N, lr=lr)
    C = np.zeros((3, 6, 4))
    mom, vel = np.zeros_like(C), np.zeros_like(C)
    for n in range(N + 1):
        X = oracle.forward(C, eps, 15)
        imp = oracle.impact(r, e, X)
        assert oracle.nsw(imp) == res["F_hist"][n]
        if n == N:
            break
        gC, _ = oracle.grad(r, e, eps, 15, C, imp=imp)
        oracle.adam(C, mom, vel, gC, lr, step=n + 1)
    assert np.array_equal(C, res["C"])


def test_gradient_norm_stop_of_algorithm_1():
    """The loop condition of Algorithm 1: ascend only while ||dF/dC|| > t."""
    inst = W.config("C1")
    r, e, eps, T = inst.r, inst.e, float(inst.eps), 30
    full = oracle.solve(r, e, eps, T, 6, rule="gd", lr=0.5)
    g = full["gnorm"]
    assert full["updates"] == 6 and np.all(np.isfinite(g))
    # t above every norm: stop at C0 = 0, no update, F constant
    top = oracle.solve(r, e, eps, T, 6, rule="gd", lr=0.5, grad_tol=2 * g.max())
    assert top["updates"] == 0 and np.all(top["C"] == 0.0)
    assert np.all(top["F_hist"] == full["F_hist"][0])
    # t between the running minimum before step j and the norm at step j: j updates
    j = next(k for k in range(1, 6) if g[k] < g[:k].min())
    t = 0.5 * (g[j] + g[:j].min())
    part = oracle.solve(r, e, eps, T, 6, rule="gd", lr=0.5, grad_tol=t)
    assert part["updates"] == j
    assert np.array_equal(part["F_hist"][: j + 1], full["F_hist"][: j + 1])
    assert np.all(part["F_hist"][j + 1:] == full["F_hist"][j])
    ref = oracle.solve(r, e, eps, T, j, rule="gd", lr=0.5)
    assert np.array_equal(part["C"], ref["C"]) and np.array_equal(part["X"], ref["X"])
