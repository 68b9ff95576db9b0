"""Brute-force optima and closed forms for tiny fair-ranking instances.

TEST INFRASTRUCTURE ONLY.  NumPy/SciPy code that is independent of
``fr_oracle.c``: it never runs Sinkhorn.  It pins the oracle to results that
the mathematics fixes:

* Exact optima of problem nsw (Section 2) on tiny instances, by grid search
  (U=2, I=2, m=2 and U=2, I=3, m=2) or by exponentiated-gradient ascent over
  the Birkhoff polytope (U=2, I=3, m=3), each with a Frank-Wolfe duality-gap
  certificate.  F is concave in X and the feasible set is convex, so
  F* <= F(X) + gap(X) for every feasible X.
* Closed forms of the entropic transport problem otp (Section 3): the 2x2
  plan, the rank-one (separable cost) plan, the uniform-policy impacts, and
  the implicit-function gradient of F at a converged Sinkhorn plan.
"""
from __future__ import annotations

import itertools

import numpy as np
from scipy.optimize import linear_sum_assignment


# --------------------------------------------------------------------------
# objective of problem nsw (Eqs. Imp and objF) on an explicit plan
def impacts(r: np.ndarray, e: np.ndarray, X: np.ndarray) -> np.ndarray:
    """Imp_i = sum_u sum_{k<m} r(u,i) e(k) x_uik, written with einsum."""
    m = X.shape[2]
    return np.einsum("ui,k,uik->i", r, e, X[:, :, : m - 1])


def objective(r, e, X) -> float:
    return float(np.sum(np.log(impacts(r, e, X))))


def fw_gap(r: np.ndarray, e: np.ndarray, X: np.ndarray) -> float:
    """Frank-Wolfe gap max_V <grad F(X), V - X> over the feasible set.

    The linear maximisation over one consumer's transportation polytope puts
    m-1 distinct items on the m-1 real positions (an assignment problem) and
    the rest on the dummy, whose column carries no exposure and hence zero
    gradient.  Solved exactly with scipy's assignment routine."""
    U, I, m = X.shape
    imp = impacts(r, e, X)
    G = r[:, :, None] * e[None, None, :] / imp[None, :, None]       # [U, I, m-1]
    gap = 0.0
    for u in range(U):
        rows, cols = linear_sum_assignment(G[u], maximize=True)
        best = G[u][rows, cols].sum()
        gap += best - float(np.sum(G[u] * X[u, :, : m - 1]))
    return gap


# --------------------------------------------------------------------------
# tiny-instance optima
def _plan_t1(p):
    """U x 2 x 2 plans [[p, 1-p], [1-p, p]] for p [U]."""
    p = np.asarray(p, dtype=np.float64)
    X = np.empty((p.shape[0], 2, 2))
    X[:, 0, 0] = p
    X[:, 0, 1] = 1 - p
    X[:, 1, 0] = 1 - p
    X[:, 1, 1] = p
    return X


def optimum_t1(r: np.ndarray, e: np.ndarray):
    """U=2, I=2, m=2.  Each plan is fixed by p_u = x_u11 in [0,1]; a
    1001 x 1001 grid followed by five 10x zooms around the best point."""
    assert r.shape == (2, 2) and e.shape == (1,)
    lo = np.zeros(2)
    hi = np.ones(2)
    best = None
    for _ in range(6):
        g0 = np.linspace(lo[0], hi[0], 1001)
        g1 = np.linspace(lo[1], hi[1], 1001)
        P0, P1 = np.meshgrid(g0, g1, indexing="ij")
        imp1 = e[0] * (r[0, 0] * P0 + r[1, 0] * P1)
        imp2 = e[0] * (r[0, 1] * (1 - P0) + r[1, 1] * (1 - P1))
        with np.errstate(divide="ignore"):
            Fg = np.log(imp1) + np.log(imp2)
        j = np.unravel_index(np.argmax(Fg), Fg.shape)
        best = np.array([g0[j[0]], g1[j[1]]])
        w = (hi - lo) / 100.0
        lo = np.maximum(best - w, 0.0)
        hi = np.minimum(best + w, 1.0)
    X = _plan_t1(best)
    return objective(r, e, X), X


def _simplex_grid(n: int):
    """All (a, b, c) >= 0 with a + b + c = 1 on a grid of step 1/n."""
    pts = [(a, b, n - a - b) for a in range(n + 1) for b in range(n + 1 - a)]
    return np.array(pts, dtype=np.float64) / n


def optimum_t2(r: np.ndarray, e: np.ndarray):
    """U=2, I=3, m=2.  X_u has one real position: column 0 is a point q_u of
    the 3-simplex and the dummy column is 1 - q_u.  Grid of step 1/60 on both
    simplices, then coordinate zooms around the best pair."""
    assert r.shape == (2, 3) and e.shape == (1,)
    S = _simplex_grid(60)
    best_F, best = -np.inf, None
    for a in S:
        imp = e[0] * (r[0][None, :] * a[None, :] + r[1][None, :] * S)
        with np.errstate(divide="ignore"):
            Fv = np.log(imp).sum(1)
        j = int(np.argmax(Fv))
        if Fv[j] > best_F:
            best_F, best = Fv[j], (a.copy(), S[j].copy())
    q0, q1 = best
    step = 1.0 / 60
    for _ in range(8):
        loc = _simplex_grid(20) * 2 - 2.0 / 3          # offsets summing to zero
        cands0 = q0[None, :] + step * loc
        cands1 = q1[None, :] + step * loc
        cands0 = cands0[(cands0 >= 0).all(1)]
        cands1 = cands1[(cands1 >= 0).all(1)]
        A = cands0[:, None, :]
        B = cands1[None, :, :]
        imp = e[0] * (r[0] * A + r[1] * B)
        with np.errstate(divide="ignore"):
            Fv = np.log(imp).sum(2)
        j0, j1 = np.unravel_index(np.argmax(Fv), Fv.shape)
        q0, q1 = cands0[j0].copy(), cands1[j1].copy()
        step /= 4
    X = np.empty((2, 3, 2))
    X[0, :, 0], X[0, :, 1] = q0, 1 - q0
    X[1, :, 0], X[1, :, 1] = q1, 1 - q1
    return objective(r, e, X), X


def vertices(I: int, m: int) -> np.ndarray:
    """All vertices of one consumer's feasible set (Eqs. dsm1-dsm4 with the
    dummy column of mass I - m + 1): 0/1 plans that put m-1 distinct items
    on the m-1 real positions and every other item on the dummy."""
    out = []
    for sel in itertools.permutations(range(I), m - 1):
        V = np.zeros((I, m))
        V[:, m - 1] = 1.0
        for k, i in enumerate(sel):
            V[i, k] = 1.0
            V[i, m - 1] = 0.0
        out.append(V)
    return np.array(out)


def optimum_vertex_weights(r: np.ndarray, e: np.ndarray, m: int, lam0=None,
                           iters: int = 200000, tol: float = 1e-12):
    """Maximise F over convex weights of the vertices of each consumer's
    feasible set by exponentiated-gradient ascent; stops once the
    Frank-Wolfe gap is below tol.  Returns (F, X, gap)."""
    U, I = r.shape
    V = vertices(I, m)
    nv = V.shape[0]
    lam = np.full((U, nv), 1.0 / nv) if lam0 is None else np.array(lam0, dtype=np.float64)
    lam = np.maximum(lam, 1e-300)
    lam /= lam.sum(1, keepdims=True)
    eta = 0.5
    gap = np.inf
    for it in range(iters):
        X = np.einsum("up,pik->uik", lam, V)
        imp = impacts(r, e, X)
        G = np.zeros_like(X)
        G[:, :, : m - 1] = r[:, :, None] * e[None, None, :] / imp[None, :, None]
        glam = np.einsum("uik,pik->up", G, V)
        lam = lam * np.exp(eta * (glam - glam.max(1, keepdims=True)))
        lam = np.maximum(lam, 1e-300)
        lam /= lam.sum(1, keepdims=True)
        if it % 500 == 499:
            gap = fw_gap(r, e, np.einsum("up,pik->uik", lam, V))
            if gap < tol:
                break
    X = np.einsum("up,pik->uik", lam, V)
    return objective(r, e, X), X, fw_gap(r, e, X)


def optimum_birkhoff(r: np.ndarray, e: np.ndarray, iters: int = 200000):
    """U consumers, I = m = 3: every plan is a 3x3 doubly-stochastic matrix
    (the dummy's mass is I - m + 1 = 1), a convex combination of the six
    permutation matrices.  Returns (F, X, gap)."""
    assert r.shape[1] == 3 and e.shape == (2,)
    return optimum_vertex_weights(r, e, 3, iters=iters)


# --------------------------------------------------------------------------
# closed forms of the entropic problem otp
def plan_2x2(c: np.ndarray, eps: float) -> np.ndarray:
    """I = m = 2, marginals all one: minimising the entropic objective over
    [[p, 1-p], [1-p, p]] gives p = sigmoid(-(c11 + c22 - c12 - c21)/(2 eps))."""
    d = c[0, 0] + c[1, 1] - c[0, 1] - c[1, 0]
    p = 1.0 / (1.0 + np.exp(d / (2.0 * eps)))
    return np.array([[p, 1 - p], [1 - p, p]])


def plan_rank_one(I: int, m: int) -> np.ndarray:
    """Separable cost c_ik = alpha_i + beta_k: the Gibbs kernel is rank one,
    so the plan is the product of the marginals, x_ik = b_k / I."""
    b = np.ones(m)
    b[-1] = I - m + 1
    return np.tile(b / I, (I, 1))


def column_masses(I: int, m: int) -> np.ndarray:
    b = np.ones(m)
    b[-1] = I - m + 1
    return b


def uniform_impacts(r: np.ndarray, e: np.ndarray, I: int) -> np.ndarray:
    """Impacts of the uniform policy x_uik = b_k / I (the plan at C = 0):
    Imp_i = (sum_u r_ui) (sum_{k<m} e_k) / I."""
    return r.sum(0) * e.sum() / I


def implicit_grad(X: np.ndarray, G: np.ndarray, eps: float) -> np.ndarray:
    """Gradient of sum G * X*(C) at an exactly balanced entropic plan X of one
    consumer, by implicit differentiation of the optimality conditions:
        dF/dC = -(1/eps) X * (G - lam 1^T - 1 mu^T)
    with (lam, mu) solving  diag(X1) lam + X mu = (X*G) 1,
                            X^T lam + diag(X^T 1) mu = (X*G)^T 1,  mu_m = 0."""
    I, m = X.shape
    A = np.zeros((I + m, I + m))
    A[:I, :I] = np.diag(X.sum(1))
    A[:I, I:] = X
    A[I:, :I] = X.T
    A[I:, I:] = np.diag(X.sum(0))
    rhs = np.concatenate([(X * G).sum(1), (X * G).sum(0)])
    # gauge: drop mu_m (last unknown) and the last equation (redundant)
    sol = np.linalg.solve(A[:-1, :-1], rhs[:-1])
    lam = sol[:I]
    mu = np.concatenate([sol[I:], [0.0]])
    return -(1.0 / eps) * X * (G - lam[:, None] - mu[None, :])


def entropic_primal(C: np.ndarray, X: np.ndarray, eps: float) -> float:
    """Objective of problem otp for one consumer."""
    return float(np.sum(C * X) + eps * np.sum(X * (np.log(X) - 1.0)))


def entropic_dual(f: np.ndarray, g: np.ndarray, b: np.ndarray, eps: float) -> float:
    """At the balanced optimum the primal equals <f, a> + <g, b> - eps * I
    (a = 1), since sum_ik x_ik = I."""
    return float(np.sum(f) + np.sum(g * b) - eps * f.shape[0])
