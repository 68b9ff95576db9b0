"""Algorithm 1 on the converged map, FP64: Sinkhorn warm-started from the
previous outer step's column potentials and run until they stop moving
(Section 3 solves problem otp; Section 4 iterates Algorithm 1), and the
gradient of the converged plan by the implicit function theorem instead of
reverse mode through a fixed number of iterations.

TEST INFRASTRUCTURE ONLY (see the package docstring).  This is a different
map from the fixed-T Algorithm 1 of ``oracle.core`` (it differentiates the
exact entropic plan, which the T-iterate only approaches).

For one consumer with plan X (I x m) and G = dF/dX, the balanced plan's
optimality conditions give dF/dC = -(1/eps) X * (G - lam 1^T - 1 mu^T) with
(lam, mu) solving
    diag(X 1) lam + X mu = (X * G) 1,   X^T lam + diag(X^T 1) mu = (X * G)^T 1,
gauge mu_{m-1} = 0 (``brute.implicit_grad`` solves it directly).
"""
from __future__ import annotations

import numpy as np

from . import brute
from .core import adam, forward_warm, gd, impact, nsw


def grad_implicit(r, e, eps, X, imp):
    """dF/dC [U][I][m] at the plans X by the implicit function theorem."""
    r = np.asarray(r, dtype=np.float64)
    e = np.asarray(e, dtype=np.float64)
    U, I, m = X.shape
    out = np.empty_like(X)
    for u in range(U):
        G = np.zeros((I, m))
        G[:, : m - 1] = (r[u] / imp)[:, None] * e[None, :]
        out[u] = brute.implicit_grad(X[u], G, eps)
    return out


def solve_warm(r, e, eps, T_max, tol, N, rule="adam", lr=None, b1=0.9, b2=0.999, aeps=1e-8):
    """Algorithm 1 with warm starts and implicit gradients.  Returns dict(C, X,
    F_hist, imp, iters [N+1][U], g)."""
    r = np.asarray(r, dtype=np.float64)
    e = np.asarray(e, dtype=np.float64)
    U, I = r.shape
    m = e.shape[0] + 1
    if lr is None:
        lr = 0.1 * float(eps)
    C = np.zeros((U, I, m))
    mom, vel = np.zeros_like(C), np.zeros_like(C)
    g = np.zeros((U, m))
    Fh = np.empty(N + 1)
    iters = np.empty((N + 1, U), dtype=np.int32)
    for n in range(N + 1):
        X, g, it = forward_warm(C, eps, g, tol, T_max)
        iters[n] = it
        imp = impact(r, e, X)
        Fh[n] = nsw(imp)
        if n == N:
            break
        grad = grad_implicit(r, e, eps, X, imp)
        if rule == "adam":
            adam(C, mom, vel, grad, lr, b1, b2, aeps, step=n + 1)
        else:
            gd(C, grad, lr)
    return {"C": C, "X": X, "F_hist": Fh, "imp": imp, "iters": iters, "g": g}
