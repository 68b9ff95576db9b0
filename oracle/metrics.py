"""Evaluation metrics of a ranking policy, FP64 (Section 4.1, the list of
evaluation metrics).

TEST INFRASTRUCTURE ONLY (see the package docstring).  A policy is a plan
X [U][I][m] (column m-1 the dummy position, Section 2); r [U][I] are the
relevances, e [m-1] the exposures of the real positions.

* user utility      -- mean over consumers of sum_i sum_{k<m-1} r_ui e_k x_uik,
                       i.e. (sum_i Imp_i) / |U| (Eq. Imp).
* mean max envy     -- mean over items i of max_j (Imp_i(X_j) - Imp_i(X_i)),
                       where Imp_i(X_j) is the impact item i would have with
                       item j's allocation: sum_u r_ui sum_{k<m-1} e_k x_ujk.
                       The max includes j = i, so every term is >= 0.
* items better off  -- fraction of items whose impact exceeds 1.1 times the
                       impact under the uniform ranking policy (strictly).
* items worse off   -- fraction below 0.9 times it (strictly).

The uniform policy ranks every item at every real position with probability
1/I (the plan b_k / I of problem otp with C = 0), so its impacts are
Imp_i = (sum_u r_ui) (sum_{k<m-1} e_k) / I.

``envy_matrix`` uses one library matrix product as a step: with the
exposure matrix W_uj = sum_{k<m-1} e_k x_ujk, Imp_i(X_j) = (R^T W)_ij.
``envy_loops`` evaluates the definition with plain loops (tiny inputs only).
"""
from __future__ import annotations

import numpy as np

BETTER = 1.1
WORSE = 0.9


def _d(a) -> np.ndarray:
    return np.asarray(a, dtype=np.float64)


def exposure_matrix(e, X) -> np.ndarray:
    """W_uj = sum_{k<m-1} e_k x_ujk: the exposure consumer u gives item j."""
    X = _d(X)
    e = _d(e)
    m = X.shape[2]
    return X[:, :, : m - 1] @ e


def item_impacts(r, e, X) -> np.ndarray:
    """Eq. Imp: Imp_i = sum_u r_ui W_ui."""
    return (_d(r) * exposure_matrix(e, X)).sum(0)


def user_utility(r, e, X) -> float:
    return float(item_impacts(r, e, X).sum() / _d(r).shape[0])


def envy_matrix(r, e, X) -> np.ndarray:
    """E_ij = Imp_i(X_j) = sum_u r_ui W_uj."""
    return _d(r).T @ exposure_matrix(e, X)


def item_envy(r, e, X) -> np.ndarray:
    """envy_i = max_j E_ij - E_ii (>= 0)."""
    E = envy_matrix(r, e, X)
    return E.max(1) - np.diag(E)


def mean_max_envy(r, e, X) -> float:
    return float(item_envy(r, e, X).mean())


def envy_loops(r, e, X) -> np.ndarray:
    """Per-item envy from the definition, with explicit loops."""
    r = _d(r)
    e = _d(e)
    X = _d(X)
    U, I, m = X.shape

    def imp_with(i, j):   # impact of item i under item j's allocation
        tot = 0.0
        for u in range(U):
            for k in range(m - 1):
                tot += r[u, i] * e[k] * X[u, j, k]
        return tot

    out = np.zeros(I)
    for i in range(I):
        own = imp_with(i, i)
        out[i] = max(imp_with(i, j) - own for j in range(I))
    return out


def uniform_policy_impacts(r, e, I: int) -> np.ndarray:
    return _d(r).sum(0) * _d(e).sum() / I


def better_worse(r, e, X):
    """(fraction better off, fraction worse off) against the uniform policy."""
    imp = item_impacts(r, e, X)
    uni = uniform_policy_impacts(r, e, imp.shape[0])
    return float(np.mean(imp > BETTER * uni)), float(np.mean(imp < WORSE * uni))


def threshold_margin(r, e, X) -> float:
    """Smallest relative distance of an item's impact ratio to a threshold
    (how far the better/worse decisions are from flipping)."""
    imp = item_impacts(r, e, X)
    uni = uniform_policy_impacts(r, e, imp.shape[0])
    q = imp / uni
    return float(min(np.min(np.abs(q - BETTER)), np.min(np.abs(q - WORSE))))


def metrics(r, e, X) -> dict:
    b, w = better_worse(r, e, X)
    return {"user_utility": user_utility(r, e, X), "mean_max_envy": mean_max_envy(r, e, X),
            "items_better": b, "items_worse": w}
