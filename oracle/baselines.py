"""Baselines of the comparison in Section 4.1: MaxRele and NSW(Greedy), FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Wrappers of the C
oracle's ``fro_maxrele`` / ``fro_greedy`` (their comment states the greedy
rule this repository fixes, since the paper gives only its idea), and the
plan a selection defines.

A selection ``sel`` [U][m-1] (int32) lists the item each consumer sees at each
real position; every other item goes to the dummy position m-1, so the plan
is a 0/1 point of the polytope of problem otp: rows sum to 1, real columns
to 1, the dummy column to I - m + 1.
"""
from __future__ import annotations

import numpy as np

from .core import _d, _load, _ok, _p


def maxrele(r, m: int) -> np.ndarray:
    """sel [U][m-1]: each consumer's m-1 most relevant items, best first
    (equal relevances by item index)."""
    r = _d(r)
    U, I = r.shape
    sel = np.empty((U, m - 1), dtype=np.int32)
    _ok(_load().fro_maxrele(U, I, m, _p(r), _p(sel)), "maxrele")
    return sel


def greedy(r, e):
    """NSW(Greedy): (sel [U][m-1], Imp [I]).  Positions in order, consumers
    in index order within a position, each taking the unplaced item with the
    largest increase of F = sum_i log Imp_i."""
    r, e = _d(r), _d(e)
    U, I = r.shape
    m = e.shape[0] + 1
    sel = np.empty((U, m - 1), dtype=np.int32)
    imp = np.empty(I)
    _ok(_load().fro_greedy(U, I, m, _p(r), _p(e), _p(sel), _p(imp)), "greedy")
    return sel, imp


def plan_from_selection(sel, I: int) -> np.ndarray:
    """The 0/1 plan X [U][I][m] of a selection."""
    sel = np.asarray(sel)
    U, mm1 = sel.shape
    m = mm1 + 1
    X = np.zeros((U, I, m))
    X[:, :, m - 1] = 1.0
    for k in range(m - 1):
        X[np.arange(U), sel[:, k], m - 1] = 0.0
        X[np.arange(U), sel[:, k], k] = 1.0
    return X
