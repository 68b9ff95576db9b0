"""Pins of the baseline rankings of the comparison in Section 4.1
(oracle/baselines.py): MaxRele and NSW(Greedy).

MaxRele is pinned by the rearrangement inequality (it maximises every
consumer's utility over all deterministic rankings, checked by brute force);
Greedy by re-deriving every decision from the objective itself (F = sum_i
log Imp_i evaluated with logarithms for each candidate, not the ratio the
oracle compares), by hand-worked and closed-form cases, and by the C
oracle's independent Eq. Imp on the plan it returns."""
import itertools

import numpy as np

import oracle
import workloads as W
from oracle import baselines as B


def _feasible(X, I, m):
    b = np.ones(m)
    b[-1] = I - m + 1
    assert np.all((X == 0) | (X == 1))
    assert np.all(X.sum(2) == 1)
    assert np.all(X.sum(1) == b[None, :])


def test_hand_worked_instance():
    # two consumers, three items, positions e = (1, 0.5) plus the dummy
    r = np.array([[0.9, 0.5, 0.2], [0.8, 0.6, 0.1]])
    e = np.array([1.0, 0.5])
    assert B.maxrele(r, 3).tolist() == [[0, 1], [0, 1]]
    sel, imp = B.greedy(r, e)
    # k=0: u0 takes item 0 (all impacts 0, largest r); u1 takes item 1 (items 1, 2 have
    # Imp 0, r 0.6 > 0.1).  k=1: u0 takes item 2 (Imp 0); u1 compares 0.8/0.9 with
    # 0.1/0.1 and takes item 2.
    assert sel.tolist() == [[0, 2], [1, 2]]
    assert np.allclose(imp, [0.9, 0.6, 0.1 + 0.05], atol=1e-15)


def test_maxrele_maximises_each_consumers_utility():
    rng = np.random.default_rng(0)
    U, I, m = 4, 5, 4
    r = rng.uniform(0.05, 1.0, (U, I))
    e = W.exposure(m).astype(np.float64)
    sel = B.maxrele(r, m)
    for u in range(U):
        best = max(sum(r[u, p[k]] * e[k] for k in range(m - 1))
                   for p in itertools.permutations(range(I), m - 1))
        got = sum(r[u, sel[u, k]] * e[k] for k in range(m - 1))
        assert abs(got - best) < 1e-14
    _feasible(B.plan_from_selection(sel, I), I, m)


def test_maxrele_ties_go_to_the_smaller_index():
    r = np.array([[0.5, 0.7, 0.5, 0.7, 0.1]])
    assert B.maxrele(r, 5).tolist() == [[1, 3, 0, 2]]


def test_greedy_decisions_maximise_the_objective():
    rng = np.random.default_rng(1)
    U, I, m = 5, 7, 4
    r = rng.uniform(0.05, 1.0, (U, I))
    e = W.exposure(m).astype(np.float64)
    sel, imp = B.greedy(r, e)
    X = np.zeros((U, I, m))
    cur = np.zeros(I)
    for k in range(m - 1):
        for u in range(U):
            placed = set(sel[u, :k].tolist())
            cand = [i for i in range(I) if i not in placed]
            zero = [i for i in cand if cur[i] == 0.0]
            if zero:   # log Imp_i rises from -inf: the largest relevance among them
                best = max(zero, key=lambda i: (r[u, i], -i))
            else:
                gain = {i: np.log(cur[i] + r[u, i] * e[k]) - np.log(cur[i]) for i in cand}
                top = max(gain.values())
                assert gain[sel[u, k]] >= top - 1e-12 * abs(top)
                best = sel[u, k]
            assert sel[u, k] == best
            X[u, best, k] = 1.0
            cur[best] += r[u, best] * e[k]
    assert np.allclose(cur, imp, rtol=1e-15, atol=0)
    Xp = B.plan_from_selection(sel, I)
    _feasible(Xp, I, m)
    assert np.max(np.abs(oracle.impact(r, e, Xp) / imp - 1)) < 1e-13


def test_greedy_equal_relevance_cycles_through_the_items():
    # all relevances equal: every item is shown once before any is shown twice,
    # in index order, and ties among shown items go to the smaller index
    r = np.full((4, 3), 0.5)
    sel, imp = B.greedy(r, np.array([1.0]))
    assert sel[:, 0].tolist() == [0, 1, 2, 0]
    assert np.allclose(imp, [1.0, 0.5, 0.5])


def test_greedy_gives_every_item_impact_once_there_are_enough_slots():
    rng = np.random.default_rng(2)
    U, I, m = 30, 40, 3
    r = rng.uniform(0.01, 1.0, (U, I))
    e = W.exposure(m).astype(np.float64)
    sel, imp = B.greedy(r, e)
    assert U * (m - 1) >= I
    assert np.all(imp > 0)
    assert np.isfinite(oracle.nsw(imp))
    # MaxRele leaves the least relevant items without exposure
    imp_mr = oracle.impact(r, e, B.plan_from_selection(B.maxrele(r, m), I))
    assert oracle.nsw(imp) > np.sum(np.log(np.maximum(imp_mr, 1e-300)))
