"""Pins of the FP64 evaluation metrics (oracle/metrics.py) against the
definitions of Section 4.1's metric list: the uniform policy, a hand-worked
deterministic policy, a two-item closed form, brute-force loops, invariance
under relabelling, and the independent C implementation of Eq. Imp."""
import numpy as np

import oracle
import workloads as W
from oracle import brute
from oracle import metrics as M


def _plan(U, I, m, seed, scale=0.3, eps=0.05, T=60):
    C = W.random_costs(U, I, m, scale, seed=seed)
    return oracle.forward(C, eps, T)


def test_uniform_policy_has_no_envy_and_no_better_or_worse_items():
    U, I, m = 7, 9, 4
    rng = np.random.default_rng(0)
    r = rng.uniform(0.1, 1.0, (U, I))
    e = W.exposure(m).astype(np.float64)
    X = np.broadcast_to(brute.plan_rank_one(I, m), (U, I, m)).copy()
    assert np.max(np.abs(M.item_envy(r, e, X))) < 1e-14
    assert M.better_worse(r, e, X) == (0.0, 0.0)
    uni = M.uniform_policy_impacts(r, e, I)
    assert abs(M.user_utility(r, e, X) - uni.sum() / U) < 1e-13


def test_hand_worked_deterministic_policy():
    # one real position (e_1 = 1) and the dummy; both consumers show item 0
    r = np.array([[0.9, 0.5, 0.2], [0.8, 0.6, 0.1]])
    e = np.array([1.0])
    X = np.zeros((2, 3, 2))
    X[:, 0, 0] = 1.0
    X[:, 1:, 1] = 1.0
    # Imp = [1.7, 0, 0]; uniform Imp = [1.7, 1.1, 0.3] / 3
    # E_i0 = r_0i + r_1i, E_i1 = E_i2 = 0 -> envy = [0, 1.1, 0.3]
    assert np.allclose(M.item_impacts(r, e, X), [1.7, 0.0, 0.0], atol=1e-15)
    assert np.allclose(M.item_envy(r, e, X), [0.0, 1.1, 0.3], atol=1e-15)
    assert abs(M.mean_max_envy(r, e, X) - 1.4 / 3) < 1e-15
    assert abs(M.user_utility(r, e, X) - 0.85) < 1e-15
    assert M.better_worse(r, e, X) == (1 / 3, 2 / 3)


def test_two_items_closed_form():
    # one consumer, one real position: item 0 shown with probability x
    r0, r1, e0 = 0.7, 0.4, 1.0
    r = np.array([[r0, r1]])
    for x in (0.1, 0.3, 0.5, 0.8):
        X = np.array([[[x, 1 - x], [1 - x, x]]])
        env = M.item_envy(r, np.array([e0]), X)
        assert abs(env[0] - r0 * e0 * max(0.0, 1 - 2 * x)) < 1e-15
        assert abs(env[1] - r1 * e0 * max(0.0, 2 * x - 1)) < 1e-15


def test_matrix_envy_equals_definition_loops():
    for seed, (U, I, m) in enumerate(((3, 4, 3), (5, 6, 4), (2, 7, 7))):
        rng = np.random.default_rng(10 + seed)
        r = rng.uniform(0.05, 1.0, (U, I))
        e = W.exposure(m).astype(np.float64)
        X = _plan(U, I, m, seed=20 + seed)
        assert np.max(np.abs(M.item_envy(r, e, X) - M.envy_loops(r, e, X))) < 1e-13


def test_metrics_invariant_under_relabelling():
    U, I, m = 6, 8, 5
    rng = np.random.default_rng(3)
    r = rng.uniform(0.05, 1.0, (U, I))
    e = W.exposure(m).astype(np.float64)
    X = _plan(U, I, m, seed=31)
    pu, pi = rng.permutation(U), rng.permutation(I)
    a, b = M.metrics(r, e, X), M.metrics(r[pu][:, pi], e, X[pu][:, pi])
    for k in a:
        assert abs(a[k] - b[k]) < 1e-13
    assert np.max(np.abs(M.item_envy(r, e, X)[pi] - M.item_envy(r[:, pi], e, X[:, pi]))) < 1e-13


def test_impacts_match_the_c_oracle():
    U, I, m = 9, 13, 6
    rng = np.random.default_rng(5)
    r = rng.uniform(0.05, 1.0, (U, I))
    e = W.exposure(m).astype(np.float64)
    X = _plan(U, I, m, seed=41)
    assert np.max(np.abs(M.item_impacts(r, e, X) / oracle.impact(r, e, X) - 1)) < 1e-13
