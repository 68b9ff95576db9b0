"""Evaluation metrics on the GPU (fr_metrics) against the FP64 oracle
(oracle/metrics.py) on the same FP32 (or BF16) plan: user utility, per-item
and mean max envy, items better / worse off (Section 4.1's metric list).

The plans are the oracle's Sinkhorn plans of seeded random costs, rounded to
the storage type; both sides then work in FP64 from identical inputs, so the
bar is 1e-12 (utility relative, envy relative to max_ij E_ij) and the
better / worse counts are compared exactly where no item lies within 1e-9 of
a threshold."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from gpu_util import device_problem
from oracle import metrics as M

pytestmark = pytest.mark.gpu
TOL = 1e-12


def _case(U, I, m, seed, scale):
    r = W.relevance_lowrank(U, I, 8, 1 / 16, np.random.default_rng(seed))
    e = W.exposure(m)
    C = W.random_costs(U, I, m, scale, seed=seed + 1)
    X = oracle.forward(C, 0.05, 40).astype(np.float32)
    return r, e, X


def _check(fr, r, e, Xs, Xd):
    """Xs: storage tensor handed to the GPU; Xd: the same values in float64."""
    U, I, m = Xd.shape
    ctx = fr.Context(0)
    p = device_problem(fr, r, e, 0.05, 1)
    out, envy, imp = fr.metrics(ctx, p, Xs, per_item=True)
    out, envy, imp = out.cpu().numpy(), envy.cpu().numpy(), imp.cpu().numpy()
    rd, ed = r.astype(np.float64), e.astype(np.float64)
    scale = float(np.max(M.envy_matrix(rd, ed, Xd)))
    imp_ref = M.item_impacts(rd, ed, Xd)
    assert np.max(np.abs(imp - imp_ref)) <= TOL * np.max(imp_ref)
    assert abs(out[0] / M.user_utility(rd, ed, Xd) - 1) <= TOL
    assert np.max(np.abs(envy - M.item_envy(rd, ed, Xd))) <= TOL * scale
    assert abs(out[1] - M.mean_max_envy(rd, ed, Xd)) <= TOL * scale
    if M.threshold_margin(rd, ed, Xd) > 1e-9:
        b, w = M.better_worse(rd, ed, Xd)
        assert (out[2], out[3]) == (b, w)
    return out


@pytest.mark.parametrize("U,I,m,scale", [(300, 150, 8, 0.3), (64, 64, 5, 1.0), (1, 37, 6, 0.5),
                                         (2000, 100, 10, 0.04), (50, 200, 20, 2.0)])
def test_metrics_match_oracle_f32(fr, U, I, m, scale):
    print(f"case metrics f32 U={U} I={I} m={m} scale={scale}", flush=True)
    r, e, X = _case(U, I, m, seed=U + I + m, scale=scale)
    _check(fr, r, e, torch.from_numpy(X).cuda(), X.astype(np.float64))


def test_metrics_match_oracle_bf16(fr):
    print("case metrics bf16 U=300 I=150 m=8", flush=True)
    r, e, X = _case(300, 150, 8, seed=9, scale=0.3)
    Xb = torch.from_numpy(X).to(torch.bfloat16)
    _check(fr, r, e, Xb.cuda(), Xb.float().numpy().astype(np.float64))


def test_hand_worked_policy_on_gpu(fr):
    print("case metrics hand-worked", flush=True)
    r = np.array([[0.9, 0.5, 0.2], [0.8, 0.6, 0.1]], dtype=np.float32)
    e = np.array([1.0], dtype=np.float32)
    X = np.zeros((2, 3, 2), dtype=np.float32)
    X[:, 0, 0] = 1.0
    X[:, 1:, 1] = 1.0
    out = _check(fr, r, e, torch.from_numpy(X).cuda(), X.astype(np.float64))
    assert abs(out[1] - (0.5 + 0.6 + 0.2 + 0.1) / 3) < 1e-7   # envy of items 1 and 2
    assert (out[2], out[3]) == (1 / 3, 2 / 3)


def test_uniform_policy_on_gpu(fr):
    print("case metrics uniform policy", flush=True)
    U, I, m = 40, 70, 6
    r = W.relevance_uniform(U, I, np.random.default_rng(2))
    e = W.exposure(m)
    b = np.ones(m)
    b[-1] = I - m + 1
    X = np.broadcast_to((b / I).astype(np.float32), (U, I, m)).copy()
    out = _check(fr, r, e, torch.from_numpy(X).cuda(), X.astype(np.float64))
    assert out[2] == 0.0 and out[3] == 0.0


def test_plan_not_aligned_to_16_bytes(fr):
    """A plan that starts mid-allocation (a view one consumer in, 37 * 6 * 4 =
    888 bytes, not a multiple of 16) takes the element-wise staging path."""
    print("case metrics unaligned plan", flush=True)
    U, I, m = 41, 37, 6
    r, e, X = _case(U, I, m, seed=17, scale=0.5)
    Xd = torch.from_numpy(X).cuda()
    view = Xd[1:]
    assert view.data_ptr() % 16 != 0
    _check(fr, np.ascontiguousarray(r[1:]), e, view, X[1:].astype(np.float64))
