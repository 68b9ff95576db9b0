"""The baseline rankings on the GPU (fr_rank_maxrele, fr_rank_greedy) against
the FP64 oracle (oracle/baselines.py).  Selections are integer results and
must agree exactly; greedy decisions compare FP64 ratios r_ui / Imp_i formed
the same way on both sides, and its impacts are FP64 sums in the same
decision order, so they agree exactly too.  Plans are compared exactly."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from gpu_util import device_problem
from oracle import baselines as B
from oracle import metrics as M

pytestmark = pytest.mark.gpu

# (U, I, m, seed): ragged item counts, one consumer, m = I, the widest case
CASES = [(50, 20, 5, 1), (37, 23, 5, 2), (5, 100, 10, 3), (200, 300, 20, 4), (3, 1000, 50, 5),
         (1, 10, 10, 6), (1, 70, 3, 7), (2, 4096, 64, 8), (640, 65, 11, 9)]


def _inst(U, I, m, seed):
    rng = np.random.default_rng(seed)
    r = W.relevance_lowrank(U, I, 4, 0.25, rng)
    return r, W.exposure(m)


@pytest.fixture(scope="module")
def ctx(fr):
    return fr.Context(0)


@pytest.mark.parametrize("U,I,m,seed", CASES)
def test_maxrele_matches_oracle(fr, ctx, U, I, m, seed):
    print(f"case maxrele U={U} I={I} m={m}", flush=True)
    r, e = _inst(U, I, m, seed)
    out = fr.rank_maxrele(ctx, device_problem(fr, r, e, 0.05, 1))
    sel = out["sel"].cpu().numpy()
    ref = B.maxrele(r, m)
    assert np.array_equal(sel, ref)
    assert np.array_equal(out["X"].cpu().numpy().astype(np.float64), B.plan_from_selection(ref, I))


@pytest.mark.parametrize("U,I,m,seed", CASES)
def test_greedy_matches_oracle(fr, ctx, U, I, m, seed):
    print(f"case greedy U={U} I={I} m={m}", flush=True)
    r, e = _inst(U, I, m, seed)
    out = fr.rank_greedy(ctx, device_problem(fr, r, e, 0.05, 1))
    sel = out["sel"].cpu().numpy()
    ref, imp_ref = B.greedy(r, e)
    assert np.array_equal(sel, ref)
    assert np.array_equal(out["imp"].cpu().numpy(), imp_ref)
    assert np.array_equal(out["X"].cpu().numpy().astype(np.float64), B.plan_from_selection(ref, I))


def test_ties_on_gpu(fr, ctx):
    print("case baselines with tied relevances", flush=True)
    r = np.tile(np.array([0.5, 0.7, 0.5, 0.7, 0.1, 0.7], dtype=np.float32), (9, 1))
    e = W.exposure(4)
    p = device_problem(fr, r, e, 0.05, 1)
    assert np.array_equal(fr.rank_maxrele(ctx, p)["sel"].cpu().numpy(), B.maxrele(r, 4))
    g = fr.rank_greedy(ctx, p)
    ref, imp_ref = B.greedy(r, e)
    assert np.array_equal(g["sel"].cpu().numpy(), ref)
    assert np.array_equal(g["imp"].cpu().numpy(), imp_ref)


def test_bf16_plans_and_metrics(fr, ctx):
    """The baselines' plans in BF16 (0 and 1 are exact) and their evaluation
    metrics on the GPU against the oracle's metrics of the oracle's plan."""
    print("case baselines bf16 plans and metrics", flush=True)
    inst = W.config("C2", U=300)
    p = device_problem(fr, inst.r, inst.e, inst.eps, 1)
    rd, ed = inst.r.astype(np.float64), inst.e.astype(np.float64)
    for name, run, ref_sel in (("maxrele", fr.rank_maxrele, B.maxrele(inst.r, inst.m)),
                               ("greedy", fr.rank_greedy, B.greedy(inst.r, inst.e)[0])):
        out = run(ctx, p, x_dtype="bf16")
        Xref = B.plan_from_selection(ref_sel, inst.I)
        assert np.array_equal(out["X"].float().cpu().numpy().astype(np.float64), Xref), name
        met = fr.metrics(ctx, p, out["X"]).cpu().numpy()
        scale = float(np.max(M.envy_matrix(rd, ed, Xref)))
        assert abs(met[0] / M.user_utility(rd, ed, Xref) - 1) <= 1e-12
        assert abs(met[1] - M.mean_max_envy(rd, ed, Xref)) <= 1e-12 * scale
        b, w = M.better_worse(rd, ed, Xref)
        assert (met[2], met[3]) == (b, w)


def test_baseline_argument_errors(fr, ctx):
    lib = fr.load()
    inst = W.small_instance(4, 6, 3, seed=1)
    p = device_problem(fr, inst.r, inst.e, inst.eps, 1).c()
    import ctypes
    assert lib.fr_rank_maxrele(ctx.handle, ctypes.byref(p), None, None, 0, None) == 1
    assert lib.fr_rank_greedy(None, ctypes.byref(p), None, None, 0, None, None) == 1
    sel = torch.empty((4, 2), dtype=torch.int32, device="cuda")
    assert lib.fr_rank_greedy(ctx.handle, ctypes.byref(p), ctypes.c_void_p(sel.data_ptr()), None,
                              5, None, None) == 3
