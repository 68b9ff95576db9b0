"""The loop condition of Algorithm 1 on the GPU: ascend only while
||dF/dC||_F > t (fr_optim.grad_tol), against the FP64 oracle's run with the
same t.  t is placed between gradient norms the oracle reports, with a
relative margin far above FP32 rounding, so both sides stop at the same step."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from gpu_util import F_REL, device_problem, f_err

pytestmark = pytest.mark.gpu
N, T, LR = 6, 30, 0.5


def _setup(fr):
    inst = W.config("C1")
    full = oracle.solve(inst.r, inst.e, float(inst.eps), T, N, rule="gd", lr=LR)
    g = full["gnorm"]
    cands = [k for k in range(1, N) if g[k] < g[:k].min() * (1 - 1e-3)]
    assert cands, g
    j = cands[0]
    t = 0.5 * (g[j] + g[:j].min())
    return inst, j, t, device_problem(fr, inst.r, inst.e, inst.eps, T)


@pytest.mark.parametrize("plain", [False, True])
def test_stop_at_the_oracle_step(fr, plain):
    inst, j, t, p = _setup(fr)
    print(f"case grad-norm stop plain={plain} j={j} t={t:.6g}", flush=True)
    ctx = fr.Context(0)
    run = fr.solve_plain if plain else fr.solve
    res = run(ctx, p, N, LR, rule="gd", grad_tol=t)
    ref = oracle.solve(inst.r, inst.e, float(inst.eps), T, N, rule="gd", lr=LR, grad_tol=t)
    assert ref["updates"] == j and res["updates"] == j
    Fh = res["F_hist"].cpu().numpy()
    assert f_err(Fh, ref["F_hist"], inst.I) <= F_REL
    assert np.all(Fh[j + 1:] == Fh[j])   # C no longer changes after the stop
    C = res["C"].double().cpu().numpy()
    assert np.max(np.abs(C - ref["C"])) <= 1e-5 * np.max(np.abs(ref["C"]))
    assert np.max(np.abs(res["X"].double().cpu().numpy() - ref["X"])) <= 1e-5


def test_stop_before_the_first_update(fr):
    inst, j, t, p = _setup(fr)
    print("case grad-norm stop at C0", flush=True)
    ctx = fr.Context(0)
    res = fr.solve(ctx, p, N, 0.01, grad_tol=1e9)
    assert res["updates"] == 0
    assert float(res["C"].abs().max()) == 0.0
    Fh = res["F_hist"].cpu().numpy()
    assert np.all(Fh == Fh[0])


def test_zero_tolerance_runs_every_step(fr):
    inst, j, t, p = _setup(fr)
    print("case grad-norm stop off", flush=True)
    ctx = fr.Context(0)
    a = fr.solve(ctx, p, N, LR, rule="gd")
    assert a["updates"] == N
    b = fr.solve(ctx, p, N, LR, rule="gd", grad_tol=1e-30)
    assert b["updates"] == N
    assert torch.equal(a["C"], b["C"])
