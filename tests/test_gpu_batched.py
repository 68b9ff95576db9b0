"""Batched solver (fr_solve_batched): uneven instances in persistent kernels.
Each instance must equal the single-instance solver run with the same launch
shape, and the FP64 oracle."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from gpu_util import F_REL, X_ABS, check_forward_at_own_C, device_problem, f_err

pytestmark = pytest.mark.gpu


def _instances():
    # the batched workload's generator at smaller U, plus ragged extremes
    shapes = W.batched_shapes(128, seed=4)[:12]
    out = [W.batched_instance(j, (min(U, 150), I, m), T=40, N=6)
           for j, (U, I, m) in enumerate(shapes)]
    out.append(W.small_instance(3, 7, 7, seed=91, eps=0.03, T=40, N=6))
    out.append(W.small_instance(1, 2, 2, seed=92, eps=0.03, T=40, N=6))
    return out


def _pin_launch(ctx, insts):
    """Same team shape for the batched and the single-instance kernels."""
    for x in insts:
        ctx.set_launch(x.I, x.m, 256, 1 if x.I <= 256 else 2)


@pytest.fixture(scope="module")
def adam_run(fr):
    insts = _instances()
    ctx = fr.Context(0)
    _pin_launch(ctx, insts)
    probs = [device_problem(fr, x.r, x.e, x.eps, x.T) for x in insts]
    print("case batched Adam solve of", len(insts), "instances", flush=True)
    res = fr.solve_batched(ctx, probs, 6, 0.003)
    torch.cuda.synchronize()
    return insts, probs, res, ctx


def test_batched_equals_single_instance_solver(fr, adam_run):
    insts, probs, res, ctx = adam_run
    for j, (x, p) in enumerate(zip(insts, probs)):
        print(f"case instance {j} U={x.U} I={x.I} m={x.m}", flush=True)
        one = fr.solve(ctx, p, 6, 0.003)
        assert torch.equal(res[j]["C"], one["C"])
        assert torch.equal(res[j]["X"], one["X"])
        assert torch.equal(res[j]["mom"], one["mom"]) and torch.equal(res[j]["vel"], one["vel"])
        Fb = res[j]["F_hist"].cpu().numpy()
        Fs = one["F_hist"].cpu().numpy()
        assert np.max(np.abs(Fb / Fs - 1)) <= 1e-14


def test_batched_log_form_equals_single_instance_solver(fr):
    """With the log-domain forward selected, the batched kernels run it too."""
    insts = _instances()[:4] + _instances()[12:]
    ctx = fr.Context(0)
    ctx.set_form("log")
    _pin_launch(ctx, insts)
    probs = [device_problem(fr, x.r, x.e, x.eps, x.T) for x in insts]
    print("case batched log-domain solve of", len(insts), "instances", flush=True)
    res = fr.solve_batched(ctx, probs, 3, 0.003)
    for j, p in enumerate(probs):
        one = fr.solve(ctx, p, 3, 0.003)
        assert torch.equal(res[j]["C"], one["C"])
        assert torch.equal(res[j]["F_hist"], one["F_hist"])


@pytest.mark.parametrize("j", [0, 3, 7, 12, 13])
def test_batched_adam_objective_matches_oracle(fr, adam_run, j):
    """F history against the oracle's Adam trajectory, and the forward at the
    GPU's own final C (plan, impacts and F).  Under Adam the trajectory itself
    is ill-conditioned (entries whose exact gradient is ~0 take sign-like
    steps from rounding noise), so plans and impacts are compared where they
    are well conditioned: at identical C."""
    insts, probs, res, ctx = adam_run
    x = insts[j]
    print(f"case oracle Adam instance {j} U={x.U} I={x.I} m={x.m}", flush=True)
    ref = oracle.solve(x.r, x.e, float(x.eps), x.T, 6, lr=0.003)
    Fb = res[j]["F_hist"].cpu().numpy()
    assert f_err(Fb, ref["F_hist"], x.I) <= F_REL
    check_forward_at_own_C(fr, ctx, probs[j], x.r, x.e, x.eps, x.T, res[j]["C"],
                           X=res[j]["X"], F=Fb[-1])


@pytest.mark.parametrize("j", [0, 7, 12])
def test_batched_gradient_ascent_matches_oracle(fr, j):
    """Plain ascent is well conditioned: costs and plans follow the oracle's
    trajectory to the single-instance bars."""
    insts = _instances()
    ctx = fr.Context(0)
    _pin_launch(ctx, insts)
    probs = [device_problem(fr, x.r, x.e, x.eps, x.T) for x in insts]
    res = fr.solve_batched(ctx, probs, 4, 0.5, rule="gd")
    x = insts[j]
    print(f"case oracle GD instance {j} U={x.U} I={x.I} m={x.m}", flush=True)
    ref = oracle.solve(x.r, x.e, float(x.eps), x.T, 4, rule="gd", lr=0.5)
    assert f_err(res[j]["F_hist"].cpu().numpy(), ref["F_hist"], x.I) <= F_REL
    C = res[j]["C"].double().cpu().numpy()
    Cref = ref["C"]
    cerr = float(np.max(np.abs(C - Cref)) / np.max(np.abs(Cref)))
    X = res[j]["X"].double().cpu().numpy()
    xerr = float(np.max(np.abs(X - ref["X"])))
    print(f"  C error {cerr:.3e} of max |C|, X error {xerr:.3e}", flush=True)
    check_forward_at_own_C(fr, ctx, probs[j], x.r, x.e, x.eps, x.T, res[j]["C"], X=res[j]["X"])
    assert cerr <= 1e-5, cerr
    assert xerr <= X_ABS, xerr


def test_batched_ignores_team_widths_that_do_not_tile_its_blocks(fr):
    """A 192-lane team does not divide the batched kernels' 256-thread blocks;
    the batched path must fall back to a tiling shape (it once ran a phantom
    partial team on such a request)."""
    x = W.batched_instance(19, (300, 319, 41), T=30, N=2)
    ctx = fr.Context(0)
    ctx.set_launch(x.I, x.m, 192, 2)
    p = device_problem(fr, x.r, x.e, x.eps, x.T)
    b = fr.solve_batched(ctx, [p], 2, 0.003)
    one = fr.solve(ctx, p, 2, 0.003)
    Fb, Fs = b[0]["F_hist"].cpu().numpy(), one["F_hist"].cpu().numpy()
    # different launch shapes sum in different orders; Adam's first steps
    # turn rounding-level gradient differences into lr-sized cost changes
    assert np.all(np.isfinite(Fb)) and f_err(Fb, Fs, x.I) <= F_REL
