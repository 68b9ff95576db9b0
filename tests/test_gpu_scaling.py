"""The scaling form of the Sinkhorn forward (fr_ctx_set_form FR_FORM_SCALING,
the default) against the FP64 oracle, with its absorption forced.  It computes the same T iterates as the log-domain
form (Section 3's Sinkhorn iteration from g = 0), so the oracle and the bars
are those of the log-domain forward: plans 1e-5, F 1e-6, impacts 2e-6.

Absorption of the scalings into the potentials is exercised three ways: on
its range test alone, forced every iteration, and forced every fifth
iteration; and on costs whose column scalings cross 2^32 in the first
iteration."""
import json
import os

import numpy as np
import pytest
import torch

import oracle
import workloads as W
from gpu_util import (F_REL, GRAD_REL, IMP_REL, X_ABS, assert_step_close, device_problem,
                      f_err, oracle_step)
from test_gpu_forward import SHAPES

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(fr):
    return fr.Context(0)


def _step(fr, ctx, inst, C, absorb, launch=None, x_dtype="f32", T=None):
    ctx.set_form("scaling", absorb)
    prob = device_problem(fr, inst.r, inst.e, inst.eps, inst.T if T is None else T)
    U, I, m = C.shape
    if launch is not None:
        ctx.set_launch(I, m, *launch)
    out = fr.step(ctx, prob, torch.from_numpy(C).cuda(), want_X=True, x_dtype=x_dtype,
                  want_pot=True)
    torch.cuda.synchronize()
    return out


@pytest.mark.parametrize("absorb", [0, 1, 5])
@pytest.mark.parametrize("U,I,m,L,R", SHAPES)
def test_scaling_step_shapes(fr, ctx, U, I, m, L, R, absorb):
    inst = W.small_instance(U, I, m, seed=U * 1000 + I + m, eps=0.05, T=40)
    C = W.random_costs(U, I, m, 0.1, seed=I + m)
    print(f"case scaling U={U} I={I} m={m} L={L} R={R} absorb={absorb}", flush=True)
    try:
        out = _step(fr, ctx, inst, C, absorb, launch=(L, R))
    except fr.FairRankError as ex:
        if ex.code == 8:
            pytest.skip(f"launch ({L},{R}) not instantiated for m={m}")
        raise
    X_ref, imp_ref, F_ref = oracle_step(inst.r, inst.e, inst.eps, inst.T, C)
    assert_step_close(out, X_ref, imp_ref, F_ref)
    pot = out["pot"].cpu().numpy().astype(np.float64)
    f, g = pot[:, :I], pot[:, I:]
    Xp = np.exp((f[:, :, None] + g[:, None, :] - C.astype(np.float64)) / float(inst.eps))
    assert np.max(np.abs(Xp - X_ref)) < 1e-4


@pytest.mark.parametrize("which,scale", [("C1", 2.0), ("C2", 2.0)])
def test_scaling_step_workloads(fr, ctx, which, scale):
    inst = W.config(which)
    C = W.random_costs(inst.U, inst.I, inst.m, scale * float(inst.eps), seed=33)
    print(f"case scaling {which} scale {scale}", flush=True)
    out = _step(fr, ctx, inst, C, 0)
    X_ref, imp_ref, F_ref = oracle_step(inst.r, inst.e, inst.eps, inst.T, C)
    assert_step_close(out, X_ref, imp_ref, F_ref)


# Exponents here reach |z| ~ 64 (costs spread over 60 log2 units, potentials
# compensating), where half an FP32 ulp is 2^-19 of absolute error, i.e.
# 2^-19 ln 2 ~ 1.3e-6 relative in x per rounding: four roundings bound the
# impacts for either form.
WIDE_RANGE_IMP = 4 * 2.0 ** -19 * np.log(2.0)


@pytest.mark.parametrize("U,I,m", [(40, 30, 5), (6, 200, 12), (3, 600, 40)])
def test_absorption_on_range(fr, ctx, U, I, m):
    """Column costs rising by 60 log2 units over the positions: after the first
    row half-step the dummy column's scaling is ~2^60, beyond the range.  The
    log-domain form runs on the same input against the same bar."""
    inst = W.small_instance(U, I, m, seed=7 + m, eps=0.05, T=60)
    lin = np.arange(m) / (m - 1) * 60.0 * float(np.float32(inst.eps)) * np.log(2.0)
    C = (W.random_costs(U, I, m, 0.05, seed=m) + lin[None, None, :]).astype(np.float32)
    print(f"case scaling range absorption U={U} I={I} m={m}", flush=True)
    X_ref, imp_ref, F_ref = oracle_step(inst.r, inst.e, inst.eps, inst.T, C)
    for form in ("scaling", "log"):
        out = _step(fr, ctx, inst, C, 0)
        if form == "log":
            ctx.set_form("log")
            prob = device_problem(fr, inst.r, inst.e, inst.eps, inst.T)
            out = fr.step(ctx, prob, torch.from_numpy(C).cuda(), want_X=True)
        imp = out["imp"].cpu().numpy()
        e_imp = np.max(np.abs(imp / imp_ref - 1))
        print(f"  {form}: imp {e_imp:.3g} (bar {WIDE_RANGE_IMP:.3g})", flush=True)
        assert e_imp <= WIDE_RANGE_IMP
        assert f_err(float(out["F"].cpu()[0]), F_ref, I) <= F_REL
        assert np.max(np.abs(out["X"].double().cpu().numpy() - X_ref)) <= X_ABS


def test_scaling_bf16_and_subsample(fr, ctx):
    g = np.load(os.path.join(os.path.dirname(__file__), "golden", "c5_sub.npz"))
    inst = W.config("C5")
    print("case scaling C5 subsample forward bf16", flush=True)
    ctx.set_form("scaling", 0)
    prob = device_problem(fr, inst.r[g["users"]], inst.e, inst.eps, inst.T)
    C = torch.from_numpy(W.random_costs(1000, inst.I, inst.m, 2 * float(inst.eps), seed=56)).cuda()
    out = fr.step(ctx, prob, C, want_X=True, x_dtype="bf16")
    assert np.max(np.abs(out["imp"].cpu().numpy() / g["rand_imp"] - 1)) <= IMP_REL
    assert abs(float(out["F"].cpu()[0]) / float(g["rand_F"][0]) - 1) <= F_REL
    X = out["X"][torch.from_numpy(g["sel"]).long()].float().cpu().numpy()
    Xr = g["rand_X_sel"].astype(np.float64)
    assert np.all(np.abs(X - Xr) <= 2.0 ** -8 * np.abs(Xr) + X_ABS)


def test_scaling_solve_C2_trajectory(fr, ctx):
    """The full 2000 x 100 x 10 solve (T 200, 100 Adam steps) with the scaling
    forward absorbing every fourth iteration and the log-domain reverse sweep,
    against the stored FP64 oracle trajectory."""
    with open(os.path.join(os.path.dirname(__file__), "golden", "c2_trajectory.json")) as fh:
        gold = json.load(fh)
    inst = W.config("C2")
    print("case scaling C2 solve, absorbing every 4th iteration", flush=True)
    ctx.set_form("scaling", 4)
    prob = device_problem(fr, inst.r, inst.e, inst.eps, inst.T)
    res = fr.solve(ctx, prob, inst.N, float(inst.lr))
    Fh = res["F_hist"].cpu().numpy()
    err = np.max(np.abs(Fh / np.array(gold["F_hist"]) - 1))
    print("  F rel err", err, flush=True)
    assert err <= F_REL


def test_scaling_solve_gd_matches_oracle(fr, ctx):
    inst = W.small_instance(20, 15, 4, seed=5, eps=0.05, T=60)
    print("case scaling GD solve", flush=True)
    ctx.set_form("scaling", 3)
    prob = device_problem(fr, inst.r, inst.e, inst.eps, inst.T)
    res = fr.solve(ctx, prob, 20, 0.002, rule="gd")
    ref = oracle.solve(inst.r, inst.e, float(inst.eps), inst.T, 20, rule="gd", lr=0.002)
    assert np.max(np.abs(res["F_hist"].cpu().numpy() / ref["F_hist"] - 1)) <= F_REL
    assert np.max(np.abs(res["X"].double().cpu().numpy() - ref["X"])) <= X_ABS
    assert np.max(np.abs(res["C"].double().cpu().numpy() - ref["C"])) <= 1e-5


def test_form_validation(fr, ctx):
    with pytest.raises(fr.FairRankError):
        ctx.set_form("scaling", -1)
    import ctypes
    lib = fr.load()
    assert lib.fr_ctx_set_form(ctx.handle, 7, 0) == 3
    assert lib.fr_ctx_set_form(None, 0, 0) == 1


@pytest.mark.parametrize("absorb", [0, 1, 6])
@pytest.mark.parametrize("U,I,m,L,R", [(37, 23, 5, 8, 3), (5, 100, 10, 64, 2), (6, 100, 10, 128, 1),
                                       (3, 300, 20, 128, 3), (2, 257, 13, 64, 6)])
def test_scaling_reverse_sweep_matches_oracle(fr, ctx, U, I, m, L, R, absorb):
    """The reverse sweep in the scaling form (K = 1), its reference rebased on
    the range test alone, every iteration, or every sixth, against the oracle's
    reverse mode."""
    inst = W.small_instance(U, I, m, seed=U + 7 * I + m, eps=0.05, T=40)
    C = W.random_costs(U, I, m, 0.1, seed=3 * I + m)
    print(f"case scaling backward U={U} I={I} m={m} L={L} R={R} absorb={absorb}", flush=True)
    ctx.set_form("scaling", absorb)
    try:
        ctx.set_launch(I, m, L, R)
    except fr.FairRankError as ex:
        if ex.code == 8:
            pytest.skip(f"launch ({L},{R}) not instantiated for m={m}")
        raise
    prob = device_problem(fr, inst.r, inst.e, inst.eps, inst.T)
    Cd = torch.from_numpy(C).cuda()
    out = fr.step(ctx, prob, Cd)
    dC, dr = fr.backward(ctx, prob, Cd, out["imp"], 1.0, K=1)
    gC, gr = oracle.grad(inst.r, inst.e, float(inst.eps), inst.T, C)
    scale = np.max(np.abs(gC))
    assert np.max(np.abs(dC.double().cpu().numpy() - gC)) <= GRAD_REL * scale
    assert np.max(np.abs(dr.double().cpu().numpy() - gr)) <= 1e-5 * np.max(np.abs(gr))
