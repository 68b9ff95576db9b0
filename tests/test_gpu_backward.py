"""Parity of the adjoint backward (fr_backward) and of Algorithm 1 (fr_solve)
against the FP64 oracle."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from gpu_util import F_REL, GRAD_REL, check_forward_at_own_C, device_problem, f_err, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", params=["scaling", "log"])
def ctx(fr, request):
    """Every solve runs with each Sinkhorn form of the forward."""
    c = fr.Context(0)
    c.set_form(request.param)
    return c


def _grad_case(fr, ctx, inst, C, K, launch=None):
    prob = device_problem(fr, inst.r, inst.e, inst.eps, inst.T)
    U, I, m = C.shape
    if launch is not None:
        ctx.set_launch(I, m, *launch)
    Cd = torch.from_numpy(C).cuda()
    out = fr.step(ctx, prob, Cd)
    dC, dr = fr.backward(ctx, prob, Cd, out["imp"], 1.0, want_dr=True, K=K)
    torch.cuda.synchronize()
    X = oracle.forward(C, float(inst.eps), inst.T)
    imp = oracle.impact(inst.r, inst.e, X)
    gC, gr = oracle.grad(inst.r, inst.e, float(inst.eps), inst.T, C, imp=imp)
    dC = dC.cpu().numpy().astype(np.float64)
    dr = dr.cpu().numpy().astype(np.float64)
    errC = np.max(np.abs(dC - gC)) / np.max(np.abs(gC))
    errr = np.max(np.abs(dr - gr)) / np.max(np.abs(gr))
    return errC, errr


@pytest.mark.parametrize("K", [1, 7, 50])
def test_backward_matches_oracle_C1(fr, ctx, K):
    inst = W.config("C1")
    C = W.random_costs(inst.U, inst.I, inst.m, 2 * float(inst.eps), seed=33)
    print(f"case C1 K={K}", flush=True)
    errC, errr = _grad_case(fr, ctx, inst, C, K)
    assert errC <= GRAD_REL and errr <= 1e-5, (errC, errr)


SHAPES = [(6, 100, 10, 64, 2, 1), (6, 100, 10, 16, 8, 9), (3, 300, 20, 320, 1, 1),
          (3, 300, 20, 128, 3, 25), (2, 500, 50, 512, 1, 10), (5, 33, 33, 64, 1, 4),
          (7, 45, 5, 8, 6, 3), (2, 130, 11, 192, 1, 1)]


@pytest.mark.parametrize("U,I,m,L,R,K", SHAPES)
def test_backward_shapes(fr, ctx, U, I, m, L, R, K):
    inst = W.small_instance(U, I, m, seed=7 * I + m, eps=0.05, T=30)
    C = W.random_costs(U, I, m, 0.1, seed=m)
    print(f"case U={U} I={I} m={m} L={L} R={R} K={K}", flush=True)
    errC, errr = _grad_case(fr, ctx, inst, C, K, launch=(L, R))
    assert errC <= GRAD_REL and errr <= 1e-5, (errC, errr)


def test_backward_rows_sum_to_zero(fr, ctx):
    inst = W.config("C2", U=200)
    C = W.random_costs(inst.U, inst.I, inst.m, 2 * float(inst.eps), seed=2)
    prob = device_problem(fr, inst.r, inst.e, inst.eps, inst.T)
    Cd = torch.from_numpy(C).cuda()
    out = fr.step(ctx, prob, Cd)
    dC, _ = fr.backward(ctx, prob, Cd, out["imp"], 1.0, want_dr=False, K=1)
    dC = dC.double().cpu().numpy()
    assert np.max(np.abs(dC.sum(2))) < 1e-5 * np.max(np.abs(dC)) * inst.m


def test_solve_C1_trajectory(fr, ctx):
    inst = W.config("C1")
    prob = device_problem(fr, inst.r, inst.e, inst.eps, inst.T)
    res = fr.solve(ctx, prob, inst.N, float(inst.lr))
    ref = oracle.solve(inst.r, inst.e, float(inst.eps), inst.T, inst.N, lr=float(inst.lr))
    Fh = res["F_hist"].cpu().numpy()
    err = np.max(np.abs(Fh / ref["F_hist"] - 1))
    print("C1 trajectory F rel err", err, flush=True)
    assert err <= F_REL
    Xerr = np.max(np.abs(res["X"].double().cpu().numpy() - ref["X"]))
    print("C1 final X max abs err against the oracle's trajectory", Xerr, flush=True)
    assert Xerr <= 1e-4
    check_forward_at_own_C(fr, ctx, prob, inst.r, inst.e, inst.eps, inst.T, res["C"],
                           X=res["X"], F=Fh[-1])


def test_solve_gd_trajectory(fr, ctx):
    inst = W.small_instance(20, 15, 4, seed=5, eps=0.05, T=60)
    prob = device_problem(fr, inst.r, inst.e, inst.eps, inst.T)
    res = fr.solve(ctx, prob, 20, 0.002, rule="gd")
    ref = oracle.solve(inst.r, inst.e, float(inst.eps), inst.T, 20, rule="gd", lr=0.002)
    Fh = res["F_hist"].cpu().numpy()
    assert np.max(np.abs(Fh / ref["F_hist"] - 1)) <= F_REL
    assert np.max(np.abs(res["X"].double().cpu().numpy() - ref["X"])) <= 1e-5
    assert np.max(np.abs(res["C"].double().cpu().numpy() - ref["C"])) <= 1e-5


def test_solve_resume_matches_single_run(fr, ctx):
    inst = W.small_instance(30, 40, 6, seed=6, eps=0.05, T=30)
    prob = device_problem(fr, inst.r, inst.e, inst.eps, inst.T)
    full = fr.solve(ctx, prob, 6, 0.005)
    a = fr.solve(ctx, prob, 2, 0.005)
    b = fr.solve(ctx, prob, 4, 0.005, C0=a["C"], mom=a["mom"], vel=a["vel"], start_step=2)
    assert torch.equal(b["C"], full["C"])
    assert torch.equal(b["F_hist"], full["F_hist"][2:])
    assert torch.equal(a["F_hist"], full["F_hist"][:3])


def test_plain_form_matches_oracle_and_fused(fr, ctx):
    inst = W.config("C1")
    prob = device_problem(fr, inst.r, inst.e, inst.eps, inst.T)
    res = fr.solve_plain(ctx, prob, 10, float(inst.lr))
    ref = oracle.solve(inst.r, inst.e, float(inst.eps), inst.T, 10, lr=float(inst.lr))
    Fh = res["F_hist"].cpu().numpy()
    assert np.max(np.abs(Fh / ref["F_hist"] - 1)) <= F_REL
    assert np.max(np.abs(res["X"].double().cpu().numpy() - ref["X"])) <= 1e-5
    fused = fr.solve(ctx, prob, 10, float(inst.lr))
    assert np.max(np.abs(fused["F_hist"].cpu().numpy() / Fh - 1)) <= F_REL


def test_solve_timing_mode_matches_graph_mode(fr, ctx):
    import ctypes
    inst = W.config("C1")
    prob = device_problem(fr, inst.r, inst.e, inst.eps, inst.T)
    lib = fr.load()
    lib.fr_ctx_set_timing.argtypes = [ctypes.c_void_p, ctypes.c_int]
    g = fr.solve(ctx, prob, 5, float(inst.lr))
    lib.fr_ctx_set_timing(ctx.handle, 1)
    t = fr.solve(ctx, prob, 5, float(inst.lr))
    lib.fr_ctx_set_timing(ctx.handle, 0)
    assert torch.equal(g["C"], t["C"]) and torch.equal(g["F_hist"], t["F_hist"])


def test_solve_C2_matches_oracle_trajectory(fr, ctx):
    """2000 x 100 x 10, T=200, N=100 Adam steps against the stored FP64
    oracle trajectory (tests/golden/c2_trajectory.json)."""
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "c2_trajectory.json")) as fh:
        gold = json.load(fh)
    inst = W.config("C2")
    prob = device_problem(fr, inst.r, inst.e, inst.eps, inst.T)
    res = fr.solve(ctx, prob, inst.N, float(inst.lr))
    Fh = res["F_hist"].cpu().numpy()
    ref = np.array(gold["F_hist"])
    err = np.max(np.abs(Fh / ref - 1))
    print("C2 trajectory F rel err", err, flush=True)
    assert err <= F_REL
    check_forward_at_own_C(fr, ctx, prob, inst.r, inst.e, inst.eps, inst.T, res["C"],
                           X=res["X"], F=Fh[-1])
    imp_ref = np.array(gold["imp_final"])
    prob_out = fr.nsw(ctx, prob, res["X"])
    imp = prob_out[0].cpu().numpy()
    print("C2 final impacts rel err", np.max(np.abs(imp / imp_ref - 1)), flush=True)
    assert np.max(np.abs(imp / imp_ref - 1)) <= 1e-5


def test_autotune_picks_a_valid_shape_and_keeps_parity(fr):
    ctx = fr.Context(0)
    inst = W.config("C1")
    prob = device_problem(fr, inst.r, inst.e, inst.eps, inst.T)
    L, R = ctx.autotune(prob)
    assert ctx.get_launch(inst.U, inst.I, inst.m) == (L, R) and L * R >= inst.I
    Lb, Rb = ctx.autotune(prob, batched=True)
    assert Lb <= 256 and Lb * Rb >= inst.I
    res = fr.solve(ctx, prob, 5, float(inst.lr))
    ref = oracle.solve(inst.r, inst.e, float(inst.eps), inst.T, 5, lr=float(inst.lr))
    assert np.max(np.abs(res["F_hist"].cpu().numpy() / ref["F_hist"] - 1)) <= F_REL
