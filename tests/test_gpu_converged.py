"""The converged-map form of Algorithm 1 on the GPU (fr_grad_converged, and
fr_solve with fr_optim.sinkhorn_tol > 0) against the FP64 oracle
(oracle/warm.py): Sinkhorn run to a potential-change tolerance from warm
starts, and dF/dC of the converged plan by the implicit function theorem.

Both sides stop on the same rule, but a stopped iterate is only within the
tolerance's reach of the exact entropic plan.  The GPU is therefore compared
with the oracle's exact plan (tolerance 1e-12) and allowed three times the
distance the oracle's own run at the GPU's tolerance keeps from it, plus an
FP32 floor: impacts 1e-5 relative, gradients 5e-4 of the
largest entry (the FP32 conjugate-gradient solve of the Schur system stops
at a relative residual of 1e-6 or after 2m + 8 steps)."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from gpu_util import device_problem, f_err
from oracle import warm

pytestmark = pytest.mark.gpu
TOL = 3e-5
T_MAX = 20000
IMP_FLOOR, G_FLOOR = 1e-5, 5e-4


def _exact(C, eps, tol=1e-12):
    U, I, m = C.shape
    X, _, it = oracle.forward_warm(C, eps, np.zeros((U, m)), tol, 200000)
    return X, it


@pytest.mark.parametrize("U,I,m,eps,scale,seed", [(50, 20, 5, 0.05, 0.3, 1), (7, 37, 6, 0.05, 0.3, 2),
                                                  (40, 100, 10, 0.02, 0.1, 3),
                                                  (12, 300, 20, 0.02, 0.1, 4),
                                                  (3, 1000, 50, 0.05, 0.3, 5)])
def test_implicit_gradient_matches_oracle(fr, U, I, m, eps, scale, seed):
    print(f"case converged grad U={U} I={I} m={m} eps={eps} scale={scale}", flush=True)
    rng = np.random.default_rng(seed)
    r = W.relevance_lowrank(U, I, 4, 0.25, rng)
    e = W.exposure(m)
    C = W.random_costs(U, I, m, scale, seed=seed + 10)
    rd, ed, Cd = r.astype(np.float64), e.astype(np.float64), C.astype(np.float64)
    X_ex, it_ex = _exact(Cd, float(np.float32(eps)))
    assert np.all(it_ex < 200000)
    imp_ex = oracle.impact(rd, ed, X_ex)
    g_ex = warm.grad_implicit(rd, ed, float(np.float32(eps)), X_ex, imp_ex)
    X_t, _ = _exact(Cd, float(np.float32(eps)), TOL)
    imp_t = oracle.impact(rd, ed, X_t)
    g_t = warm.grad_implicit(rd, ed, float(np.float32(eps)), X_t, imp_t)

    ctx = fr.Context(0)
    p = device_problem(fr, r, e, eps, T_MAX)
    gF = 0.75
    out = fr.grad_converged(ctx, p, torch.from_numpy(C).cuda(), TOL, gF=gF)
    imp = out["imp"].cpu().numpy()
    dC = out["dC"].double().cpu().numpy() / gF
    dr = out["dr"].double().cpu().numpy() / gF

    e_imp = np.max(np.abs(imp / imp_ex - 1))
    b_imp = 3 * np.max(np.abs(imp_t / imp_ex - 1)) + IMP_FLOOR
    gmax = np.max(np.abs(g_ex))
    e_g = np.max(np.abs(dC - g_ex)) / gmax
    b_g = 3 * np.max(np.abs(g_t - g_ex)) / gmax + G_FLOOR
    dr_ex = (X_ex[:, :, : m - 1] @ ed) / imp_ex[None, :]
    e_dr = np.max(np.abs(dr - dr_ex)) / np.max(np.abs(dr_ex))
    print(f"  imp {e_imp:.3g} (bar {b_imp:.3g})  dC {e_g:.3g} (bar {b_g:.3g})  dr {e_dr:.3g}",
          flush=True)
    assert e_imp <= b_imp
    assert f_err(float(out["F"].cpu()[0]), oracle.nsw(imp_ex), I) <= b_imp
    assert e_g <= b_g
    assert e_dr <= b_imp + 1e-6
    # shifting a row of C leaves the converged plan unchanged
    assert np.max(np.abs(dC.sum(2))) <= G_FLOOR * gmax


@pytest.mark.parametrize("rule,lr", [("gd", 0.5), ("adam", 0.005)])
def test_converged_map_solve_matches_oracle(fr, rule, lr):
    inst = W.config("C1")
    N = 5
    print(f"case converged solve C1 rule={rule} N={N}", flush=True)
    eps = float(inst.eps)
    ref = warm.solve_warm(inst.r, inst.e, eps, T_MAX, TOL, N, rule=rule, lr=lr)
    ctx = fr.Context(0)
    p = device_problem(fr, inst.r, inst.e, inst.eps, T_MAX)
    res = fr.solve(ctx, p, N, lr, rule=rule, sinkhorn_tol=TOL)
    Fh = res["F_hist"].cpu().numpy()
    ef = f_err(Fh, ref["F_hist"], inst.I)
    iters, iters_ref = res["sinkhorn_iters"], int(ref["iters"].sum())
    print(f"  F {ef:.3g}  sinkhorn iterations {iters} (oracle {iters_ref})", flush=True)
    assert ef <= 1e-5
    assert abs(iters - iters_ref) <= 0.25 * iters_ref
    if rule == "gd":
        C = res["C"].double().cpu().numpy()
        assert np.max(np.abs(C - ref["C"])) <= 2e-3 * np.max(np.abs(ref["C"]))
        assert np.max(np.abs(res["X"].double().cpu().numpy() - ref["X"])) <= 1e-4


def test_converged_map_needs_the_fused_single_instance_path(fr):
    inst = W.config("C1")
    print("case converged form unsupported paths", flush=True)
    ctx = fr.Context(0)
    p = device_problem(fr, inst.r, inst.e, inst.eps, 100)
    with pytest.raises(fr.FairRankError):
        fr._solve(fr.load().fr_solve_plain, ctx, p, 2, 0.1, "gd", 0.9, 0.999, 1e-8, None, None,
                  None, 0, 1, True, "f32", True, 0.0, TOL, 0)
