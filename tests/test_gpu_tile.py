"""Tile kernels of large plans (512 < |I| <= 1024 items, 40 <= m <= 50
columns; the 100000 x 1000 x 50 workload's plans): scaling-form forward on
2-D lane tiles, and the reverse sweep whose cost adjoint is contracted on the
matrix cores from per-iteration row and column factors, with the row
scalings kept by the forward (row store, the default) or formed by the sweep.
Parity with the FP64 oracle (Section 3 forward and chain rule, Eqs. Imp and
objF), with the reference kernel rebased on range and by a forced period
(several stretches per consumer), Adam and plain-ascent trajectories, and the
error raised when a consumer needs more stretches than the sweep keeps."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from gpu_util import (F_REL, GRAD_REL, IMP_REL, X_ABS, check_forward_at_own_C, device_problem,
                      f_err)

pytestmark = pytest.mark.gpu

SHAPES = [(3, 1000, 50), (2, 1024, 48), (4, 513, 40), (2, 700, 41)]


def _ctx(fr, absorb=0, store=True):
    ctx = fr.Context(0)
    ctx.set_form("scaling", absorb)
    ctx.set_row_store(store)
    return ctx


@pytest.mark.parametrize("U,I,m", SHAPES)
@pytest.mark.parametrize("absorb", [0, 7])
def test_tile_forward_matches_oracle(fr, U, I, m, absorb):
    print(f"case tile forward U={U} I={I} m={m} absorb={absorb}", flush=True)
    inst = W.small_instance(U, I, m, seed=I + m, eps=0.02, T=60, kind="lowrank")
    ctx = _ctx(fr, absorb)
    assert ctx.get_launch(U, I, m) == (512, 0)
    prob = device_problem(fr, inst.r, inst.e, inst.eps, inst.T)
    C = W.random_costs(U, I, m, 0.04, seed=I)
    out = fr.step(ctx, prob, torch.from_numpy(C).cuda(), want_X=True, want_pot=True)
    X, f, g = oracle.forward(C, float(inst.eps), inst.T, want_potentials=True)
    imp = oracle.impact(inst.r, inst.e, X)
    xerr = float(np.max(np.abs(out["X"].double().cpu().numpy() - X)))
    ierr = float(np.max(np.abs(out["imp"].cpu().numpy() / imp - 1)))
    print(f"  X {xerr:.3e} Imp {ierr:.3e}", flush=True)
    assert xerr <= X_ABS and ierr <= IMP_REL
    assert f_err(float(out["F"].cpu()[0]), oracle.nsw(imp), I) <= F_REL
    # potentials in cost units: the plan they define is the plan
    pot = out["pot"].double().cpu().numpy()
    fg = pot[:, :I, None] + pot[:, None, I:] - C.astype(np.float64)
    Xp = np.exp(fg / float(inst.eps))
    assert np.max(np.abs(Xp - X)) <= 5 * X_ABS


@pytest.mark.parametrize("U,I,m", SHAPES)
@pytest.mark.parametrize("absorb", [0, 5])
@pytest.mark.parametrize("store", [True, False])
def test_tile_backward_matches_oracle(fr, U, I, m, absorb, store):
    """dF/dC and dF/dr through the T unrolled iterations; absorb = 5 rebases
    the reference every 5 iterations (12 stretches at T = 60): the forward's
    with the row store, the sweep's own without it."""
    print(f"case tile backward U={U} I={I} m={m} absorb={absorb} store={store}", flush=True)
    inst = W.small_instance(U, I, m, seed=I + m + 1, eps=0.02, T=60, kind="lowrank")
    ctx = _ctx(fr, absorb, store)
    prob = device_problem(fr, inst.r, inst.e, inst.eps, inst.T)
    C = W.random_costs(U, I, m, 0.04, seed=I + 1)
    Cd = torch.from_numpy(C).cuda()
    out = fr.step(ctx, prob, Cd)
    dC, dr = fr.backward(ctx, prob, Cd, out["imp"], 1.0, want_dr=True, K=1)
    gC, gr = oracle.grad(inst.r, inst.e, float(inst.eps), inst.T, C)
    cerr = float(np.max(np.abs(dC.double().cpu().numpy() - gC)) / np.max(np.abs(gC)))
    rerr = float(np.max(np.abs(dr.double().cpu().numpy() - gr)) / np.max(np.abs(gr)))
    print(f"  dC {cerr:.3e} of max, dr {rerr:.3e} of max", flush=True)
    assert cerr <= GRAD_REL and rerr <= 1e-5


def test_tile_backward_scales_with_gF(fr):
    U, I, m = 2, 800, 45
    inst = W.small_instance(U, I, m, seed=3, eps=0.03, T=40, kind="lowrank")
    ctx = _ctx(fr)
    prob = device_problem(fr, inst.r, inst.e, inst.eps, inst.T)
    Cd = torch.from_numpy(W.random_costs(U, I, m, 0.05, seed=4)).cuda()
    out = fr.step(ctx, prob, Cd)
    d1, _ = fr.backward(ctx, prob, Cd, out["imp"], 1.0, want_dr=False, K=1)
    # a positive power of two scales every product and every rounding
    # exactly: the results are bitwise 2 d1
    d2, _ = fr.backward(ctx, prob, Cd, out["imp"], 2.0, want_dr=False, K=1)
    assert torch.equal(d2, 2.0 * d1)
    # the BF16 matrix products round a sum and its negation differently (by
    # about an ulp), so gF = -1 gives -d1 to the contraction's rounding
    d3, _ = fr.backward(ctx, prob, Cd, out["imp"], -1.0, want_dr=False, K=1)
    assert float((d3 + d1).abs().max()) <= 1e-6 * float(d1.abs().max())


@pytest.mark.parametrize("rule", ["gd", "adam"])
@pytest.mark.parametrize("store", [True, False])
def test_tile_solve_matches_oracle(fr, rule, store):
    """Algorithm 1 on tile plans: GD is well conditioned (costs and plans to
    1e-5); Adam is compared through F and the forward at the GPU's own C."""
    U, I, m, T, N = 4, 600, 40, 40, 5
    print(f"case tile solve {rule} store={store}", flush=True)
    inst = W.small_instance(U, I, m, seed=11, eps=0.03, T=T, kind="lowrank")
    ctx = _ctx(fr, 0, store)
    prob = device_problem(fr, inst.r, inst.e, inst.eps, T)
    lr = 0.002 if rule == "gd" else 0.003   # GD: F rises monotonically (oracle)
    res = fr.solve(ctx, prob, N, lr, rule=rule)
    ref = oracle.solve(inst.r, inst.e, float(inst.eps), T, N, rule=rule, lr=lr)
    assert f_err(res["F_hist"].cpu().numpy(), ref["F_hist"], I) <= F_REL
    if rule == "gd":
        C = res["C"].double().cpu().numpy()
        cerr = float(np.max(np.abs(C - ref["C"])) / np.max(np.abs(ref["C"])))
        xerr = float(np.max(np.abs(res["X"].double().cpu().numpy() - ref["X"])))
        print(f"  C {cerr:.3e} of max, X {xerr:.3e}", flush=True)
        assert cerr <= 1e-5 and xerr <= X_ABS
    check_forward_at_own_C(fr, ctx, prob, inst.r, inst.e, inst.eps, T, res["C"], X=res["X"],
                           F=res["F_hist"].cpu().numpy()[-1])


def test_tile_solve_is_deterministic_and_resumable(fr):
    U, I, m = 3, 900, 50
    inst = W.small_instance(U, I, m, seed=12, eps=0.02, T=30, kind="lowrank")
    ctx = _ctx(fr)
    prob = device_problem(fr, inst.r, inst.e, inst.eps, inst.T)
    a = fr.solve(ctx, prob, 4, 0.002)
    b = fr.solve(ctx, prob, 4, 0.002)
    assert torch.equal(a["C"], b["C"]) and torch.equal(a["F_hist"], b["F_hist"])
    h = fr.solve(ctx, prob, 2, 0.002)
    c = fr.solve(ctx, prob, 2, 0.002, C0=h["C"], mom=h["mom"], vel=h["vel"], start_step=2)
    assert torch.equal(c["C"], a["C"]) and torch.equal(c["F_hist"], a["F_hist"][2:])


def test_tile_matches_pinned_kernels(fr):
    """The same problem on the tile kernels and on the (512, 2) register kernels
    pinned through fr_set_launch: equal to the FP32 bars of the oracle parity."""
    U, I, m = 3, 1000, 50
    inst = W.small_instance(U, I, m, seed=13, eps=0.01, T=80, kind="lowrank")
    prob = device_problem(fr, inst.r, inst.e, inst.eps, inst.T)
    Cd = torch.from_numpy(W.random_costs(U, I, m, 0.02, seed=14)).cuda()
    t = _ctx(fr)
    p = _ctx(fr)
    p.set_launch(I, m, 512, 2)
    ot, op = fr.step(t, prob, Cd, want_X=True), fr.step(p, prob, Cd, want_X=True)
    assert float(torch.max(torch.abs(ot["X"] - op["X"]))) <= X_ABS
    dt, _ = fr.backward(t, prob, Cd, ot["imp"], 1.0, want_dr=False, K=1)
    dp, _ = fr.backward(p, prob, Cd, op["imp"], 1.0, want_dr=False, K=1)
    assert float(torch.max(torch.abs(dt - dp))) <= GRAD_REL * float(torch.max(torch.abs(dp)))


@pytest.mark.parametrize("store", [True, False])
def test_tile_too_many_stretches_is_reported(fr, store):
    """Rebasing every iteration for T = 30 > 16 stretches (the forward's, kept
    in the row store, or the sweep's own): the solve reports
    FR_E_UNSUPPORTED (8)."""
    U, I, m = 2, 600, 40
    inst = W.small_instance(U, I, m, seed=15, eps=0.03, T=30, kind="lowrank")
    ctx = _ctx(fr, 1, store)
    prob = device_problem(fr, inst.r, inst.e, inst.eps, inst.T)
    with pytest.raises(fr.FairRankError) as ex:
        fr.solve(ctx, prob, 1, 0.003)
    assert ex.value.code == 8
    ctx = _ctx(fr, 1, store)   # a fresh workspace: device flags stay set until read
    Cd = torch.from_numpy(W.random_costs(U, I, m, 0.05, seed=16)).cuda()
    out = fr.step(ctx, prob, Cd)
    with pytest.raises(fr.FairRankError) as ex:
        fr.backward(ctx, prob, Cd, out["imp"], 1.0, want_dr=False, K=1)
    assert ex.value.code == 8


@pytest.mark.parametrize("absorb", [0, 7])
def test_tile_row_store_matches_sweep_own_rows(fr, absorb):
    """The reverse sweep with the forward's row scalings and stretches against
    the sweep that forms them (and its own stretches): the same gradient to
    the FP32 bars, on a consumer count that spans several blocks."""
    U, I, m = 9, 1000, 50
    print(f"case tile row store vs own rows absorb={absorb}", flush=True)
    inst = W.small_instance(U, I, m, seed=21, eps=0.01, T=100, kind="lowrank")
    prob = device_problem(fr, inst.r, inst.e, inst.eps, inst.T)
    Cd = torch.from_numpy(W.random_costs(U, I, m, 0.02, seed=22)).cuda()
    s, o = _ctx(fr, absorb, True), _ctx(fr, absorb, False)
    out = fr.step(s, prob, Cd)
    ds, rs = fr.backward(s, prob, Cd, out["imp"], 1.0, want_dr=True, K=1)
    do, ro = fr.backward(o, prob, Cd, out["imp"], 1.0, want_dr=True, K=1)
    cerr = float(torch.max(torch.abs(ds - do)) / torch.max(torch.abs(do)))
    rerr = float(torch.max(torch.abs(rs - ro)) / torch.max(torch.abs(ro)))
    print(f"  dC {cerr:.3e} of max, dr {rerr:.3e} of max", flush=True)
    assert cerr <= GRAD_REL and rerr <= 1e-5
