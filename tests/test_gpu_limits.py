"""The largest plans the fused kernels hold, in both Sinkhorn forms, against
the FP64 oracle (forward and reverse mode), and the status for plans beyond
them: I = 4096 rows with m = 32 columns, I = 2048 with m = 64, and
FR_E_UNSUPPORTED for 2049 rows with m = 40 (the plain form still runs it).
Also the 1000 x 50 plans of the 100000-consumer workload, whose reverse sweep
keeps one row of cost adjoints per lane in LDS (k_bwdl)."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import workloads as W
from gpu_util import GRAD_REL, assert_step_close, device_problem, oracle_step

pytestmark = pytest.mark.gpu
T = 20


@pytest.mark.parametrize("form", ["scaling", "log"])
@pytest.mark.parametrize("U,I,m", [(2, 4096, 32), (2, 2048, 64), (3, 4096, 5), (3, 1000, 50)])
def test_largest_plans_match_oracle(fr, U, I, m, form):
    print(f"case largest plan U={U} I={I} m={m} form={form}", flush=True)
    inst = W.small_instance(U, I, m, seed=I + m, eps=0.05, T=T, kind="lowrank")
    C = W.random_costs(U, I, m, 0.1, seed=m)
    ctx = fr.Context(0)
    ctx.set_form(form)
    if (I, m) == (1000, 50):
        ctx.set_launch(I, m, 512, 2)   # the launch of the 100000-consumer workload
    L, R = ctx.get_launch(U, I, m)
    assert L * R >= I
    prob = device_problem(fr, inst.r, inst.e, inst.eps, T)
    Cd = torch.from_numpy(C).cuda()
    out = fr.step(ctx, prob, Cd, want_X=True)
    X_ref, imp_ref, F_ref = oracle_step(inst.r, inst.e, inst.eps, T, C)
    assert_step_close(out, X_ref, imp_ref, F_ref)
    dC, _ = fr.backward(ctx, prob, Cd, out["imp"], 1.0, want_dr=False, K=1)
    gC, _ = oracle.grad(inst.r, inst.e, float(inst.eps), T, C)
    assert np.max(np.abs(dC.double().cpu().numpy() - gC)) <= GRAD_REL * np.max(np.abs(gC))


def _lds_rows(fr, ctx, U, I, m, K=0):
    lib = fr.load()
    lib.fr_ctx_bwd_lds_rows.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                                        ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p]
    rows = ctypes.c_int32(-1)
    assert lib.fr_ctx_bwd_lds_rows(ctx.handle, U, I, m, K, ctypes.byref(rows)) == 0
    return rows.value


@pytest.mark.parametrize("form", ["scaling", "log"])
def test_wide_recompute_sweeps_keep_cost_adjoints_in_lds(fr, form):
    """The parity cases above at I = 1000, m = 50 (launch 512 x 2) and at
    I = 4096, m = 32 (1024 x 4) run the LDS variant of the reverse sweep in
    both forms (the scaling form keeps the
    log-domain sweep on two-pass shapes); small plans keep everything in
    registers."""
    print(f"case lds rows form={form}", flush=True)
    ctx = fr.Context(0)
    ctx.set_form(form)
    if form == "scaling":
        # the 1000 x 50 plans run on the tile kernels in the scaling form
        assert ctx.get_launch(100000, 1000, 50) == (512, 0)
        assert _lds_rows(fr, ctx, 100000, 1000, 50) == 0
        ctx.set_launch(1000, 50, 512, 2)
    assert ctx.get_launch(100000, 1000, 50) == (512, 2)
    assert _lds_rows(fr, ctx, 100000, 1000, 50) == 1
    assert _lds_rows(fr, ctx, 2000, 100, 10) == 0
    for U, I, m in ((2, 2048, 64), (2, 4096, 32), (3, 4096, 5)):
        L, R = ctx.get_launch(U, I, m)
        # only two-pass shapes of more than 256 lanes (at least two rows per
        # lane) may keep rows in LDS, as many as fit the block's LDS, fewer than R
        lb = 512 if L <= 512 else 1024
        two_pass = L > 256 and R >= 2 and 2 * R * m + 2 * m > min(131072 // lb, 256) - 32
        rows = _lds_rows(fr, ctx, U, I, m)
        assert (0 <= rows < R) if two_pass else rows == 0, (U, I, m, L, R, rows)
    ctx.set_launch(1000, 50, 512, 2)
    assert _lds_rows(fr, ctx, 3, 1000, 50) == 1


def test_plans_beyond_the_registers_are_unsupported(fr):
    U, I, m = 2, 2049, 40
    print(f"case unsupported plan U={U} I={I} m={m}", flush=True)
    inst = W.small_instance(U, I, m, seed=1, eps=0.05, T=5)
    ctx = fr.Context(0)
    prob = device_problem(fr, inst.r, inst.e, inst.eps, 5)
    C = torch.zeros((U, I, m), device="cuda")
    with pytest.raises(fr.FairRankError) as ex:
        fr.step(ctx, prob, C)
    assert ex.value.code == 8
    with pytest.raises(fr.FairRankError) as ex:
        ctx.get_launch(U, I, m)
    assert ex.value.code == 8
    # the unfused form has no such limit
    res = fr.solve_plain(ctx, prob, 1, 0.01, rule="gd")
    ref = oracle.solve(inst.r, inst.e, float(inst.eps), 5, 1, rule="gd", lr=0.01)
    assert np.max(np.abs(res["F_hist"].cpu().numpy() / ref["F_hist"] - 1)) <= 1e-6


@pytest.mark.parametrize("form", ["scaling", "log"])
@pytest.mark.parametrize("K", [7, 50])
def test_checkpointed_sweep_with_cost_adjoints_in_lds(fr, form, K):
    """The reverse sweep that rebuilds each segment of K iterations from its
    checkpoint, on the 1000 x 50 plans at the (512, 2) launch, where it keeps
    one row of cost adjoints per lane in LDS: gradient against the FP64
    oracle; K = 50 > T is one segment of all T iterations."""
    U, I, m = 2, 1000, 50
    print(f"case checkpointed lds sweep K={K} form={form}", flush=True)
    inst = W.small_instance(U, I, m, seed=K + 3, eps=0.05, T=T, kind="lowrank")
    C = W.random_costs(U, I, m, 0.1, seed=K)
    ctx = fr.Context(0)
    ctx.set_form(form)
    ctx.set_launch(I, m, 512, 2)
    assert _lds_rows(fr, ctx, U, I, m, K) == 1
    prob = device_problem(fr, inst.r, inst.e, inst.eps, T)
    Cd = torch.from_numpy(C).cuda()
    out = fr.step(ctx, prob, Cd)
    dC, _ = fr.backward(ctx, prob, Cd, out["imp"], 1.0, want_dr=False, K=K)
    gC, _ = oracle.grad(inst.r, inst.e, float(inst.eps), T, C)
    err = float(np.max(np.abs(dC.double().cpu().numpy() - gC)) / np.max(np.abs(gC)))
    print(f"  dC {err:.3e} of max", flush=True)
    assert err <= GRAD_REL
