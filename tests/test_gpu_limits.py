"""The largest plans the fused kernels hold, in both Sinkhorn forms, against
the FP64 oracle (forward and reverse mode), and the status for plans beyond
them: I = 4096 rows with m = 32 columns, I = 2048 with m = 64, and
FR_E_UNSUPPORTED for 2049 rows with m = 40 (the plain form still runs it)."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from gpu_util import GRAD_REL, assert_step_close, device_problem, oracle_step

pytestmark = pytest.mark.gpu
T = 20


@pytest.mark.parametrize("form", ["scaling", "log"])
@pytest.mark.parametrize("U,I,m", [(2, 4096, 32), (2, 2048, 64), (3, 4096, 5)])
def test_largest_plans_match_oracle(fr, U, I, m, form):
    print(f"case largest plan U={U} I={I} m={m} form={form}", flush=True)
    inst = W.small_instance(U, I, m, seed=I + m, eps=0.05, T=T, kind="lowrank")
    C = W.random_costs(U, I, m, 0.1, seed=m)
    ctx = fr.Context(0)
    ctx.set_form(form)
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
