"""fr_step_noalloc (the allocation-free fr_step, for callers that cannot
allocate): through the C ABI its outputs equal fr_step's on the same inputs,
over two calls in a row on one context (the second smaller, so it runs on
the device array the first call left behind); problems beyond its array are
rejected on the host."""
import ctypes

import numpy as np
import pytest
import torch

import workloads as W
from gpu_util import device_problem

pytestmark = pytest.mark.gpu


def _noalloc(fr, lib, ctx, prob, C, X, x_dtype, pot, imp, F):
    lib.fr_step_noalloc.argtypes = [ctypes.c_void_p, ctypes.c_void_p] + [ctypes.c_void_p] * 2 + [
        ctypes.c_int] + [ctypes.c_void_p] * 4
    p = prob.c()
    return lib.fr_step_noalloc(ctx.handle, ctypes.byref(p), fr._ptr(C), fr._ptr(X),
                               fr.FR_BF16 if x_dtype == "bf16" else fr.FR_F32, fr._ptr(pot),
                               fr._ptr(imp), fr._ptr(F),
                               ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))


@pytest.mark.parametrize("x_dtype", ["f32", "bf16"])
def test_noalloc_step_equals_step_twice(fr, x_dtype):
    lib = fr.load()
    ctx = fr.Context(0)
    for U, I, m, seed in ((700, 300, 20, 1), (37, 45, 7, 2)):
        print(f"case fr_step_noalloc {x_dtype} U={U} I={I} m={m}", flush=True)
        inst = W.small_instance(U, I, m, seed=seed, eps=0.05, T=40, kind="lowrank")
        prob = device_problem(fr, inst.r, inst.e, inst.eps, inst.T)
        C = torch.from_numpy(W.random_costs(U, I, m, 0.1, seed=seed + 10)).cuda()
        ref = fr.step(ctx, prob, C, want_X=True, x_dtype=x_dtype, want_pot=True)
        xd = torch.bfloat16 if x_dtype == "bf16" else torch.float32
        X = torch.full((U, I, m), float("nan"), dtype=xd, device="cuda")
        pot = torch.full((U, I + m), float("nan"), dtype=torch.float32, device="cuda")
        imp = torch.full((I,), float("nan"), dtype=torch.float64, device="cuda")
        F = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
        assert _noalloc(fr, lib, ctx, prob, C, X, x_dtype, pot, imp, F) == 0
        torch.cuda.synchronize()
        assert torch.equal(X, ref["X"])
        assert torch.equal(pot, ref["pot"])
        assert torch.equal(imp, ref["imp"])
        assert torch.equal(F, ref["F"])
    ctx.close()


def test_noalloc_rejects_problems_beyond_its_array(fr):
    lib = fr.load()
    ctx = fr.Context(0)
    U, I, m = 40000, 400, 5   # 4 U I = 64 MB of impact contributions alone
    r = torch.ones((U, I), dtype=torch.float32, device="cuda")
    e = torch.from_numpy(W.exposure(m)).cuda()
    prob = fr.Problem(r, e, 0.05, 10)
    C = torch.zeros((U, I, m), dtype=torch.float32, device="cuda")
    imp = torch.empty(I, dtype=torch.float64, device="cuda")
    F = torch.empty(1, dtype=torch.float64, device="cuda")
    assert _noalloc(fr, lib, ctx, prob, C, None, "f32", None, imp, F) == 4   # FR_E_WORKSPACE
    assert _noalloc(fr, lib, ctx, prob, C, None, "f32", None, None, F) == 1  # FR_E_NULL
    ctx.close()
