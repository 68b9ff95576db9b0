"""Precision at scale: 1000 consumers sampled from the 100000 x 1000 x 50
workload (eps 0.01, T 300), plans stored in BF16, FP64 impacts and log-NSW,
against the FP64 oracle's stored values (tests/golden/c5_sub.npz)."""
import os

import numpy as np
import pytest
import torch

import workloads as W
from gpu_util import F_REL, IMP_REL, X_ABS, device_problem

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "c5_sub.npz")


@pytest.fixture(scope="module")
def sub(fr):
    g = np.load(GOLDEN)
    inst = W.config("C5")
    users = g["users"]
    ctx = fr.Context(0)
    prob = device_problem(fr, inst.r[users], inst.e, inst.eps, inst.T)
    return g, inst, ctx, prob


@pytest.mark.parametrize("x_dtype", ["f32", "bf16"])
def test_subsample_forward(fr, sub, x_dtype):
    g, inst, ctx, prob = sub
    print(f"case C5 subsample forward {x_dtype}", flush=True)
    C = torch.from_numpy(W.random_costs(1000, inst.I, inst.m, 2 * float(inst.eps), seed=56)).cuda()
    out = fr.step(ctx, prob, C, want_X=True, x_dtype=x_dtype)
    assert np.max(np.abs(out["imp"].cpu().numpy() / g["rand_imp"] - 1)) <= IMP_REL
    assert abs(float(out["F"].cpu()[0]) / float(g["rand_F"][0]) - 1) <= F_REL
    X = out["X"][torch.from_numpy(g["sel"]).long()].float().cpu().numpy()
    Xr = g["rand_X_sel"].astype(np.float64)
    if x_dtype == "f32":
        assert np.max(np.abs(X - Xr)) <= X_ABS
    else:
        assert np.all(np.abs(X - Xr) <= 2.0 ** -8 * np.abs(Xr) + X_ABS)


def test_subsample_solve_bf16(fr, sub):
    g, inst, ctx, prob = sub
    print("case C5 subsample 3-step solve", flush=True)
    res = fr.solve(ctx, prob, 3, float(inst.lr), x_dtype="bf16")
    Fh = res["F_hist"].cpu().numpy()
    assert np.max(np.abs(Fh / g["adam_F_hist"] - 1)) <= F_REL
