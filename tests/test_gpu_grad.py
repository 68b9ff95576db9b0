"""Gradient workload (10000 consumers x 300 items x 20 positions, eps 0.02,
T = 300, potentials checkpointed every 50 iterations): the HIP forward and
adjoint against the FP64 oracle's values and central differences stored in
tests/golden/c3_grad.npz."""
import os

import numpy as np
import pytest
import torch

import workloads as W
from gpu_util import F_REL, GRAD_REL, IMP_REL, device_problem

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "c3_grad.npz")


@pytest.fixture(scope="module")
def setup(fr):
    d = np.load(GOLDEN)
    inst = W.config("C3")
    ctx = fr.Context(0)
    prob = device_problem(fr, inst.r, inst.e, inst.eps, inst.T)
    points = {"zero": torch.zeros((inst.U, inst.I, inst.m), device="cuda"),
              "rand": torch.from_numpy(W.random_costs(inst.U, inst.I, inst.m,
                                                      2 * float(inst.eps), seed=33)).cuda()}
    return d, inst, ctx, prob, points


@pytest.mark.parametrize("tag", ["zero", "rand"])
def test_forward_impacts_and_F(fr, setup, tag):
    d, inst, ctx, prob, points = setup
    print(f"case C3 forward {tag}", flush=True)
    out = fr.step(ctx, prob, points[tag])
    imp = out["imp"].cpu().numpy()
    assert np.max(np.abs(imp / d[tag + "_imp"] - 1)) <= IMP_REL
    assert abs(float(out["F"].cpu()[0]) / float(d[tag + "_F"][0]) - 1) <= F_REL


@pytest.mark.parametrize("tag", ["zero", "rand"])
def test_backward_checkpointed_against_oracle_and_fd(fr, setup, tag):
    d, inst, ctx, prob, points = setup
    print(f"case C3 backward {tag} K=50", flush=True)
    C = points[tag]
    out = fr.step(ctx, prob, C)
    dC, dr = fr.backward(ctx, prob, C, out["imp"], 1.0, want_dr=True, K=50)
    users = torch.from_numpy(d["users"].astype(np.int64)).cuda()
    dCu = dC[users].double().cpu().numpy()
    dru = dr[users].double().cpu().numpy()
    ref = d[tag + "_dC"].astype(np.float64)
    scale = np.max(np.abs(ref))
    err = np.max(np.abs(dCu - ref)) / scale
    print(f"  dC rel-to-max err {err:.2e}", flush=True)
    assert err <= GRAD_REL
    rref = d[tag + "_dr"].astype(np.float64)
    assert np.max(np.abs(dru - rref)) <= 1e-5 * np.max(np.abs(rref))
    # central differences of F at 64 cost and 64 relevance coordinates
    g = dC[torch.from_numpy(d["c_u"]).long(), torch.from_numpy(d["c_i"]).long(),
           torch.from_numpy(d["c_k"]).long()].double().cpu().numpy()
    fd = d[tag + "_fdC"]
    assert np.all(np.abs(g - fd) <= 1e-5 * scale + 1e-3 * np.abs(fd))
    gr = dr[torch.from_numpy(d["r_u"]).long(), torch.from_numpy(d["r_i"]).long()]
    fdr = d[tag + "_fdr"]
    assert np.all(np.abs(gr.double().cpu().numpy() - fdr) <= 1e-5 * np.max(np.abs(rref)) +
                  1e-4 * np.abs(fdr))


@pytest.mark.parametrize("form,bar", [("log", 1e-5), ("scaling", GRAD_REL)])
def test_checkpoint_interval_does_not_change_the_gradient(fr, setup, form, bar):
    """K = 1 reads the forward's stored potentials, K > 1 rebuilds each
    segment in the log domain from a checkpoint.  With the log-domain forward
    both run the same arithmetic (bar: rounding of the reduction order); the
    scaling forward's potentials carry their own FP32 rounding, so the bar is
    the gradient tolerance."""
    d, inst, ctx, prob, points = setup
    ctx.set_form(form)
    C = points["rand"]
    out = fr.step(ctx, prob, C)
    a, _ = fr.backward(ctx, prob, C, out["imp"], 1.0, want_dr=False, K=1)
    b, _ = fr.backward(ctx, prob, C, out["imp"], 1.0, want_dr=False, K=50)
    c, _ = fr.backward(ctx, prob, C, out["imp"], 1.0, want_dr=False, K=7)
    ctx.set_form("scaling")
    scale = float(a.abs().max())
    assert float((a - b).abs().max()) <= bar * scale
    assert float((a - c).abs().max()) <= bar * scale


def test_autograd_function(fr, setup):
    """F = SinkhornNSW(C, r); F.backward() gives the same dF/dC and dF/dr as
    fr_backward, scaled by the upstream gradient."""
    d, inst, ctx, prob, points = setup
    C = points["rand"].clone().requires_grad_(True)
    r = prob.r.clone().requires_grad_(True)
    F = fr.sinkhorn_nsw(C, r, prob.e, prob.eps, prob.T, K=50, ctx=ctx)
    (2.5 * F).backward()
    out = fr.step(ctx, prob, points["rand"])
    dC, dr = fr.backward(ctx, prob, points["rand"], out["imp"], 2.5, want_dr=True, K=50)
    assert abs(float(F.detach()) / float(d["rand_F"][0]) - 1) <= F_REL
    assert torch.allclose(C.grad, dC, rtol=0, atol=1e-6 * float(dC.abs().max()))
    assert torch.allclose(r.grad, dr, rtol=0, atol=1e-6 * float(dr.abs().max()))
