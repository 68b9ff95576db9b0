"""Parity of the fused forward (fr_step) and the impact / NSW reduction
(fr_nsw) against the FP64 oracle, element by element, on seeded inputs."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from gpu_util import assert_step_close, device_problem, oracle_step

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", params=["scaling", "log"])
def ctx(fr, request):
    """Both Sinkhorn forms compute the same iterates; every test runs on each."""
    c = fr.Context(0)
    c.set_form(request.param)
    return c


def _run(fr, ctx, r, e, eps, T, C, launch=None, want_X=True, x_dtype="f32"):
    prob = device_problem(fr, r, e, eps, T)
    U, I, m = C.shape
    if launch is not None:
        ctx.set_launch(I, m, *launch)
    out = fr.step(ctx, prob, torch.from_numpy(C).cuda(), want_X=want_X, x_dtype=x_dtype,
                  want_pot=True)
    torch.cuda.synchronize()
    return out


@pytest.mark.parametrize("which,scale", [("C1", 0.0), ("C1", 2.0), ("C2", 2.0)])
def test_step_matches_oracle_on_workloads(fr, ctx, which, scale):
    inst = W.config(which)
    C = W.random_costs(inst.U, inst.I, inst.m, scale * float(inst.eps), seed=33)
    print(f"case {which} scale {scale} U={inst.U} I={inst.I} m={inst.m}", flush=True)
    out = _run(fr, ctx, inst.r, inst.e, inst.eps, inst.T, C)
    X_ref, imp_ref, F_ref = oracle_step(inst.r, inst.e, inst.eps, inst.T, C)
    assert_step_close(out, X_ref, imp_ref, F_ref)


# (U, I, m, lanes, rows): ragged row tails, every reduction width, multi-wave
# teams, padded column classes.
SHAPES = [
    (37, 23, 5, 8, 3), (37, 23, 5, 16, 2), (5, 100, 10, 64, 2), (5, 100, 10, 32, 4),
    (6, 100, 10, 128, 1), (4, 61, 7, 16, 4), (3, 300, 20, 320, 1), (3, 300, 20, 128, 3),
    (2, 257, 13, 64, 6), (2, 500, 50, 512, 1), (3, 64, 64, 64, 1), (9, 2, 2, 2, 1),
    (4, 33, 33, 64, 1), (1, 1000, 50, 1024, 1), (3, 130, 11, 192, 1), (5, 45, 17, 8, 6),
]


@pytest.mark.parametrize("U,I,m,L,R", SHAPES)
def test_step_shapes_and_launches(fr, ctx, U, I, m, L, R):
    inst = W.small_instance(U, I, m, seed=U * 1000 + I + m, eps=0.05, T=40)
    C = W.random_costs(U, I, m, 0.1, seed=I + m)
    print(f"case U={U} I={I} m={m} L={L} R={R}", flush=True)
    try:
        ctx.set_launch(I, m, L, R)
    except fr.FairRankError as ex:
        if ex.code == 8:
            pytest.skip(f"launch ({L},{R}) not instantiated for m={m}")
        raise
    out = _run(fr, ctx, inst.r, inst.e, inst.eps, inst.T, C)
    X_ref, imp_ref, F_ref = oracle_step(inst.r, inst.e, inst.eps, inst.T, C)
    assert_step_close(out, X_ref, imp_ref, F_ref)
    # potentials reproduce the plan: x = exp((f_i + g_k - c_ik)/eps)
    pot = out["pot"].cpu().numpy().astype(np.float64)
    f, g = pot[:, :I], pot[:, I:]
    Xp = np.exp((f[:, :, None] + g[:, None, :] - C.astype(np.float64)) / float(inst.eps))
    assert np.max(np.abs(Xp - X_ref)) < 1e-4


def test_column_marginals_exact_on_gpu(fr, ctx):
    inst = W.small_instance(16, 77, 9, seed=4, eps=0.03, T=7)
    C = W.random_costs(16, 77, 9, 0.2, seed=5)
    out = _run(fr, ctx, inst.r, inst.e, inst.eps, inst.T, C)
    X = out["X"].double().cpu().numpy()
    b = np.ones(9)
    b[-1] = 77 - 9 + 1
    assert np.max(np.abs(X.sum(1) - b[None]) / b[None]) < 2e-5


def test_bf16_plan_storage(fr, ctx):
    inst = W.config("C2", U=300)
    C = W.random_costs(inst.U, inst.I, inst.m, 2 * float(inst.eps), seed=9)
    out = _run(fr, ctx, inst.r, inst.e, inst.eps, inst.T, C, x_dtype="bf16")
    X_ref, imp_ref, F_ref = oracle_step(inst.r, inst.e, inst.eps, inst.T, C)
    X = out["X"].float().cpu().numpy()
    assert np.all(np.abs(X - X_ref) <= 2.0 ** -8 * np.abs(X_ref) + 1e-5)
    # impacts come from the FP32 plan, not the BF16 copy
    assert_step_close({"imp": out["imp"], "F": out["F"]}, X_ref, imp_ref, F_ref)


def test_nsw_of_given_plan(fr, ctx):
    inst = W.small_instance(40, 30, 6, seed=12)
    rng = np.random.default_rng(3)
    X = rng.uniform(0, 1, (40, 30, 6)).astype(np.float32)
    prob = device_problem(fr, inst.r, inst.e, inst.eps, 1)
    imp, F = fr.nsw(ctx, prob, torch.from_numpy(X).cuda())
    imp_ref = oracle.impact(inst.r, inst.e, X)
    assert np.max(np.abs(imp.cpu().numpy() / imp_ref - 1)) < 1e-6
    assert abs(float(F.cpu()[0]) / oracle.nsw(imp_ref) - 1) < 1e-6
    Xb = torch.from_numpy(X).cuda().to(torch.bfloat16)
    imp_b, _ = fr.nsw(ctx, prob, Xb)
    imp_ref_b = oracle.impact(inst.r, inst.e, Xb.float().cpu().numpy())
    assert np.max(np.abs(imp_b.cpu().numpy() / imp_ref_b - 1)) < 1e-6


def test_step_is_deterministic(fr, ctx):
    inst = W.config("C2", U=500)
    C = W.random_costs(inst.U, inst.I, inst.m, 0.05, seed=1)
    a = _run(fr, ctx, inst.r, inst.e, inst.eps, 50, C)
    b = _run(fr, ctx, inst.r, inst.e, inst.eps, 50, C)
    assert torch.equal(a["X"], b["X"]) and torch.equal(a["imp"], b["imp"])
    assert torch.equal(a["F"], b["F"])


def test_device_flags(fr, ctx):
    inst = W.small_instance(8, 12, 4, seed=2)
    prob = device_problem(fr, inst.r, inst.e, inst.eps, 5)
    C = torch.zeros((8, 12, 4), device="cuda")
    C[3, 4, 1] = float("nan")
    with pytest.raises(fr.FairRankError) as ex:
        fr.step(ctx, prob, C)
    assert ex.value.code == 6
    r0 = inst.r.copy()
    r0[:, 5] = 0.0   # an item nobody finds relevant has zero impact
    prob0 = device_problem(fr, r0, inst.e, inst.eps, 5)
    with pytest.raises(fr.FairRankError) as ex:
        fr.step(ctx, prob0, torch.zeros((8, 12, 4), device="cuda"))
    assert ex.value.code == 7
    # the flags were cleared: a valid call succeeds again
    fr.step(ctx, prob, torch.zeros((8, 12, 4), device="cuda"))
