"""Helpers shared by the GPU parity tests: device copies of seeded workloads
and the oracle's results on the identical float32 inputs."""
import numpy as np
import torch

import oracle

# Tolerances of the FP32 GPU path against the FP64 oracle.
X_ABS = 1e-5          # plan entries, FP32 storage
F_REL = 1e-6          # objective F = sum_i log Imp_i, relative to max(|F|, I): a sum of I
                      # logarithms whose terms can cancel (|F| << I) keeps the bound per term
IMP_REL = 2e-6        # every item impact: exponents |z| ~ 16 hold half an FP32 ulp
                      # (~1e-6) of absolute error, i.e. ~7e-7 relative in x, per rounding
GRAD_REL = 1e-4       # max |dC - dC_ref| <= GRAD_REL * max |dC_ref|


def device_problem(fr, r: np.ndarray, e: np.ndarray, eps, T: int):
    return fr.Problem(torch.from_numpy(np.ascontiguousarray(r)).cuda(),
                      torch.from_numpy(np.ascontiguousarray(e)).cuda(), float(eps), int(T))


def oracle_step(r, e, eps, T, C):
    X = oracle.forward(C, float(eps), T)
    imp = oracle.impact(r, e, X)
    return X, imp, oracle.nsw(imp)


def rel(a, b):
    return abs(float(a) - float(b)) / max(abs(float(b)), 1e-300)


def f_err(F, F_ref, I):
    """Error of F = sum_i log Imp_i (Eq. objF) against the oracle's, relative to
    max(|F_ref|, I), elementwise over a history, maximum returned.  The plain
    relative error max |F / F_ref - 1| is printed beside it."""
    F = np.asarray(F, dtype=np.float64)
    F_ref = np.asarray(F_ref, dtype=np.float64)
    floored = float(np.max(np.abs(F - F_ref) / np.maximum(np.abs(F_ref), float(I))))
    plain = float(np.max(np.abs(F / F_ref - 1)))
    print(f"  F error: {floored:.3e} relative to max(|F|, I), {plain:.3e} relative to |F|",
          flush=True)
    return floored


def check_forward_at_own_C(fr, ctx, prob, r, e, eps, T, C, X=None, F=None):
    """The well-conditioned check after a trajectory: the oracle's forward at
    the GPU's own final costs C (Section 3, Eqs. Imp and objF) against the
    GPU's plan X (max-abs X_ABS), the impacts of that plan (fr_nsw, IMP_REL)
    and the GPU's F (F_REL)."""
    Cn = C.double().cpu().numpy()
    Xr = oracle.forward(Cn, float(eps), T)
    imp_r = oracle.impact(r, e, Xr)
    F_r = oracle.nsw(imp_r)
    msgs = []
    if X is not None:
        xerr = float(np.max(np.abs(X.double().cpu().numpy() - Xr)))
        imp = fr.nsw(ctx, prob, X)[0].cpu().numpy()
        ierr = float(np.max(np.abs(imp / imp_r - 1)))
        msgs.append(f"X {xerr:.3e} Imp {ierr:.3e}")
        assert xerr <= X_ABS, xerr
        assert ierr <= IMP_REL, ierr
    if F is not None:
        ferr = f_err(F, F_r, len(imp_r))
        msgs.append(f"F {ferr:.3e}")
        assert ferr <= F_REL, ferr
    print("  forward at own C:", ", ".join(msgs), flush=True)


def assert_step_close(out, X_ref, imp_ref, F_ref, x_abs=X_ABS):
    imp = out["imp"].cpu().numpy()
    F = float(out["F"].cpu()[0])
    assert np.max(np.abs(imp / imp_ref - 1)) <= IMP_REL, np.max(np.abs(imp / imp_ref - 1))
    assert f_err(F, F_ref, len(imp_ref)) <= F_REL, (F, F_ref)
    if out.get("X") is not None:
        X = out["X"].float().cpu().numpy()
        err = np.max(np.abs(X - X_ref))
        assert err <= x_abs, err
