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
    max(|F_ref|, I), elementwise over a history, maximum returned."""
    F = np.asarray(F, dtype=np.float64)
    F_ref = np.asarray(F_ref, dtype=np.float64)
    return float(np.max(np.abs(F - F_ref) / np.maximum(np.abs(F_ref), float(I))))


def assert_step_close(out, X_ref, imp_ref, F_ref, x_abs=X_ABS):
    imp = out["imp"].cpu().numpy()
    F = float(out["F"].cpu()[0])
    assert np.max(np.abs(imp / imp_ref - 1)) <= IMP_REL, np.max(np.abs(imp / imp_ref - 1))
    assert f_err(F, F_ref, len(imp_ref)) <= F_REL, (F, F_ref)
    if out.get("X") is not None:
        X = out["X"].float().cpu().numpy()
        err = np.max(np.abs(X - X_ref))
        assert err <= x_abs, err
