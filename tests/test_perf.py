"""Timing comparisons on the GPU.  Not parity tests: marked perf only (not
gpu), so the parity run (-m gpu) does not include them; run with -m perf."""
import numpy as np
import pytest
import torch

import workloads as W
from gpu_util import device_problem


@pytest.mark.perf
def test_autotune_times_the_whole_reverse_sweep(fr):
    """The autotuner once timed a backward that ran no reverse iterations (its
    checkpoint interval was left at 0) and so ranked shapes by their forward
    alone.  On the 1000 x 50 plans its pick must be as fast, measured
    directly over forward and backward, as the (512, 2) shape.  A timing
    check: marked perf, outside the gpu parity tests (run with -m perf)."""
    import time
    inst = W.config("C5", U=2000)
    prob = device_problem(fr, inst.r, inst.e, inst.eps, 20)
    C = torch.from_numpy(W.random_costs(inst.U, inst.I, inst.m, 2 * float(inst.eps), seed=3)).cuda()
    ctx = fr.Context(0)
    pick = ctx.autotune(prob, C=C, iters=20)
    print("case autotune pick for 2000 x 1000 x 50:", pick, flush=True)

    def timed(L, R):
        ctx.set_launch(inst.I, inst.m, L, R)
        best = 1e9
        for _ in range(3):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            out = fr.step(ctx, prob, C, sync=False)
            fr.backward(ctx, prob, C, out["imp"], 1.0, want_dr=False, K=1)
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t0)
        return best

    t_pick, t_ref = timed(*pick), timed(512, 2)
    print(f"  pick {t_pick * 1e3:.2f} ms, (512, 2) {t_ref * 1e3:.2f} ms", flush=True)
    assert t_pick <= 1.3 * t_ref
