"""FP64 CPU oracle of the impact-based fair ranking solver.

TEST INFRASTRUCTURE ONLY: this package is the slow, plain reference against
which the GPU library is checked.  Only the test suite, the package's smoke
check and the benchmark's CPU-baseline leg may import it.  It shares no code
with the GPU path (``paper_2406_10262_amd``) and never imports it.

* ``oracle.core``  -- ctypes wrapper of ``fr_oracle.c`` (Sinkhorn forward,
  impacts, NSW, reverse-mode gradient, Adam / gradient ascent, Algorithm 1).
* ``oracle.brute`` -- NumPy brute-force optima and closed forms for tiny
  instances, used to pin the oracle itself.
* ``oracle.metrics`` -- the evaluation metrics of a plan.
* ``oracle.warm`` -- Algorithm 1 on the converged map: warm-started Sinkhorn
  and the implicit-function gradient.
* ``oracle.baselines`` -- the MaxRele and NSW(Greedy) rankings of the
  comparison in Section 4.1.
"""
from .core import (  # noqa: F401
    build_oracle, forward, forward_converge, forward_warm, impact, nsw, grad, adam, gd, solve,
    num_threads, library_path,
)
