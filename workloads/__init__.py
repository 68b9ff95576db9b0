"""Seeded synthetic inputs for the impact-based fair ranking solver.

This module is shared by the FP64 oracle's tests, the GPU parity tests and the
benchmark.  It draws only the problem data -- relevance r(u,i), exposure e(k),
sizes, entropic weight and iteration counts, and starting cost tensors -- and
performs no step of the method itself (no Sinkhorn, no impact, no gradient).

Problem data follow the paper's problem statement (Section 2): consumers U,
items I, m columns per plan of which the last is the dummy position, relevance
r(u,i) > 0 and exposure e(k) for the m-1 real positions.  The paper's own
datasets are not available, so the generators below stand in for them:

* ``uniform``: r ~ Uniform(0, 1).
* ``lowrank``: r = sigmoid(p_u . q_i + b_i) with p, q ~ N(0, var) of a given
  rank and item bias b_i ~ N(-1, 1), which gives a popularity skew.

All values are drawn in float64 with ``numpy.random.default_rng(seed)`` and then
rounded to float32; both the oracle and the GPU path consume the identical
float32 numbers (the oracle promotes them to float64).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

__all__ = [
    "Instance", "exposure", "relevance_uniform", "relevance_lowrank",
    "config", "CONFIG_NAMES", "batched_shapes", "batched_instance",
    "random_costs", "subsample_users", "small_instance", "PAPER_SHAPES", "paper_shape",
    "user_sweep",
]


@dataclasses.dataclass
class Instance:
    """One fair-ranking problem (Section 2 notation)."""
    name: str
    U: int            # |U| consumers
    I: int            # |I| items
    m: int            # columns of X_u including the dummy (m-1 real positions)
    r: np.ndarray     # float32 [U, I] relevance r(u,i)
    e: np.ndarray     # float32 [m-1] exposure e(k) of the real positions
    eps: np.float32   # entropic weight (Section 3, problem otp)
    T: int            # Sinkhorn iterations per outer step
    N: int            # outer ascent steps (Algorithm 1)
    seed: int

    @property
    def cells(self) -> int:
        return self.U * self.I * self.m

    @property
    def lr(self) -> np.float32:
        """Adam learning rate used by the frozen configurations: 0.1 * eps."""
        return np.float32(0.1) * self.eps


def exposure(m: int) -> np.ndarray:
    """e(k) = 1 / log2(k + 1) for the m-1 real positions k = 1..m-1 (float32)."""
    k = np.arange(1, m, dtype=np.float64)
    return (1.0 / np.log2(k + 1.0)).astype(np.float32)


def relevance_uniform(U: int, I: int, rng: np.random.Generator) -> np.ndarray:
    r = rng.uniform(0.0, 1.0, size=(U, I)).astype(np.float32)
    # exact zeros have probability ~2^-53 but would violate r > 0
    r[r <= 0] = np.float32(np.finfo(np.float32).tiny)
    return r


def relevance_lowrank(U: int, I: int, rank: int, var: float,
                      rng: np.random.Generator) -> np.ndarray:
    sd = math.sqrt(var)
    p = rng.normal(0.0, sd, size=(U, rank))
    q = rng.normal(0.0, sd, size=(I, rank))
    b = rng.normal(-1.0, 1.0, size=I)
    out = np.empty((U, I), dtype=np.float32)
    step = max(1, (1 << 24) // max(I, 1))
    for s in range(0, U, step):
        z = p[s:s + step] @ q.T + b[None, :]
        out[s:s + step] = (1.0 / (1.0 + np.exp(-z))).astype(np.float32)
    return out


CONFIG_NAMES = ("C1", "C2", "C3", "C4", "C5")


def config(name: str, U: Optional[int] = None) -> Instance:
    """Frozen workloads.

    C1  U=50,     I=20,   m=5,  r uniform,        eps=0.05, T=100, N=50
    C2  U=2000,   I=100,  m=10, low-rank 16,      eps=0.02, T=200, N=100
    C3  U=10000,  I=300,  m=20, low-rank 16,      eps=0.02, T=300 (gradient only)
    C5  U=100000, I=1000, m=50, low-rank 32 (var 1/32), eps=0.01, T=300, N=50
    (C4 is the batch of 128 instances, see ``batched_shapes``.)

    ``U`` overrides the number of consumers (the first U rows of the full draw
    are NOT used; the draw itself is made at the requested size).
    """
    if name == "C1":
        U_ = 50 if U is None else U
        rng = np.random.default_rng(1)
        r = relevance_uniform(U_, 20, rng)
        return Instance("C1", U_, 20, 5, r, exposure(5), np.float32(0.05), 100, 50, 1)
    if name == "C2":
        U_ = 2000 if U is None else U
        rng = np.random.default_rng(2)
        r = relevance_lowrank(U_, 100, 16, 1.0 / 16, rng)
        return Instance("C2", U_, 100, 10, r, exposure(10), np.float32(0.02), 200, 100, 2)
    if name == "C3":
        U_ = 10000 if U is None else U
        rng = np.random.default_rng(3)
        r = relevance_lowrank(U_, 300, 16, 1.0 / 16, rng)
        return Instance("C3", U_, 300, 20, r, exposure(20), np.float32(0.02), 300, 1, 3)
    if name == "C5":
        U_ = 100000 if U is None else U
        rng = np.random.default_rng(5)
        r = relevance_lowrank(U_, 1000, 32, 1.0 / 32, rng)
        return Instance("C5", U_, 1000, 50, r, exposure(50), np.float32(0.01), 300, 50, 5)
    raise KeyError(name)


# The shapes of the paper's experiments (Section 4: Figs. 1-3), m counting the
# dummy column (top-10 rankings plus the dummy), with seeds 6-8; the sweep over
# consumers of Section 4.2 at 250 items (seed 9).  Entropic weight, iteration
# counts and relevance model as the 2000 x 100 x 10 workload, N = 10 outer steps.
PAPER_SHAPES = {"fig1": (1000, 500, 11, 6), "fig2": (1014, 100, 11, 7), "fig3": (250, 250, 11, 8)}


def paper_shape(name: str, U: Optional[int] = None, N: int = 10) -> Instance:
    """One of the paper's shapes (PAPER_SHAPES), low-rank-16 sigmoid relevance,
    eps 0.02, T 200."""
    U0, I, m, seed = PAPER_SHAPES[name]
    U_ = U0 if U is None else U
    rng = np.random.default_rng(seed)
    r = relevance_lowrank(U_, I, 16, 1.0 / 16, rng)
    return Instance(name, U_, I, m, r, exposure(m), np.float32(0.02), 200, N, seed)


def user_sweep(U: int, N: int = 10) -> Instance:
    """The consumer sweep: U consumers x 250 items x 11 columns (seed 9)."""
    rng = np.random.default_rng(9)
    r = relevance_lowrank(U, 250, 16, 1.0 / 16, rng)
    return Instance(f"sweep{U}", U, 250, 11, r, exposure(11), np.float32(0.02), 200, N, 9)


def batched_shapes(n_inst: int = 128, seed: int = 4):
    """(U, I, m) per instance of the batched workload: U~U[100,5000],
    I~U[20,500], m~U[5,50], with m clamped to at most I (dummy mass >= 1)."""
    rng = np.random.default_rng(seed)
    U = rng.integers(100, 5001, size=n_inst)
    I = rng.integers(20, 501, size=n_inst)
    m = rng.integers(5, 51, size=n_inst)
    m = np.minimum(m, I)
    return [(int(a), int(b), int(c)) for a, b, c in zip(U, I, m)]


def batched_instance(j: int, shape, eps: float = 0.03, T: int = 200, N: int = 50) -> Instance:
    U, I, m = shape
    rng = np.random.default_rng(4000 + j)
    r = relevance_lowrank(U, I, 16, 1.0 / 16, rng)
    return Instance(f"C4[{j}]", U, I, m, r, exposure(m), np.float32(eps), T, N, 4000 + j)


def small_instance(U: int, I: int, m: int, seed: int, eps: float = 0.05, T: int = 50,
                   N: int = 10, kind: str = "uniform") -> Instance:
    """Small seeded instance for unit tests."""
    rng = np.random.default_rng(seed)
    if kind == "uniform":
        r = relevance_uniform(U, I, rng)
    else:
        r = relevance_lowrank(U, I, 4, 0.25, rng)
    return Instance(f"small{U}x{I}x{m}", U, I, m, r, exposure(m), np.float32(eps), T, N, seed)


def random_costs(U: int, I: int, m: int, scale: float, seed: int) -> np.ndarray:
    """C ~ N(0, scale^2) i.i.d., float32 [U, I, m] (evaluation points for gradients)."""
    rng = np.random.default_rng(seed)
    return rng.normal(0.0, scale, size=(U, I, m)).astype(np.float32)


def subsample_users(U: int, n: int, seed: int) -> np.ndarray:
    """Sorted seeded sample of n distinct consumer indices out of U."""
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(U, size=n, replace=False))


def instance_list_sizes(insts: List[Instance]) -> int:
    return sum(x.cells for x in insts)
