"""The seeded input generators shared by the oracle tests, the GPU parity tests
and the benchmark: the documented shapes, types and ranges, determinism, and
that the module holds none of the method's arithmetic (it imports neither the
oracle nor the GPU package)."""
import os
import re

import numpy as np
import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SHAPES = {"C1": (50, 20, 5, 0.05, 100, 50), "C2": (2000, 100, 10, 0.02, 200, 100),
          "C3": (10000, 300, 20, 0.02, 300, 1)}


@pytest.mark.parametrize("name", sorted(SHAPES))
def test_configs_have_the_documented_shapes(name):
    U, I, m, eps, T, N = SHAPES[name]
    x = W.config(name)
    assert (x.U, x.I, x.m, x.T, x.N) == (U, I, m, T, N)
    assert x.eps == np.float32(eps)
    assert x.r.shape == (U, I) and x.r.dtype == np.float32 and x.r.flags.c_contiguous
    assert np.all(x.r > 0) and np.all(x.r < 1)
    assert x.e.shape == (m - 1,) and x.e.dtype == np.float32
    assert x.lr == np.float32(0.1) * x.eps


def test_large_config_at_a_smaller_consumer_count():
    x = W.config("C5", U=300)
    assert (x.U, x.I, x.m, x.T) == (300, 1000, 50, 300) and x.eps == np.float32(0.01)


def test_exposure_is_one_over_log2_of_the_rank_plus_one():
    e = W.exposure(11)
    k = np.arange(1, 11)
    assert np.allclose(e, 1.0 / np.log2(k + 1), rtol=1e-7, atol=0)
    assert e[0] == 1.0 and np.all(np.diff(e) < 0)


def test_draws_are_deterministic():
    a, b = W.config("C2", U=50), W.config("C2", U=50)
    assert np.array_equal(a.r, b.r)
    assert np.array_equal(W.random_costs(3, 4, 5, 0.1, seed=7), W.random_costs(3, 4, 5, 0.1, seed=7))
    assert not np.array_equal(W.random_costs(3, 4, 5, 0.1, seed=7),
                              W.random_costs(3, 4, 5, 0.1, seed=8))


def test_batched_shapes_respect_the_ranges_and_the_dummy_mass():
    shapes = W.batched_shapes(128, seed=4)
    assert len(shapes) == 128
    for U, I, m in shapes:
        assert 100 <= U <= 5000 and 20 <= I <= 500 and 5 <= m <= 50
        assert 2 <= m <= I   # dummy mass I - m + 1 >= 1
    x = W.batched_instance(0, shapes[0])
    assert (x.U, x.I, x.m) == shapes[0] and x.r.dtype == np.float32


def test_subsample_is_sorted_and_distinct():
    s = W.subsample_users(1000, 100, seed=55)
    assert len(s) == 100 and np.all(np.diff(s) > 0) and s[0] >= 0 and s[-1] < 1000


def test_generators_hold_no_step_of_the_method():
    src = open(os.path.join(ROOT, "workloads", "__init__.py")).read()
    assert not re.search(r"^\s*(import|from)\s+(oracle|paper_2406_10262_amd)\b", src, flags=re.M)
    for word in ("sinkhorn(", "logsumexp", "impact("):
        assert word not in src.lower()
