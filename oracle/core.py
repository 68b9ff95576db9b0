"""ctypes wrapper of the FP64 C oracle (``fr_oracle.c``).

TEST INFRASTRUCTURE ONLY (see the package docstring).  Every function takes
NumPy arrays, promotes them to float64, and returns float64 arrays.  The
C source follows the paper step by step:

* forward          -- log-domain Sinkhorn on problem otp (Section 3), T
                      iterations from g = 0, two LSEs per iteration.
* impact / nsw     -- Eq. Imp and Eq. objF (Section 2).
* grad             -- reverse mode ("chain rule", Section 3) through the T
                      stored iterates.
* adam / gd        -- the ascent step of Algorithm 1 (Adam as named in
                      Section 4.1).
* solve            -- Algorithm 1 with a fixed number of outer steps (long
                      Adam trajectories: parity unpinned, see ``solve``).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fr_oracle.c")
_LIB = os.path.join(_HERE, "libfr_oracle.so")
_lock = threading.Lock()
_lib = None


def library_path() -> str:
    return _LIB


def build_oracle(force: bool = True) -> str:
    """Compile fr_oracle.c with gcc -O2 -fopenmp (IEEE semantics, no fast-math)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-fvisibility=hidden",
           "-Wall", "-Wextra", "-Wno-unused-parameter", _SRC, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build_oracle(force=True)
            lib = ctypes.CDLL(_LIB)
            P = ctypes.c_void_p
            i64, i32, dbl = ctypes.c_int64, ctypes.c_int, ctypes.c_double
            lib.fro_forward.argtypes = [i64, i32, i32, P, dbl, i32, P, P, P]
            lib.fro_forward_converge.argtypes = [i64, i32, i32, P, dbl, dbl, i32, P, P, P, P]
            lib.fro_impact.argtypes = [i64, i32, i32, P, P, P, P]
            lib.fro_forward_warm.argtypes = [i64, i32, i32, P, dbl, P, dbl, i32, P, P, P]
            lib.fro_nsw.argtypes = [i32, P]
            lib.fro_nsw.restype = dbl
            lib.fro_grad.argtypes = [i64, i32, i32, P, P, dbl, i32, P, P, P, P]
            lib.fro_adam.argtypes = [i64, P, P, P, P, dbl, dbl, dbl, dbl, i64]
            lib.fro_gd.argtypes = [i64, P, P, dbl]
            lib.fro_solve.argtypes = [i64, i32, i32, P, P, dbl, i32, i32, i32, dbl, dbl, dbl,
                                      dbl, P, P, P, i64, P, P, P, dbl, P, P]
            lib.fro_num_threads.restype = i32
            lib.fro_maxrele.argtypes = [i64, i32, i32, P, P]
            lib.fro_greedy.argtypes = [i64, i32, i32, P, P, P, P]
            _lib = lib
    return _lib


def _d(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _ok(rc: int, what: str):
    if rc != 0:
        raise ValueError(f"oracle {what} failed with code {rc}")


def num_threads() -> int:
    return int(_load().fro_num_threads())


def forward(C, eps, T, want_potentials=False):
    """X = Sinkhorn_T(C) per consumer.  C [U, I, m].  Returns X (and f, g)."""
    C = _d(C)
    U, I, m = C.shape
    X = np.empty_like(C)
    f = np.empty((U, I)) if want_potentials else None
    g = np.empty((U, m)) if want_potentials else None
    _ok(_load().fro_forward(U, I, m, _p(C), float(eps), int(T), _p(X), _p(f), _p(g)), "forward")
    return (X, f, g) if want_potentials else X


def forward_converge(C, eps, tol=1e-13, cap=100000):
    """Sinkhorn run until the largest row-marginal error is < tol.
    Returns X, f, g, iterations used per consumer."""
    C = _d(C)
    U, I, m = C.shape
    X = np.empty_like(C)
    f = np.empty((U, I))
    g = np.empty((U, m))
    its = np.empty(U, dtype=np.int32)
    _ok(_load().fro_forward_converge(U, I, m, _p(C), float(eps), float(tol), int(cap), _p(X),
                                     _p(f), _p(g), _p(its)), "forward_converge")
    return X, f, g, its


def forward_warm(C, eps, g0, tol, T_max):
    """Sinkhorn from column potentials g0 [U][m] until no potential moves by
    more than tol (log2 units) in an iteration, or T_max iterations.
    Returns (X, g, iters)."""
    C = _d(C)
    U, I, m = C.shape
    g = _d(g0).copy()
    X = np.empty_like(C)
    it = np.empty(U, dtype=np.int32)
    _ok(_load().fro_forward_warm(U, I, m, _p(C), float(eps), _p(g), float(tol), int(T_max),
                                 _p(X), None, _p(it)), "forward_warm")
    return X, g, it


def impact(r, e, X):
    """Eq. Imp.  r [U, I], e [m-1], X [U, I, m] -> Imp [I]."""
    r, e, X = _d(r), _d(e), _d(X)
    U, I, m = X.shape
    assert r.shape == (U, I) and e.shape == (m - 1,)
    imp = np.empty(I)
    _ok(_load().fro_impact(U, I, m, _p(r), _p(e), _p(X), _p(imp)), "impact")
    return imp


def nsw(imp) -> float:
    """Eq. objF: F = sum_i log Imp_i."""
    imp = _d(imp)
    return float(_load().fro_nsw(imp.shape[0], _p(imp)))


def grad(r, e, eps, T, C, imp=None):
    """(dF/dC [U,I,m], dF/dr [U,I]) through the T unrolled Sinkhorn iterations.
    If imp is None it is computed from the forward at C."""
    r, e, C = _d(r), _d(e), _d(C)
    U, I, m = C.shape
    if imp is None:
        imp = impact(r, e, forward(C, eps, T))
    imp = _d(imp)
    gC = np.empty_like(C)
    gr = np.empty((U, I))
    _ok(_load().fro_grad(U, I, m, _p(r), _p(e), float(eps), int(T), _p(C), _p(imp), _p(gC),
                         _p(gr)), "grad")
    return gC, gr


def adam(C, mom, vel, g, lr, b1=0.9, b2=0.999, aeps=1e-8, step=1):
    """In-place Adam ascent step on float64 arrays C, mom, vel (maximises F)."""
    for a in (C, mom, vel):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    g = _d(g)
    _ok(_load().fro_adam(C.size, _p(C), _p(mom), _p(vel), _p(g), float(lr), float(b1), float(b2),
                         float(aeps), int(step)), "adam")


def gd(C, g, lr):
    assert C.dtype == np.float64 and C.flags.c_contiguous
    g = _d(g)
    _ok(_load().fro_gd(C.size, _p(C), _p(g), float(lr)), "gd")


def solve(r, e, eps, T, N, C0=None, rule="adam", lr=None, b1=0.9, b2=0.999, aeps=1e-8,
          mom=None, vel=None, start_step=0, m=None, grad_tol=0.0):
    """Algorithm 1 with at most N ascent steps; with grad_tol = t > 0 the loop
    ends at the first C whose gradient has ||dF/dC||_F <= t (no update there;
    the remaining F history repeats its F).  Returns dict(C, X, F_hist, imp,
    mom, vel, gnorm (norm at each step taken, NaN after a stop), updates).

    Parity unpinned for long Adam runs: each step is pinned (the forward, the
    gradient and the Adam formula separately, and the first step in closed
    form), but a many-step Adam trajectory has no closed form or independent
    reference; it is compared only with this oracle."""
    r, e = _d(r), _d(e)
    U, I = r.shape
    mm = e.shape[0] + 1 if m is None else m
    C = np.zeros((U, I, mm)) if C0 is None else _d(C0).copy()
    if lr is None:
        lr = 0.1 * float(eps)
    ri = 0 if rule == "adam" else 1
    mom = np.zeros_like(C) if mom is None else _d(mom).copy()
    vel = np.zeros_like(C) if vel is None else _d(vel).copy()
    X = np.empty_like(C)
    Fh = np.empty(N + 1)
    imp = np.empty(I)
    gn = np.full(max(N, 1), np.nan)
    upd = ctypes.c_int64()
    _ok(_load().fro_solve(U, I, mm, _p(r), _p(e), float(eps), int(T), int(N), ri, float(lr),
                          float(b1), float(b2), float(aeps), _p(C), _p(mom), _p(vel),
                          int(start_step), _p(X), _p(Fh), _p(imp), float(grad_tol), _p(gn),
                          ctypes.byref(upd)), "solve")
    return {"C": C, "X": X, "F_hist": Fh, "imp": imp, "mom": mom, "vel": vel, "gnorm": gn[:N],
            "updates": int(upd.value)}
