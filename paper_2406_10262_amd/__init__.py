"""MI355X-native impact-based fair ranking solver.

Python binding of ``libfairrank.so`` (C ABI in ``include/fairrank.h``).  This
module only marshals arguments: every step of the method -- Sinkhorn on each
consumer's plan (Section 3, problem otp), the impact and log-NSW sums
(Eqs. Imp and objF), the reverse sweep through the Sinkhorn iterations and
the ascent step of Algorithm 1 -- runs in the HIP library.  PyTorch supplies
device memory and streams.

The library must have been built (``python -m paper_2406_10262_amd.build``);
every entry point raises if it cannot be loaded.  There is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional

import torch

__all__ = [
    "load", "library_path", "FairRankError", "Context", "Problem", "step", "nsw",
    "backward", "solve", "solve_plain", "solve_batched", "SinkhornNSW", "sinkhorn_nsw", "metrics",
    "grad_converged", "rank_maxrele", "rank_greedy",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libfairrank.so")
_lib = None

FR_OK = 0
FR_F32, FR_BF16 = 0, 1
FR_ADAM, FR_GD = 0, 1
FR_FORM_LOG, FR_FORM_SCALING = 0, 1
STATUS = {
    0: "FR_OK", 1: "FR_E_NULL", 2: "FR_E_SHAPE", 3: "FR_E_PARAM", 4: "FR_E_WORKSPACE",
    5: "FR_E_DEVICE", 6: "FR_E_NONFINITE", 7: "FR_E_ZERO_IMPACT", 8: "FR_E_UNSUPPORTED",
}


class FairRankError(RuntimeError):
    def __init__(self, code: int, what: str):
        self.code = code
        msg = _lib.fr_status_string(code).decode() if _lib is not None else ""
        super().__init__(f"{what}: {STATUS.get(code, code)} ({msg})")


class _Problem(ctypes.Structure):
    _fields_ = [("n_users", ctypes.c_int64), ("n_items", ctypes.c_int32), ("m", ctypes.c_int32),
                ("r", ctypes.c_void_p), ("e", ctypes.c_void_p), ("eps", ctypes.c_float),
                ("sinkhorn_iters", ctypes.c_int32)]


class _Optim(ctypes.Structure):
    _fields_ = [("rule", ctypes.c_int32), ("lr", ctypes.c_float), ("beta1", ctypes.c_float),
                ("beta2", ctypes.c_float), ("adam_eps", ctypes.c_float),
                ("outer_steps", ctypes.c_int32), ("checkpoint_every", ctypes.c_int32),
                ("grad_tol", ctypes.c_double), ("sinkhorn_tol", ctypes.c_float),
                ("cg_iters", ctypes.c_int32)]


def library_path() -> str:
    return _LIB_PATH


def load():
    """Loads libfairrank.so; raises FileNotFoundError if it was not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise FileNotFoundError(
            f"{_LIB_PATH} is missing: build it with `python -m paper_2406_10262_amd.build`")
    lib = ctypes.CDLL(_LIB_PATH)
    P, I32, I64, SZ = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    PP = ctypes.POINTER(_Problem)
    PO = ctypes.POINTER(_Optim)
    lib.fr_status_string.restype = ctypes.c_char_p
    lib.fr_status_string.argtypes = [ctypes.c_int]
    lib.fr_ctx_create.argtypes = [ctypes.c_int, ctypes.POINTER(P)]
    lib.fr_ctx_destroy.argtypes = [P]
    lib.fr_ctx_destroy.restype = None
    lib.fr_workspace_bytes.argtypes = [PP, PO, ctypes.POINTER(SZ)]
    lib.fr_workspace_bytes_plain.argtypes = [PP, ctypes.POINTER(SZ)]
    lib.fr_step.argtypes = [P, PP, P, P, ctypes.c_int, P, P, P, P, SZ, P]
    lib.fr_nsw.argtypes = [P, PP, P, ctypes.c_int, P, P, P, SZ, P]
    lib.fr_backward.argtypes = [P, PP, P, P, ctypes.c_double, P, P, I32, P, SZ, P]
    lib.fr_solve.argtypes = [P, PP, PO, P, P, P, I64, P, ctypes.c_int, P, P, SZ, P]
    lib.fr_solve_plain.argtypes = [P, PP, PO, P, P, P, I64, P, ctypes.c_int, P, P, SZ, P]
    lib.fr_sync_status.argtypes = [P, P, P]
    lib.fr_workspace_bytes_batched.argtypes = [I32, PP, PO, ctypes.POINTER(SZ)]
    lib.fr_autotune.argtypes = [P, PP, P, I32, I32, P, SZ, P, ctypes.POINTER(I32),
                                ctypes.POINTER(I32)]
    lib.fr_solve_batched.argtypes = [P, I32, PP, PO, P, P, P, I64, P, ctypes.c_int, P, P, SZ, P]
    lib.fr_workspace_init.argtypes = [P, P, SZ, P]
    lib.fr_set_launch.argtypes = [P, I32, I32, I32, I32]
    lib.fr_ctx_set_form.argtypes = [P, I32, I32]
    lib.fr_ctx_set_row_store.argtypes = [P, ctypes.c_int]
    lib.fr_rank_maxrele.argtypes = [P, PP, P, P, I32, P]
    lib.fr_rank_greedy.argtypes = [P, PP, P, P, I32, P, P]
    lib.fr_get_launch.argtypes = [P, I64, I32, I32, ctypes.POINTER(I32), ctypes.POINTER(I32)]
    lib.fr_workspace_bytes_metrics.argtypes = [PP, ctypes.POINTER(SZ)]
    lib.fr_solve_progress.argtypes = [P, P, P, ctypes.POINTER(I64), ctypes.POINTER(ctypes.c_double),
                                      ctypes.POINTER(I64)]
    lib.fr_grad_converged.argtypes = [P, PP, P, ctypes.c_float, I32, ctypes.c_double, P, P, P, P,
                                      P, SZ, P]
    lib.fr_metrics.argtypes = [P, PP, P, ctypes.c_int, P, P, P, P, SZ, P]
    for name in ("fr_ctx_create", "fr_workspace_bytes", "fr_workspace_init", "fr_workspace_bytes_plain", "fr_step",
                 "fr_nsw", "fr_backward", "fr_solve", "fr_solve_plain", "fr_sync_status",
                 "fr_workspace_bytes_batched", "fr_solve_batched", "fr_autotune",
                 "fr_set_launch", "fr_get_launch", "fr_workspace_bytes_metrics", "fr_metrics",
                 "fr_solve_progress", "fr_grad_converged", "fr_ctx_set_form",
                 "fr_ctx_set_row_store", "fr_rank_maxrele", "fr_rank_greedy"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(code: int, what: str):
    if code != FR_OK:
        raise FairRankError(code, what)


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


# --------------------------------------------------------------------------
class Context:
    """Owns an fr_ctx (launch-configuration cache) and a reusable workspace."""

    def __init__(self, device: int = 0):
        lib = load()
        self.device = torch.device("cuda", device)
        h = ctypes.c_void_p()
        _check(lib.fr_ctx_create(device, ctypes.byref(h)), "fr_ctx_create")
        self.handle = h
        self._ws = None

    def close(self):
        if self.handle is not None and _lib is not None:
            _lib.fr_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):  # pragma: no cover
        try:
            self.close()
        except Exception:
            pass

    def workspace(self, nbytes: int) -> torch.Tensor:
        if self._ws is None or self._ws.numel() < nbytes:
            self._ws = None
            ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=self.device)
            _check(load().fr_workspace_init(self.handle, _ptr(ws), ws.numel(),
                                            _stream(self.device)), "fr_workspace_init")
            self._ws = ws
        return self._ws

    def set_form(self, form: str = "scaling", absorb_every: int = 0):
        """fr_ctx_set_form: "scaling" (matrix scaling with absorption; the
        default) or "log" (log-domain) for the fixed-T forward of later calls."""
        code = {"log": FR_FORM_LOG, "scaling": FR_FORM_SCALING}[form]
        _check(load().fr_ctx_set_form(self.handle, code, int(absorb_every)), "fr_ctx_set_form")

    def set_row_store(self, enable: bool = True):
        """fr_ctx_set_row_store: whether the tile forward keeps its row
        scalings for the reverse sweep (the default) or the sweep forms them."""
        _check(load().fr_ctx_set_row_store(self.handle, int(bool(enable))), "fr_ctx_set_row_store")

    def set_launch(self, n_items: int, m: int, lanes: int, rows: int):
        _check(load().fr_set_launch(self.handle, n_items, m, lanes, rows), "fr_set_launch")

    def autotune(self, prob: "Problem", C: Optional[torch.Tensor] = None, batched: bool = False,
                 iters: Optional[int] = None):
        """Times the launch shapes on this problem (min(T, iters) Sinkhorn
        iterations; all T by default) and keeps the fastest."""
        if iters is None:
            iters = prob.T
        if C is None:
            C = torch.zeros((prob.U, prob.I, prob.m), dtype=torch.float32, device=self.device)
        _f32(C, (prob.U, prob.I, prob.m), "C")
        ws = self.workspace(workspace_bytes(prob, 1))
        L, R = ctypes.c_int32(), ctypes.c_int32()
        p = prob.c()
        _check(load().fr_autotune(self.handle, ctypes.byref(p), _ptr(C), int(batched), int(iters),
                                  _ptr(ws), ws.numel(), _stream(self.device), ctypes.byref(L),
                                  ctypes.byref(R)), "fr_autotune")
        return L.value, R.value

    def get_launch(self, n_users: int, n_items: int, m: int):
        """(lanes, rows per lane) a problem of this shape runs with."""
        L, R = ctypes.c_int32(), ctypes.c_int32()
        _check(load().fr_get_launch(self.handle, n_users, n_items, m, ctypes.byref(L),
                                    ctypes.byref(R)), "fr_get_launch")
        return L.value, R.value


@dataclass
class Problem:
    """One instance: r [U, I] and e [m-1] float32 tensors on the device."""
    r: torch.Tensor
    e: torch.Tensor
    eps: float
    T: int

    @property
    def U(self):
        return self.r.shape[0]

    @property
    def I(self):
        return self.r.shape[1]

    @property
    def m(self):
        return self.e.shape[0] + 1

    def c(self) -> _Problem:
        for t, nm in ((self.r, "r"), (self.e, "e")):
            if t.dtype != torch.float32 or not t.is_contiguous() or not t.is_cuda:
                raise ValueError(f"{nm} must be a contiguous float32 CUDA tensor")
        return _Problem(self.U, self.I, self.m, self.r.data_ptr(), self.e.data_ptr(),
                        float(self.eps), int(self.T))


def _f32(t: torch.Tensor, shape, name):
    if t.dtype != torch.float32 or not t.is_contiguous() or not t.is_cuda or tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must be a contiguous float32 CUDA tensor of shape {tuple(shape)}")


def _optim(rule, lr, beta1, beta2, adam_eps, N, K, grad_tol=0.0, sinkhorn_tol=0.0,
           cg_iters=0) -> _Optim:
    return _Optim(FR_ADAM if rule == "adam" else FR_GD, float(lr), float(beta1), float(beta2),
                  float(adam_eps), int(N), int(K), float(grad_tol), float(sinkhorn_tol),
                  int(cg_iters))


def workspace_bytes(prob: Problem, K: int = 1) -> int:
    n = ctypes.c_size_t()
    o = _optim("adam", 0.0, 0.9, 0.999, 1e-8, 0, K)
    p = prob.c()
    _check(load().fr_workspace_bytes(ctypes.byref(p), ctypes.byref(o), ctypes.byref(n)),
           "fr_workspace_bytes")
    return n.value


def step(ctx: Context, prob: Problem, C: torch.Tensor, want_X: bool = False, x_dtype: str = "f32",
         want_pot: bool = False, sync: bool = True):
    """fr_step: X = Sinkhorn_T(C), Imp and F.  Returns dict(imp, F, X, pot)."""
    U, I, m = prob.U, prob.I, prob.m
    _f32(C, (U, I, m), "C")
    dev = C.device
    X = None
    if want_X:
        X = torch.empty((U, I, m), dtype=torch.bfloat16 if x_dtype == "bf16" else torch.float32,
                        device=dev)
    pot = torch.empty((U, I + m), dtype=torch.float32, device=dev) if want_pot else None
    imp = torch.empty(I, dtype=torch.float64, device=dev)
    F = torch.empty(1, dtype=torch.float64, device=dev)
    nb = workspace_bytes(prob, 1)
    ws = ctx.workspace(nb)
    p = prob.c()
    _check(load().fr_step(ctx.handle, ctypes.byref(p), _ptr(C), _ptr(X),
                          FR_BF16 if x_dtype == "bf16" else FR_F32, _ptr(pot), _ptr(imp), _ptr(F),
                          _ptr(ws), ws.numel(), _stream(dev)), "fr_step")
    if sync:
        _check(load().fr_sync_status(ctx.handle, _ptr(ws), _stream(dev)), "fr_step (device)")
    return {"imp": imp, "F": F, "X": X, "pot": pot}


def nsw(ctx: Context, prob: Problem, X: torch.Tensor, sync: bool = True):
    """fr_nsw: Imp and F of a given plan X [U, I, m] (float32 or bfloat16)."""
    U, I, m = prob.U, prob.I, prob.m
    if tuple(X.shape) != (U, I, m) or not X.is_contiguous():
        raise ValueError("X must be contiguous with shape (U, I, m)")
    if X.dtype not in (torch.float32, torch.bfloat16):
        raise ValueError("X must be float32 or bfloat16")
    imp = torch.empty(I, dtype=torch.float64, device=X.device)
    F = torch.empty(1, dtype=torch.float64, device=X.device)
    ws = ctx.workspace(workspace_bytes(prob, 1))
    p = prob.c()
    _check(load().fr_nsw(ctx.handle, ctypes.byref(p), _ptr(X),
                         FR_BF16 if X.dtype == torch.bfloat16 else FR_F32, _ptr(imp), _ptr(F),
                         _ptr(ws), ws.numel(), _stream(X.device)), "fr_nsw")
    if sync:
        _check(load().fr_sync_status(ctx.handle, _ptr(ws), _stream(X.device)), "fr_nsw (device)")
    return imp, F


METRIC_NAMES = ("user_utility", "mean_max_envy", "items_better", "items_worse")


def metrics(ctx: Context, prob: Problem, X: torch.Tensor, per_item: bool = False,
            sync: bool = True):
    """fr_metrics: user utility, mean max envy and the fractions of items better
    / worse off than under the uniform policy (Section 4.1) of a plan X
    [U, I, m] (float32 or bfloat16).  Returns the four values as a float64
    device tensor (and, with per_item, the per-item envy and impacts)."""
    U, I, m = prob.U, prob.I, prob.m
    if tuple(X.shape) != (U, I, m) or not X.is_contiguous():
        raise ValueError("X must be contiguous with shape (U, I, m)")
    if X.dtype not in (torch.float32, torch.bfloat16):
        raise ValueError("X must be float32 or bfloat16")
    p = prob.c()
    nb = ctypes.c_size_t()
    _check(load().fr_workspace_bytes_metrics(ctypes.byref(p), ctypes.byref(nb)),
           "fr_workspace_bytes_metrics")
    ws = torch.empty(max(nb.value, 256), dtype=torch.uint8, device=X.device)
    out = torch.empty(4, dtype=torch.float64, device=X.device)
    envy = torch.empty(I, dtype=torch.float64, device=X.device) if per_item else None
    imp = torch.empty(I, dtype=torch.float64, device=X.device) if per_item else None
    _check(load().fr_metrics(ctx.handle, ctypes.byref(p), _ptr(X),
                             FR_BF16 if X.dtype == torch.bfloat16 else FR_F32, _ptr(out),
                             _ptr(envy), _ptr(imp), _ptr(ws), ws.numel(), _stream(X.device)),
           "fr_metrics")
    if sync:
        torch.cuda.synchronize(X.device)
    return (out, envy, imp) if per_item else out


def backward(ctx: Context, prob: Problem, C: torch.Tensor, imp: torch.Tensor, gF: float = 1.0,
             want_dr: bool = True, K: int = 1, sync: bool = True):
    """fr_backward: (gF dF/dC, gF dF/dr) through the T unrolled iterations;
    with sync, the device flags are read (fr_sync_status) and raised."""
    U, I, m = prob.U, prob.I, prob.m
    _f32(C, (U, I, m), "C")
    if imp.dtype != torch.float64 or imp.numel() != I or not imp.is_cuda:
        raise ValueError("imp must be a float64 CUDA tensor of length I")
    imp = imp.contiguous()
    dC = torch.empty_like(C)
    dr = torch.empty((U, I), dtype=torch.float32, device=C.device) if want_dr else None
    ws = ctx.workspace(workspace_bytes(prob, K))
    p = prob.c()
    _check(load().fr_backward(ctx.handle, ctypes.byref(p), _ptr(C), _ptr(imp), float(gF), _ptr(dC),
                              _ptr(dr), int(K), _ptr(ws), ws.numel(), _stream(C.device)),
           "fr_backward")
    if sync:
        _check(load().fr_sync_status(ctx.handle, _ptr(ws), _stream(C.device)),
               "fr_backward (device)")
    return dC, dr


def _solve(fn, ctx, prob, N, lr, rule, beta1, beta2, adam_eps, C0, mom, vel, start_step, K,
           want_X, x_dtype, plain, grad_tol=0.0, sinkhorn_tol=0.0, cg_iters=0, inplace=False):
    U, I, m = prob.U, prob.I, prob.m
    dev = ctx.device

    def own(t):   # the caller's tensor itself (inplace) or a copy
        return t if inplace else t.clone()

    C = torch.zeros((U, I, m), dtype=torch.float32, device=dev) if C0 is None else own(C0)
    _f32(C, (U, I, m), "C")
    if rule == "adam":
        mom = torch.zeros_like(C) if mom is None else own(mom)
        vel = torch.zeros_like(C) if vel is None else own(vel)
        _f32(mom, (U, I, m), "mom")
        _f32(vel, (U, I, m), "vel")
    else:
        mom = vel = None
    X = None
    if want_X:
        X = torch.empty((U, I, m), dtype=torch.bfloat16 if x_dtype == "bf16" else torch.float32,
                        device=dev)
    Fh = torch.empty(N + 1, dtype=torch.float64, device=dev)
    o = _optim(rule, lr, beta1, beta2, adam_eps, N, K, grad_tol, sinkhorn_tol, cg_iters)
    p = prob.c()
    n = ctypes.c_size_t()
    if plain:
        _check(load().fr_workspace_bytes_plain(ctypes.byref(p), ctypes.byref(n)),
               "fr_workspace_bytes_plain")
    else:
        _check(load().fr_workspace_bytes(ctypes.byref(p), ctypes.byref(o), ctypes.byref(n)),
               "fr_workspace_bytes")
    ws = ctx.workspace(n.value)
    _check(fn(ctx.handle, ctypes.byref(p), ctypes.byref(o), _ptr(C), _ptr(mom), _ptr(vel),
              int(start_step), _ptr(X), FR_BF16 if x_dtype == "bf16" else FR_F32, _ptr(Fh),
              _ptr(ws), ws.numel(), _stream(dev)), "fr_solve_plain" if plain else "fr_solve")
    steps, gn, sk = ctypes.c_int64(), ctypes.c_double(), ctypes.c_int64()
    _check(load().fr_solve_progress(ctx.handle, _ptr(ws), _stream(dev), ctypes.byref(steps),
                                    ctypes.byref(gn), ctypes.byref(sk)), "fr_solve_progress")
    return {"C": C, "X": X, "F_hist": Fh, "mom": mom, "vel": vel,
            "updates": int(steps.value) - int(start_step), "last_gnorm": float(gn.value),
            "sinkhorn_iters": int(sk.value)}


def solve(ctx: Context, prob: Problem, N: int, lr: float, rule: str = "adam", beta1: float = 0.9,
          beta2: float = 0.999, adam_eps: float = 1e-8, C0=None, mom=None, vel=None,
          start_step: int = 0, K: int = 0, want_X: bool = True, x_dtype: str = "f32",
          grad_tol: float = 0.0, sinkhorn_tol: float = 0.0, cg_iters: int = 0,
          inplace: bool = False):
    """fr_solve: Algorithm 1 with at most N ascent steps (captured as a HIP
    graph); grad_tol = t > 0 ends the loop at the first ||dF/dC||_F <= t;
    sinkhorn_tol > 0 selects the converged-map form (warm starts, tolerance,
    implicit gradients).  The result's "updates" counts the updates applied,
    "sinkhorn_iters" the Sinkhorn iterations of the converged-map form.
    With inplace=True the given C0, mom and vel are updated in place (a
    trajectory continued from start_step without copying its state)."""
    return _solve(load().fr_solve, ctx, prob, N, lr, rule, beta1, beta2, adam_eps, C0, mom, vel,
                  start_step, K, want_X, x_dtype, False, grad_tol, sinkhorn_tol, cg_iters,
                  inplace)


def grad_converged(ctx: Context, prob: Problem, C: torch.Tensor, sinkhorn_tol: float,
                   gF: float = 1.0, cg_iters: int = 0, want_dr: bool = True, sync: bool = True):
    """fr_grad_converged: Imp and F of the converged plan of C and gF * dF/dC
    (and dF/dr) by the implicit function theorem."""
    U, I, m = prob.U, prob.I, prob.m
    _f32(C, (U, I, m), "C")
    imp = torch.empty(I, dtype=torch.float64, device=C.device)
    F = torch.empty(1, dtype=torch.float64, device=C.device)
    dC = torch.empty_like(C)
    dr = torch.empty((U, I), dtype=torch.float32, device=C.device) if want_dr else None
    n = ctypes.c_size_t()
    o = _optim("adam", 0.0, 0.9, 0.999, 1e-8, 0, 1, 0.0, sinkhorn_tol)
    p = prob.c()
    _check(load().fr_workspace_bytes(ctypes.byref(p), ctypes.byref(o), ctypes.byref(n)),
           "fr_workspace_bytes")
    ws = ctx.workspace(n.value)
    _check(load().fr_grad_converged(ctx.handle, ctypes.byref(p), _ptr(C), float(sinkhorn_tol),
                                    int(cg_iters), float(gF), _ptr(imp), _ptr(F), _ptr(dC),
                                    _ptr(dr), _ptr(ws), ws.numel(), _stream(C.device)),
           "fr_grad_converged")
    if sync:
        _check(load().fr_sync_status(ctx.handle, _ptr(ws), _stream(C.device)),
               "fr_grad_converged (device)")
    return {"imp": imp, "F": F, "dC": dC, "dr": dr}


def solve_plain(ctx: Context, prob: Problem, N: int, lr: float, rule: str = "adam",
                beta1: float = 0.9, beta2: float = 0.999, adam_eps: float = 1e-8, C0=None,
                mom=None, vel=None, start_step: int = 0, want_X: bool = True,
                x_dtype: str = "f32", grad_tol: float = 0.0):
    """fr_solve_plain: the unfused baseline form (one launch per half-iteration)."""
    return _solve(load().fr_solve_plain, ctx, prob, N, lr, rule, beta1, beta2, adam_eps, C0, mom,
                  vel, start_step, 1, want_X, x_dtype, True, grad_tol)


def solve_batched(ctx: Context, probs, N: int, lr: float, rule: str = "adam", beta1: float = 0.9,
                  beta2: float = 0.999, adam_eps: float = 1e-8, C0=None, K: int = 1,
                  want_X: bool = True, x_dtype: str = "f32"):
    """fr_solve_batched: Algorithm 1 on many instances at once (persistent
    kernels, one graph per outer step).  Returns a list of dicts like solve()."""
    n = len(probs)
    dev = ctx.device
    Cs, Ms, Vs, Xs, Fs = [], [], [], [], []
    for j, p in enumerate(probs):
        C = torch.zeros((p.U, p.I, p.m), dtype=torch.float32, device=dev) if C0 is None \
            else C0[j].clone()
        _f32(C, (p.U, p.I, p.m), "C")
        Cs.append(C)
        if rule == "adam":
            Ms.append(torch.zeros_like(C))
            Vs.append(torch.zeros_like(C))
        Xs.append(torch.empty((p.U, p.I, p.m), dtype=torch.bfloat16 if x_dtype == "bf16"
                              else torch.float32, device=dev) if want_X else None)
        Fs.append(torch.empty(N + 1, dtype=torch.float64, device=dev))
    PArr = _Problem * n
    parr = PArr(*[p.c() for p in probs])
    VP = ctypes.c_void_p * n
    cptr = VP(*[t.data_ptr() for t in Cs])
    mptr = VP(*[t.data_ptr() for t in Ms]) if rule == "adam" else None
    vptr = VP(*[t.data_ptr() for t in Vs]) if rule == "adam" else None
    xptr = VP(*[(t.data_ptr() if t is not None else None) for t in Xs]) if want_X else None
    fptr = VP(*[t.data_ptr() for t in Fs])
    o = _optim(rule, lr, beta1, beta2, adam_eps, N, K)
    nb = ctypes.c_size_t()
    lib = load()
    _check(lib.fr_workspace_bytes_batched(n, parr, ctypes.byref(o), ctypes.byref(nb)),
           "fr_workspace_bytes_batched")
    ws = ctx.workspace(nb.value)
    _check(lib.fr_solve_batched(ctx.handle, n, parr, ctypes.byref(o), cptr, mptr, vptr, 0, xptr,
                                FR_BF16 if x_dtype == "bf16" else FR_F32, fptr, _ptr(ws),
                                ws.numel(), _stream(dev)), "fr_solve_batched")
    return [{"C": Cs[j], "X": Xs[j], "F_hist": Fs[j], "mom": Ms[j] if Ms else None,
             "vel": Vs[j] if Vs else None} for j in range(n)]


# --------------------------------------------------------------------------
class SinkhornNSW(torch.autograd.Function):
    """F = sum_i log Imp_i(X_T(C)) as a differentiable function of (C, r).

    forward calls fr_step; backward calls fr_backward, which recomputes the
    Sinkhorn iterations from C with potentials checkpointed every K."""

    @staticmethod
    def forward(actx, C, r, e, eps, T, K, fr_ctx):
        prob = Problem(r.detach().contiguous(), e.detach().contiguous(), float(eps), int(T))
        out = step(fr_ctx, prob, C.detach().contiguous())
        actx.save_for_backward(C, out["imp"])
        actx.prob = prob
        actx.K = int(K)
        actx.fr_ctx = fr_ctx
        return out["F"][0]

    @staticmethod
    def backward(actx, gF):
        C, imp = actx.saved_tensors
        dC, dr = backward(actx.fr_ctx, actx.prob, C.detach().contiguous(), imp, float(gF.item()),
                          want_dr=actx.needs_input_grad[1], K=actx.K)
        return dC, dr, None, None, None, None, None


def sinkhorn_nsw(C, r, e, eps, T, K=50, ctx: Optional[Context] = None):
    """Differentiable log-NSW objective of the Sinkhorn plans of C."""
    ctx = ctx or _default_ctx(C.device)
    return SinkhornNSW.apply(C, r, e, eps, T, K, ctx)


_ctxs = {}


def _default_ctx(device) -> Context:
    idx = device.index if device.index is not None else torch.cuda.current_device()
    if idx not in _ctxs:
        _ctxs[idx] = Context(idx)
    return _ctxs[idx]


def _rank(fn, ctx: Context, prob: Problem, want_X: bool, x_dtype: str, want_imp: bool):
    U, I, m = prob.U, prob.I, prob.m
    dev = ctx.device
    sel = torch.empty((U, m - 1), dtype=torch.int32, device=dev)
    X = None
    if want_X:
        X = torch.empty((U, I, m), dtype=torch.bfloat16 if x_dtype == "bf16" else torch.float32,
                        device=dev)
    imp = torch.empty(I, dtype=torch.float64, device=dev) if want_imp else None
    p = prob.c()
    xd = FR_BF16 if x_dtype == "bf16" else FR_F32
    if fn == "greedy":
        code = load().fr_rank_greedy(ctx.handle, ctypes.byref(p), _ptr(sel), _ptr(X), xd,
                                     _ptr(imp), _stream(dev))
    else:
        code = load().fr_rank_maxrele(ctx.handle, ctypes.byref(p), _ptr(sel), _ptr(X), xd,
                                      _stream(dev))
    _check(code, "fr_rank_" + fn)
    return {"sel": sel, "X": X, "imp": imp}


def rank_maxrele(ctx: Context, prob: Problem, want_X: bool = True, x_dtype: str = "f32"):
    """fr_rank_maxrele: the MaxRele baseline.  Returns dict(sel [U][m-1], X)."""
    return _rank("maxrele", ctx, prob, want_X, x_dtype, False)


def rank_greedy(ctx: Context, prob: Problem, want_X: bool = True, x_dtype: str = "f32"):
    """fr_rank_greedy: the NSW(Greedy) baseline.  Returns dict(sel, X, imp)."""
    return _rank("greedy", ctx, prob, want_X, x_dtype, True)
