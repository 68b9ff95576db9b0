"""The C-ABI library: it loads, exports every entry point that
include/fairrank.h declares, and rejects bad arguments on the host before
touching the device.  No call here launches GPU work."""
import ctypes
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fairrank.h")
DIAG_HEADER = os.path.join(ROOT, "include", "fairrank_diag.h")


@pytest.fixture(scope="module")
def lib():
    import paper_2406_10262_amd as fr
    if not os.path.exists(fr.library_path()):
        from paper_2406_10262_amd import build
        build.build(verbose=False)
    return fr.load()


def declared_functions(path=HEADER):
    src = open(path).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:fr_status|void|const char\*|size_t)\s+(fr_\w+)\s*\(",
                                 src, flags=re.M)))


def test_header_declares_the_core_entry_points():
    names = declared_functions()
    for n in ("fr_step", "fr_nsw", "fr_backward", "fr_solve", "fr_solve_plain", "fr_ctx_create",
              "fr_workspace_bytes", "fr_sync_status", "fr_status_string"):
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    import paper_2406_10262_amd as fr
    out = subprocess.run(["nm", "-D", "--defined-only", fr.library_path()], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT\s+(fr_\w+)", out))
    names = declared_functions() + declared_functions(DIAG_HEADER)
    assert "fr_ctx_kernel_forms" in names and "fr_rank_greedy" in names
    for n in names:
        assert n in exported, n
        assert hasattr(lib, n)


def _prob(fr, U=10, I=20, m=5, r=1, e=1, eps=0.05, T=10):
    return fr._Problem(U, I, m, r, e, eps, T)


def test_workspace_validation(lib):
    import paper_2406_10262_amd as fr
    n = ctypes.c_size_t()
    assert lib.fr_workspace_bytes(None, None, ctypes.byref(n)) == 1
    assert lib.fr_workspace_bytes(ctypes.byref(_prob(fr)), None, None) == 1
    bad_shapes = [dict(U=0), dict(I=1), dict(m=1), dict(m=21), dict(I=5000, m=5), dict(I=100, m=65)]
    for kw in bad_shapes:
        assert lib.fr_workspace_bytes(ctypes.byref(_prob(fr, **kw)), None, ctypes.byref(n)) == 2, kw
    for kw in (dict(eps=0.0), dict(eps=-1.0), dict(eps=float("nan")), dict(eps=float("inf")),
               dict(T=0)):
        assert lib.fr_workspace_bytes(ctypes.byref(_prob(fr, **kw)), None, ctypes.byref(n)) == 3, kw
    assert lib.fr_workspace_bytes(ctypes.byref(_prob(fr, r=0)), None, ctypes.byref(n)) == 1
    assert lib.fr_workspace_bytes(ctypes.byref(_prob(fr)), None, ctypes.byref(n)) == 0
    o = fr._Optim(0, 0.01, 0.9, 0.999, 1e-8, 5, 1)
    assert lib.fr_workspace_bytes(ctypes.byref(_prob(fr, T=200)), ctypes.byref(o),
                                  ctypes.byref(n)) == 0
    all_iters = n.value
    o.checkpoint_every = 50
    assert lib.fr_workspace_bytes(ctypes.byref(_prob(fr, T=200)), ctypes.byref(o),
                                  ctypes.byref(n)) == 0
    assert n.value < all_iters


def test_entry_points_reject_null_context(lib):
    import paper_2406_10262_amd as fr
    p = _prob(fr)
    o = fr._Optim(0, 0.01, 0.9, 0.999, 1e-8, 5, 1)
    assert lib.fr_step(None, ctypes.byref(p), 1, None, 0, None, None, None, 1, 10**9, None) == 1
    assert lib.fr_nsw(None, ctypes.byref(p), 1, 0, None, None, 1, 10**9, None) == 1
    assert lib.fr_backward(None, ctypes.byref(p), 1, 1, 1.0, 1, None, 1, 1, 10**9, None) == 1
    assert lib.fr_solve(None, ctypes.byref(p), ctypes.byref(o), 1, 1, 1, 0, None, 0, 1, 1,
                        10**9, None) == 1
    assert lib.fr_sync_status(None, 1, None) == 1
    assert lib.fr_set_launch(None, 20, 5, 64, 1) == 1
    assert lib.fr_metrics(None, ctypes.byref(p), 1, 0, 1, None, None, 1, 10**9, None) == 1


def test_metrics_workspace_validation(lib):
    import paper_2406_10262_amd as fr
    n = ctypes.c_size_t()
    assert lib.fr_workspace_bytes_metrics(None, ctypes.byref(n)) == 1
    assert lib.fr_workspace_bytes_metrics(ctypes.byref(_prob(fr)), None) == 1
    assert lib.fr_workspace_bytes_metrics(ctypes.byref(_prob(fr, U=0)), ctypes.byref(n)) == 2
    assert lib.fr_workspace_bytes_metrics(ctypes.byref(_prob(fr, eps=0.0)), ctypes.byref(n)) == 3
    assert lib.fr_workspace_bytes_metrics(ctypes.byref(_prob(fr)), ctypes.byref(n)) == 0
    small = n.value
    assert lib.fr_workspace_bytes_metrics(ctypes.byref(_prob(fr, U=1000)), ctypes.byref(n)) == 0
    assert n.value > small


def test_status_strings(lib):
    for code in range(9):
        assert len(lib.fr_status_string(code)) > 0
    assert lib.fr_status_string(99) == b"unknown status"


@pytest.mark.skipif(os.environ.get("HIP_VISIBLE_DEVICES") is None and
                    os.path.exists("/dev/kfd") and os.access("/dev/kfd", os.R_OK),
                    reason="a GPU may be present")
def test_context_creation_without_device_fails_cleanly(lib):
    h = ctypes.c_void_p()
    assert lib.fr_ctx_create(0, ctypes.byref(h)) == 5
    assert lib.fr_ctx_create(0, None) == 1


def test_product_package_never_touches_the_oracle():
    pkg = os.path.join(ROOT, "paper_2406_10262_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"^\s*(import|from)\s+oracle\b", txt, flags=re.M), f
                assert "fr_oracle" not in txt, f


def test_missing_library_fails_loudly(tmp_path):
    code = ("import paper_2406_10262_amd as fr\n"
            "fr._LIB_PATH = '/nonexistent/libfairrank.so'\n"
            "try:\n    fr.load()\nexcept FileNotFoundError:\n    print('raised')\n")
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True)
    assert "raised" in out.stdout, out.stderr


def test_gradient_norm_stop_needs_gradient_room(lib):
    import paper_2406_10262_amd as fr
    n0, n1 = ctypes.c_size_t(), ctypes.c_size_t()
    o = fr._Optim(0, 0.01, 0.9, 0.999, 1e-8, 5, 1)
    assert lib.fr_workspace_bytes(ctypes.byref(_prob(fr)), ctypes.byref(o), ctypes.byref(n0)) == 0
    o.grad_tol = 1e-3
    assert lib.fr_workspace_bytes(ctypes.byref(_prob(fr)), ctypes.byref(o), ctypes.byref(n1)) == 0
    assert n1.value >= n0.value + 10 * 20 * 5 * 4
    assert lib.fr_solve_progress(None, 1, None, None, None, None) == 1


def test_converged_map_form_validation(lib):
    import paper_2406_10262_amd as fr
    p = _prob(fr)
    n0, n1 = ctypes.c_size_t(), ctypes.c_size_t()
    o = fr._Optim(0, 0.01, 0.9, 0.999, 1e-8, 5, 1)
    assert lib.fr_workspace_bytes(ctypes.byref(p), ctypes.byref(o), ctypes.byref(n0)) == 0
    o.sinkhorn_tol = 1e-4
    assert lib.fr_workspace_bytes(ctypes.byref(p), ctypes.byref(o), ctypes.byref(n1)) == 0
    assert n1.value >= n0.value + 10 * 8 * 4        # warm-start potentials per consumer
    for tol, cg in ((float("nan"), 0), (float("inf"), 0), (-1e-3, 0), (1e-3, -1)):
        o.sinkhorn_tol, o.cg_iters = tol, cg
        assert lib.fr_workspace_bytes(ctypes.byref(p), ctypes.byref(o), ctypes.byref(n1)) == 3
    assert lib.fr_grad_converged(None, ctypes.byref(p), 1, 1e-4, 0, 1.0, None, None, 1, None, 1,
                                 10**9, None) == 1


def test_newer_entry_points_reject_null_context(lib):
    import paper_2406_10262_amd as fr
    p = _prob(fr)
    assert lib.fr_ctx_set_form(None, 0, 0) == 1
    assert lib.fr_rank_maxrele(None, ctypes.byref(p), 1, None, 0, None) == 1
    assert lib.fr_rank_greedy(None, ctypes.byref(p), 1, None, 0, None, None) == 1
    lib.fr_ctx_kernel_forms.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                                        ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                        ctypes.c_void_p]
    assert lib.fr_ctx_kernel_forms(None, 10, 20, 5, 0, None, None) == 1
    lib.fr_ctx_bwd_lds_rows.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                                        ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p]
    rows = ctypes.c_int32()
    assert lib.fr_ctx_bwd_lds_rows(None, 10, 20, 5, 0, ctypes.byref(rows)) == 1
    assert lib.fr_solve_progress(None, 1, None, None, None, None) == 1
