"""Builds libfairrank.so (the HIP library behind include/fairrank.h) for gfx950.

Every column class of the fused kernels is its own translation unit
(fr_fused.hip with -DFR_MP=<mp>), compiled in parallel with hipcc and linked
into one shared library next to this file.

    python -m paper_2406_10262_amd.build
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libfairrank.so")

MP_CLASSES = (5, 8, 10, 11, 12, 16, 20, 24, 32, 40, 48, 50, 64)


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


# Packed FP32 instructions stay disabled: plain float code is compiled to
# single-lane FP32 VALU operations only.
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-command-line-argument"]


def _units():
    units = []
    for mp in MP_CLASSES:
        units.append((os.path.join(CSRC, "fr_fused.hip"), os.path.join(BUILD, f"fr_fused_{mp}.o"),
                      [f"-DFR_MP={mp}"]))
    for name in ("fr_tile", "fr_reduce", "fr_plain", "fr_metrics", "fr_baselines", "fr_diag",
                 "fr_api"):
        src = os.path.join(CSRC, name + ".hip")
        if os.path.exists(src):
            units.append((src, os.path.join(BUILD, name + ".o"), []))
    return units


def _compile(unit):
    src, obj, extra = unit
    cmd = [hipcc()] + FLAGS + extra + ["-c", src, "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed for {os.path.basename(obj)}:\n{res.stderr}")
    return obj


def build(jobs: int | None = None, verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    units = _units()
    jobs = jobs or min(len(units), max(1, min(16, os.cpu_count() or 1)))
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(_compile, units))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed:\n{res.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
