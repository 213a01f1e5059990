"""Build the HIP library ``libdslash.so`` in-tree for gfx950.

Every source under ``csrc/`` is compiled with hipcc (HIP mode, -O3, packed
FP32 instructions disabled) into an object file under ``_build/``, and the
objects are linked into ``paper_1808_05506_amd/libdslash.so``.  The
microbenchmarks under ``microbench/`` (stand-alone programs, not part of the
library) are built beside their sources.  Always rebuilds everything; sources
are compiled in parallel.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libdslash.so")
ARCH = "gfx950"

SOURCES = ["apply.hip", "apply_rows.hip", "staggered_rows.hip", "brillouin_rows.hip", "grad_rows.hip", "links_grad.hip", "eo.hip", "clover.hip", "bri_grad.hip", "blas.hip", "capi.cpp", "solver.cpp"]

FLAGS = [
    "-x", "hip", f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument", "-I", os.path.join(ROOT, "include"),
]


def _hipcc() -> str:
    for c in ("/opt/rocm/bin/hipcc", shutil.which("hipcc") or ""):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def _compile(hipcc: str, src: str, extra) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc, *FLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    return obj


MICROBENCH = os.path.join(HERE, "microbench")
MICROBENCH_SOURCES = ["fp32_contraction.hip"]


def _microbench(hipcc: str, src: str) -> str:
    exe = os.path.join(MICROBENCH, os.path.splitext(src)[0])
    cmd = [hipcc, *FLAGS, os.path.join(MICROBENCH, src), "-o", exe]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    return exe


def build(verbose: bool = False, extra=()) -> str:
    hipcc = _hipcc()
    os.makedirs(BUILD, exist_ok=True)
    jobs = min(len(SOURCES), max(1, (os.cpu_count() or 2)))
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda s: _compile(hipcc, s, list(extra)), SOURCES))
        exes = list(ex.map(lambda s: _microbench(hipcc, s), MICROBENCH_SOURCES))
    tmp = LIB + ".tmp"
    cmd = [hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
        for exe in exes:
            print(f"built {exe}")
    return LIB


if __name__ == "__main__":
    build(verbose=True, extra=sys.argv[1:])
