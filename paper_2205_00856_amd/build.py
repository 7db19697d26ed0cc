"""Builds the HIP library libcntri.so for gfx950 in-tree (hipcc cross-compiles without a GPU).

The kernels are split over several translation units (csrc/kern_*.hip, one group of kernel
instantiations each) that compile in parallel; csrc/cntri.hip holds the host runtime and the
C ABI.  Objects go to paper_2205_00856_amd/_build/, the library to paper_2205_00856_amd/.
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libcntri.so")
HEADER = os.path.join(ROOT, "include", "cntri.h")

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # packed FP32 VALU forms are kept out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
]


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def deps():
    return sources() + sorted(glob.glob(os.path.join(CSRC, "*.hpp"))) + [HEADER]


def hipcc() -> str:
    for p in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if p and (os.path.sep not in p or os.path.exists(p)):
            return p
    raise RuntimeError("hipcc not found")


def _jobs() -> int:
    n = os.cpu_count() or 1
    for var in ("MAX_JOBS", "CMAKE_BUILD_PARALLEL_LEVEL"):
        v = os.environ.get(var)
        if v and v.isdigit():
            n = min(n, int(v))
    return max(1, min(n, 16))


def build(force: bool = True, verbose: bool = False) -> str:
    newest = max(os.path.getmtime(d) for d in deps())
    stale = not os.path.exists(LIB) or newest > os.path.getmtime(LIB)
    if not force and not stale:
        return LIB
    os.makedirs(BUILD, exist_ok=True)
    cc = hipcc()
    objs, pending = [], []
    for src in sources():
        obj = os.path.join(BUILD, os.path.splitext(os.path.basename(src))[0] + ".o")
        objs.append(obj)
        pending.append([cc, *HIPCC_FLAGS, "-c", "-o", obj, src])
    running = []
    failed = None
    jobs = _jobs()
    while pending or running:
        while pending and len(running) < jobs and failed is None:
            cmd = pending.pop(0)
            if verbose:
                print(" ".join(cmd), flush=True)
            running.append((cmd, subprocess.Popen(cmd)))
        cmd, p = running.pop(0)
        if p.wait() != 0 and failed is None:
            failed = cmd
        if failed is not None:
            pending.clear()
    if failed is not None:
        raise subprocess.CalledProcessError(1, failed)
    tmp = LIB + ".tmp"
    link = [cc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.check_call(link)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(force=True, verbose=True)
    sys.exit(0)
