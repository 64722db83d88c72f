"""Build libmgs.so (the C-ABI HIP library) in-tree with hipcc for gfx950.

Usage: ``python -m paper_2603_11531_amd.build`` (or ``build()`` from Python).
Every ``csrc/*.hip`` file is compiled to an object in ``_build/`` and linked
into ``paper_2603_11531_amd/libmgs.so``.  Objects are compiled in parallel.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libmgs.so")

ARCH = "gfx950"
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
CFLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17", "-I", INCLUDE, "-I", CSRC,
    # packed-FP32 VALU forms are disabled on purpose (float code is emitted unpacked)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # no implicit multiply-add contraction: every kernel that shares device code rounds the same
    # way (hot loops use explicit fmaf), so a batched render equals the single-view render bit for bit
    "-ffp-contract=off",
    "-munsafe-fp-atomics", "-Wno-unused-result",
    # matrix-instruction results in ordinary VGPRs (gfx950 allows it): no copies out of AGPRs
    # before the vector ALU can use them
    "-mllvm", "-amdgpu-mfma-vgpr-form",
]


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


CHECKED_LIB = os.path.join(PKG, "libmgs_checked.so")


def _compile(src, checked=False):
    obj = os.path.join(BUILD, os.path.basename(src)[:-4] + (".checked.o" if checked else ".o"))
    cmd = [HIPCC, *CFLAGS, *(["-DMGS_CHECK_BOUNDS"] if checked else []), "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


REFSORT_SRC = os.path.join(PKG, "refsort", "sort_reference.hip")
REFSORT_LIB = os.path.join(PKG, "libmgs_refsort.so")


def _build_refsort():
    """The measurement-only reference sort (ROCm's library radix sort), a library of its own."""
    tmp = REFSORT_LIB + ".tmp"
    cmd = [HIPCC, *CFLAGS, "-shared", REFSORT_SRC, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {REFSORT_SRC}:\n{r.stderr}")
    os.replace(tmp, REFSORT_LIB)
    return REFSORT_LIB


def _link(objs, lib):
    tmp = lib + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs, "-L/opt/rocm/lib",
           "-Wl,-rpath,/opt/rocm/lib", "-lrocprofiler-sdk-roctx"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, lib)


def build(verbose=False):
    """libmgs.so, libmgs_checked.so (the same sources with MGS_CHECK_BOUNDS: kernels check the
    indices they derive and report failures through mgs_bounds_status) and libmgs_refsort.so."""
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    with cf.ThreadPoolExecutor(max_workers=8) as ex:
        ref = ex.submit(_build_refsort)
        objs = list(ex.map(_compile, srcs))
        objs_checked = list(ex.map(lambda src: _compile(src, checked=True), srcs))
        ref.result()
    _link(objs, LIB)
    _link(objs_checked, CHECKED_LIB)
    if verbose:
        print(f"built {LIB} from {len(srcs)} sources, {CHECKED_LIB} and {REFSORT_LIB}")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
