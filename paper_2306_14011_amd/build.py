"""Build ``libfv.so`` (the HIP library behind ``include/fv.h``) for gfx950, in-tree.

Usage: ``python -m paper_2306_14011_amd.build`` or ``build()`` from Python.
The library is compiled by hipcc with ``--offload-arch=gfx950``; packed FP32
instructions are disabled for every HIP source.
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libfv.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

HIP_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


# Per-source extra flags. The split path's face kernels (one face per thread,
# and the variant that walks runs of faces) must give the same bits for every
# launch table; contracting multiply-adds only within one source expression
# makes the fused multiply-adds independent of how the compiler shares
# subexpressions between the faces a thread computes. The same holds for the
# 3D stage kernels and the curvilinear 2D ones, whose first face of a work
# item is computed before the plane or row loop and the others inside it:
# every segment height must give the same bits.
FILE_FLAGS = {"fv_kernels.hip": ["-ffp-contract=on"], "fv_fused3d.hip": ["-ffp-contract=on"],
              "fv_fused_curv.hip": ["-ffp-contract=on"]}


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def build(verbose=False, jobs=None):
    """Compile every HIP source to an object, then link the shared library."""
    objdir = os.path.join(PKG, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs = []
    procs = []
    for src in sources():
        obj = os.path.join(objdir, os.path.basename(src) + ".o")
        cmd = [HIPCC, *HIP_FLAGS, *FILE_FLAGS.get(os.path.basename(src), []), "-I", os.path.join(ROOT, "include"),
               "-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd)))
        objs.append(obj)
    bad = [src for src, p in procs if p.wait() != 0]
    if bad:
        raise RuntimeError("hipcc failed on: " + ", ".join(bad))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-q" not in sys.argv)
