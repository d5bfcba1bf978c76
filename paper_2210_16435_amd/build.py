"""Compile the HIP library libsfairsc.so for gfx950 (in-tree).

Each source compiles to an object in parallel; the objects are linked into
paper_2210_16435_amd/libsfairsc.so.  hipcc cross-compiles for the GPU, so
this runs on a machine without one.
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
LIB = os.path.join(HERE, "libsfairsc.so")
ARCH = "gfx950"

HIP_SOURCES = ["graph.hip", "operator.hip", "general.hip", "lsqr.hip", "ortho.hip", "rr.hip", "eigs.hip", "kmeans.hip",
               "backward.hip", "batched.hip"]
CXX_SOURCES = []

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
HIP_FLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-fPIC",
    "-std=c++17",
    "-Wno-unused-result",
    # no packed FP32 instructions in device code
    "-Xclang",
    "-target-feature",
    "-Xclang",
    "-packed-fp32-ops",
]

# Per-source extra options (none: every source builds with the same flags).
HIP_EXTRA = {}


def _run(cmd):
    p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if p.returncode != 0:
        raise RuntimeError("build failed:\n" + " ".join(cmd) + "\n" + p.stdout)
    return p.stdout


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = []
    objs = []
    for src in HIP_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        objs.append(obj)
        jobs.append([HIPCC, *HIP_FLAGS, *HIP_EXTRA.get(src, []), "-c", os.path.join(CSRC, src), "-o", obj])
    for src in CXX_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        objs.append(obj)
        jobs.append(["g++", "-O3", "-march=x86-64-v3", "-fopenmp-simd", "-fPIC", "-std=c++17", "-c",
                     os.path.join(CSRC, src), "-o", obj])
    workers = max(1, min(len(jobs), os.cpu_count() or 1, 8))
    with cf.ThreadPoolExecutor(workers) as ex:
        for out in ex.map(_run, jobs):
            if verbose and out:
                print(out)
    tmp = LIB + ".tmp"
    _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
