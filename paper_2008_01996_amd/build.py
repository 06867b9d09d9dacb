"""Build the stfd shared library (host C++ with OpenMP + HIP kernels for gfx950).

    python -m paper_2008_01996_amd.build        # or build() from Python

Produces paper_2008_01996_amd/libstfd.so next to this file.  Object files go
to paper_2008_01996_amd/_build/.  hipcc cross-compiles for gfx950, so this
runs on a machine without a GPU.
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
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libstfd.so")
INCLUDE = os.path.join(ROOT, "include")

HOST_SOURCES = ["host_linalg.cpp", "host_time.cpp", "host_space.cpp"]
HIP_HOST_SOURCES = ["stfd_api.cpp"]
HIP_SOURCES = ["kernels_band.hip", "kernels_sweep.hip", "kernels_gemm.hip", "kernels_tile.hip",
               "stfd_noalloc.hip"]

ARCH = "gfx950"
# packed FP32 instructions are switched off for all device code
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _run(cmd):
    p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if p.returncode != 0:
        raise RuntimeError("build step failed:\n" + " ".join(cmd) + "\n" + p.stdout)
    return p.stdout


def build(verbose: bool = False) -> str:
    """Compile every source and link libstfd.so; returns the library path."""
    os.makedirs(BUILD, exist_ok=True)
    hipcc = _hipcc()
    common = ["-O3", "-fPIC", "-std=c++17", "-I", INCLUDE, "-I", CSRC]
    # host code: complex products and quotients by the plain formulas, without
    # the inf/NaN recovery path that keeps them from vectorising (the setup's
    # values are nowhere near the range where that matters)
    host = ["-fcx-limited-range"]
    jobs = []
    for src in HOST_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        jobs.append(["g++", *common, *host, "-fopenmp", "-march=x86-64-v2", "-c", os.path.join(CSRC, src), "-o", obj])
    for src in HIP_HOST_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        jobs.append([hipcc, *common, *host, "-c", os.path.join(CSRC, src), "-o", obj])
    for src in HIP_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        jobs.append([hipcc, *common, f"--offload-arch={ARCH}", *DEVICE_FLAGS, "-c",
                     os.path.join(CSRC, src), "-o", obj])
    with cf.ThreadPoolExecutor(max_workers=min(8, len(jobs))) as ex:
        outs = list(ex.map(_run, jobs))
    if verbose:
        for o in outs:
            if o.strip():
                print(o)
    objs = [j[-1] for j in jobs]
    tmp = LIB + ".tmp"
    _run([hipcc, "-shared", "-fPIC", "-o", tmp, *objs, "-lgomp", "-Wl,-rpath,/opt/rocm/lib"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    path = build(verbose="-v" in sys.argv)
    print(path)
