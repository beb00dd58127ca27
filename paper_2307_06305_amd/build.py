"""Build libdamn.so in-tree with hipcc for gfx950.

Usage: python -m paper_2307_06305_amd.build   (or build() from Python)

Each source compiles to an object under _build/ in parallel, then one link.
The library always rebuilds when build() is called.
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
LIB = os.path.join(PKG, "libdamn.so")

ARCH = "gfx950"
HIP_SOURCES = ["spmv_kernels.hip", "spmv_grid.hip", "spmv_bsr.hip", "spmv_coo.hip",
               "spmm_stream.hip", "api.hip", "cg.hip", "batch.hip", "selector.hip"]
CPP_SOURCES = ["host_format.cpp", "host_grid.cpp", "host_blocks.cpp", "host_rcm.cpp",
               "host_features.cpp"]

COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function", f"-I{INCLUDE}", f"-I{CSRC}"]
# packed fp32 vector instructions are disabled for device code
HIP_FLAGS = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-munsafe-fp-atomics"]


def _hipcc():
    for c in ("/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def _compile(src):
    hipcc = _hipcc()
    path = os.path.join(CSRC, src)
    obj = os.path.join(BUILD, src + ".o")
    if src.endswith(".hip"):
        cmd = [hipcc, "-x", "hip", *COMMON, *HIP_FLAGS, "-c", path, "-o", obj]
    else:
        cmd = [hipcc, "-x", "c++", *COMMON, "-c", path, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


CPU_SRC = os.path.join(PKG, "cpu", "cpu_spmv.cpp")
CPU_LIB = os.path.join(PKG, "cpu", "libdamn_cpu.so")


def _build_cpu():
    """The native CPU baseline (OpenMP), a library of its own."""
    tmp = CPU_LIB + ".tmp"
    cmd = ["g++", "-O3", "-march=x86-64-v3", "-std=c++17", "-fPIC", "-shared", "-fopenmp",
           CPU_SRC, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, CPU_LIB)
    return CPU_LIB


def build(verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    srcs = HIP_SOURCES + CPP_SOURCES
    jobs = min(len(srcs), max(1, os.cpu_count() or 1))
    with cf.ThreadPoolExecutor(jobs) as ex:
        cpu = ex.submit(_build_cpu)
        objs = list(ex.map(_compile, srcs))
        cpu.result()
    tmp = LIB + ".tmp"
    cmd = [_hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp, "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
