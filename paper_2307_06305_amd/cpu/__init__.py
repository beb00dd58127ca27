"""The native CPU baseline of the products (DA-CSR and CSR SpMV with OpenMP),
for comparison in the benchmark only.  Built by the package build into
cpu/libdamn_cpu.so; it is a separate library and never a fallback for the
GPU path."""

from __future__ import annotations

import ctypes as C
import os

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libdamn_cpu.so")
_lib = None


def _get():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build with `python -m paper_2307_06305_amd.build`")
        lib = C.CDLL(LIB_PATH)
        p = C.c_void_p
        for name in ("damn_cpu_spmv_da", "damn_cpu_spmv_csr"):
            f = getattr(lib, name)
            f.restype = None
            f.argtypes = [C.c_int32, p, p, p, p, p, C.c_int]
        lib.damn_cpu_threads.restype = C.c_int
        _lib = lib
    return _lib


def threads():
    return _get().damn_cpu_threads()


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


def spmv_da(nrows, rowptr, off, vals, x, y, nthreads):
    """y = A x for DA-CSR host arrays (int32 rowptr, int16 off, float64)."""
    _get().damn_cpu_spmv_da(nrows, _p(rowptr), _p(off), _p(vals), _p(x), _p(y), int(nthreads))


def spmv_csr(nrows, rowptr, cols, vals, x, y, nthreads):
    """y = A x for CSR host arrays (int32 rowptr and columns, float64)."""
    _get().damn_cpu_spmv_csr(nrows, _p(rowptr), _p(cols), _p(vals), _p(x), _p(y), int(nthreads))


def arrays(rowptr, idx, vals, x, idx_dtype):
    """Contiguous copies with the types the kernels take."""
    return (np.ascontiguousarray(rowptr, dtype=np.int32), np.ascontiguousarray(idx, dtype=idx_dtype),
            np.ascontiguousarray(vals, dtype=np.float64), np.ascontiguousarray(x, dtype=np.float64))
