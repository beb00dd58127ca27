"""Traffic and work model (Eq. 1, Eq. 3, the work count of Sec. 4, Fig. 3).

Eq. 3: matrix traffic = (nrows + 1) * |oindex| + nnz * (|iindex| + |scalar|).
Sec. 4 adds x and y to the traffic.  Reading used for their multiplicity:
x is read once (ncols entries per right-hand side; reuse served by caches),
y is written once and additionally read when beta != 0.
Sec. 4: work W = 2*nnz + 2*nrows flops per right-hand side.
Eq. 1: for memory-bound kernels P1/P2 = T2/T1, so the predicted speedup of
a format with traffic T_new over one with T_old is T_old / T_new.
"""

from __future__ import annotations

from fractions import Fraction


def matrix_bytes(nrows, nnz, oindex=4, iindex=4, scalar=8):
    """Eq. 3."""
    return (nrows + 1) * oindex + nnz * (iindex + scalar)


def spmv_bytes(nrows, ncols, nnz, iindex, scalar, nrhs=1, beta_nonzero=False, oindex=4):
    """Matrix traffic plus x (read once) and y (written, read if beta != 0)."""
    return (
        matrix_bytes(nrows, nnz, oindex, iindex, scalar)
        + scalar * nrhs * ncols
        + scalar * nrhs * nrows * (2 if beta_nonzero else 1)
    )


def work_flops(nrows, nnz, nrhs=1):
    """Sec. 4: W = 2 nnz + 2 nrows per right-hand side."""
    return nrhs * (2 * nnz + 2 * nrows)


def predicted_speedup(bytes_old, bytes_new):
    """Eq. 1."""
    return bytes_old / bytes_new


def uplift_fraction(t_old, t_new, bytes_old, bytes_new):
    """Measured uplift relative to the model-predicted one:
    (t_old/t_new - 1) / (T_old/T_new - 1)  (the 87.5% figure of the
    abstract is 0.175 / 0.20 in this form)."""
    return (t_old / t_new - 1.0) / (bytes_old / bytes_new - 1.0)


def per_nnz_ratio(iindex_a, scalar_a, iindex_b, scalar_b):
    """Approximate matrix-traffic ratio of Fig. 3 (row pointers ignored, as
    Sec. 2 suggests for matrices with more than a few entries per row):
    (|iindex_b| + |scalar_b|) / (|iindex_a| + |scalar_a|), as an exact
    fraction.  Dense storage is iindex = 0."""
    return Fraction(iindex_b + scalar_b, iindex_a + scalar_a)
