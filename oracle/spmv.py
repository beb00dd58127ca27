"""Sparse matrix-vector products y <- alpha*A*x + beta*y (Sec. 4).

Plain float64 definitions.  For each row r,
    y_r = alpha * sum_{i in row r} values[i] * x[c_i] + beta * y0_r
where c_i is colids[i] for CSR and r + colids[i] for DA-CSR (Sec. 2).
The row sums add the products in storage order, starting from zero.

Conventions the paper leaves open (its listing always reads y):
* beta == 0 does not read y0, so NaN/Inf in y0 do not propagate (BLAS);
* alpha == 0 does not read A or x: y = beta*y0.
For float32 inputs the arithmetic is still float64 on the given values.
"""

from __future__ import annotations

import numpy as np

from .storage import entry_rows


def _rowsum(nrows, rowptr, terms):
    # bincount adds weights[i] into bin rows[i] for i = 0, 1, ... in turn,
    # i.e. each row sum runs over its entries in storage order from zero
    rows = entry_rows(nrows, rowptr)
    return np.bincount(rows, weights=terms, minlength=nrows).astype(np.float64)


def _axpby(acc, alpha, beta, y0):
    y = alpha * acc if alpha != 0 else np.zeros_like(acc)
    if beta != 0:
        y = y + beta * np.asarray(y0, dtype=np.float64)
    return y


def spmv_csr(nrows, ncols, rowptr, colids, vals, x, alpha=1.0, beta=0.0, y0=None):
    """CSR SpMV with absolute column indices."""
    if alpha != 0:
        x = np.asarray(x, dtype=np.float64)
        terms = np.asarray(vals, dtype=np.float64) * x[np.asarray(colids, dtype=np.int64)]
        acc = _rowsum(nrows, rowptr, terms)
    else:
        acc = np.zeros(nrows)
    return _axpby(acc, alpha, beta, y0)


def spmv_da(nrows, ncols, rowptr, off, vals, x, alpha=1.0, beta=0.0, y0=None):
    """DA-CSR SpMV: entry i of row r multiplies x[r + off[i]]."""
    if alpha != 0:
        x = np.asarray(x, dtype=np.float64)
        cols = entry_rows(nrows, rowptr) + np.asarray(off, dtype=np.int64)
        terms = np.asarray(vals, dtype=np.float64) * x[cols]
        acc = _rowsum(nrows, rowptr, terms)
    else:
        acc = np.zeros(nrows)
    return _axpby(acc, alpha, beta, y0)


def spmm_da(nrows, ncols, rowptr, off, vals, X, alpha=1.0, beta=0.0, Y0=None):
    """DA-CSR times a block of nrhs vectors; X is ncols x nrhs, Y nrows x nrhs
    (row-major, right-hand sides interleaved).  Column j of Y is spmv_da of
    column j of X."""
    X = np.asarray(X)
    nrhs = X.shape[1]
    Y = np.empty((nrows, nrhs))
    for j in range(nrhs):
        Y[:, j] = spmv_da(nrows, ncols, rowptr, off, vals, X[:, j], alpha, beta,
                          None if Y0 is None else np.asarray(Y0)[:, j])
    return Y


def spmm_csr(nrows, ncols, rowptr, colids, vals, X, alpha=1.0, beta=0.0, Y0=None):
    """CSR counterpart of spmm_da."""
    X = np.asarray(X)
    nrhs = X.shape[1]
    Y = np.empty((nrows, nrhs))
    for j in range(nrhs):
        Y[:, j] = spmv_csr(nrows, ncols, rowptr, colids, vals, X[:, j], alpha, beta,
                           None if Y0 is None else np.asarray(Y0)[:, j])
    return Y


def abs_products(nrows, rowptr, cols, vals, x):
    """sum_{i in row r} |values[i] * x[c_i]| per row (absolute column indices),
    the scale in the rounding-error bound of a row sum."""
    x = np.asarray(x, dtype=np.float64)
    terms = np.abs(np.asarray(vals, dtype=np.float64) * x[np.asarray(cols, dtype=np.int64)])
    return _rowsum(nrows, rowptr, terms)


def dense(nrows, ncols, rowptr, cols, vals):
    """Dense float64 matrix (repeated entries add up); for brute-force checks."""
    D = np.zeros((nrows, ncols))
    np.add.at(D, (entry_rows(nrows, rowptr), np.asarray(cols, dtype=np.int64)),
              np.asarray(vals, dtype=np.float64))
    return D
