"""Coordinate storage with diagonal addressing: DA-COO (test infrastructure
only).

COO stores every entry as (row, column, value).  The paper notes that
diagonal addressing applies to one of COO's index vectors (Sec. 1): DA-COO
keeps the row r_i and replaces the column by the offset c_i - r_i, which
fits int16 when the bandwidth w of Eq. 2 is below 2^15.

Reading R24: entries in row order (the order CSR gives; within a row, any
order), so a product can sum each row's entries as one contiguous run.
"""

from __future__ import annotations

import numpy as np

from .storage import NoFit, check_csr, entry_rows

INT16_LIMIT = 2**15


def coo_from_csr(nrows, ncols, rowptr, colids, da=True):
    """(rows int32, idx) of an int32 CSR matrix, entry order unchanged: idx is
    the int16 offset c - r (da=True; NoFit when w >= 2^15) or the int32
    column."""
    check_csr(nrows, ncols, rowptr, colids)
    r = entry_rows(nrows, rowptr)
    c = np.asarray(colids, dtype=np.int64)
    if not da:
        return r.astype(np.int32), c.astype(np.int32)
    d = c - r
    w = int(np.abs(d).max()) if d.size else 0
    if w >= INT16_LIMIT:
        raise NoFit(w)
    return r.astype(np.int32), d.astype(np.int16)


def spmv_coo(nrows, ncols, rows, idx, vals, x, alpha=1.0, beta=0.0, y0=None, da=True):
    """y <- alpha*A*x + beta*y0: entry i adds vals[i] * x[c_i] to row
    rows[i], c_i = rows[i] + idx[i] (da) or idx[i]; each row sums its entries
    in storage order from zero, in float64.  beta == 0 does not read y0;
    alpha == 0 does not read A or x.  Rows without entries get beta*y0."""
    r = np.asarray(rows, dtype=np.int64)
    if alpha != 0:
        x = np.asarray(x, dtype=np.float64)
        c = np.asarray(idx, dtype=np.int64) + (r if da else 0)
        terms = np.asarray(vals, dtype=np.float64) * x[c]
        y = alpha * np.bincount(r, weights=terms, minlength=nrows).astype(np.float64)
    else:
        y = np.zeros(nrows)
    if beta != 0:
        y = y + beta * np.asarray(y0, dtype=np.float64)
    return y


def coo_bytes(nrows, ncols, nnz, iindex=2, scalar=8, beta_nonzero=False):
    """Traffic of one product: one row index (4 bytes), one column index and
    one scalar per entry, plus x read once and y written (read too when
    beta != 0), as reading R9 counts them."""
    return nnz * (4 + iindex + scalar) + scalar * ncols + scalar * nrows * (2 if beta_nonzero else 1)
