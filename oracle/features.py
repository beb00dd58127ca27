"""Sparsity features that drive the kernel-variant selector.

The paper picks, per matrix, the fastest of its implementations (Sec. 4.1);
it does not say how to predict that choice.  These 16 features describe what
the choice depends on: size, row-length distribution, bandwidth (Eq. 2) and
gather locality, and the number of right-hand sides.  Each is a plain
statistic of the CSR arrays, computed in float64:

 0 log2(nrows + 1)              8 1 if w >= 2^15 (reordering needed) else 0
 1 log2(nnz + 1)                9 nrhs
 2 mean row length              10 log2(mean |c - r| + 1)
 3 std of row lengths           11 fraction of entries with |c - r| <= 64
 4 log2(max row length + 1)     12 std / mean of row lengths (0 if empty)
 5 fraction of empty rows       13 fraction of rows with length >= 64
 6 log2(w + 1)                  14 log2(ncols + 1)
 7 w / max(ncols, 1)            15 fraction of adjacent entry pairs in a row
                                   whose columns differ by exactly 1
(w is the bandwidth; std is the population standard deviation.)
"""

from __future__ import annotations

import numpy as np

from .storage import entry_rows

NFEAT = 16


def features(nrows, ncols, rowptr, colids, nrhs):
    rowptr = np.asarray(rowptr, dtype=np.int64)
    colids = np.asarray(colids, dtype=np.int64)
    rl = np.diff(rowptr).astype(np.float64)
    nnz = int(rowptr[-1])
    n = max(nrows, 1)
    f = np.zeros(NFEAT)
    f[0] = np.log2(nrows + 1)
    f[1] = np.log2(nnz + 1)
    mean = nnz / n
    f[2] = mean
    f[3] = np.sqrt(max(float(np.mean(rl * rl)) - mean * mean, 0.0)) if nrows else 0.0
    f[4] = np.log2((rl.max() if nrows else 0.0) + 1)
    f[5] = float(np.count_nonzero(rl == 0)) / n
    d = np.abs(colids - entry_rows(nrows, rowptr)) if nnz else np.zeros(0)
    w = int(d.max()) if nnz else 0
    f[6] = np.log2(w + 1)
    f[7] = w / max(ncols, 1)
    f[8] = 1.0 if w >= 2**15 else 0.0
    f[9] = float(nrhs)
    f[10] = np.log2(float(d.mean()) + 1) if nnz else 0.0
    f[11] = float(np.count_nonzero(d <= 64)) / nnz if nnz else 0.0
    f[12] = f[3] / mean if mean > 0 else 0.0
    f[13] = float(np.count_nonzero(rl >= 64)) / n
    f[14] = np.log2(ncols + 1)
    if nnz > 1:
        same_row = np.diff(entry_rows(nrows, rowptr)) == 0
        pairs = int(np.count_nonzero(same_row))
        unit = int(np.count_nonzero(same_row & (np.diff(colids) == 1)))
        f[15] = unit / pairs if pairs else 0.0
    return f
