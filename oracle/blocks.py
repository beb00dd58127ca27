"""Block storage with diagonal addressing: DA-BSR (test infrastructure only).

The paper notes that diagonal addressing applies to other sparse formats
than CSR, naming BSR among them (Sec. 1).  BSR cuts an nrows x ncols matrix
into b x b blocks; it stores, for each block row, the block columns of its
nonzero blocks and each block's b*b values densely.  DA-BSR stores the block
column bc of a block in block row br as the offset bc - br, which fits int16
when the block bandwidth max |bc - br| is below 2^15 (the rule of Sec. 2
applied to blocks).

Layout (reading R23): block rows in order, blocks of a block row in
ascending block column, each block's values row-major; nrows and ncols are
multiples of b.
"""

from __future__ import annotations

import numpy as np

from .storage import NoFit, check_csr, entry_rows

INT16_LIMIT = 2**15


def bsr_from_csr(nrows, ncols, rowptr, colids, vals, b):
    """The BSR form of an int32 CSR matrix.

    A block is stored when at least one pattern entry (stored zeros
    included) falls into it; the other values of a stored block are zero;
    repeated entries add up.  Returns (browptr int32 [nrows/b + 1],
    bcols int64 [nnzb], bvals float64 [nnzb, b, b]).
    """
    check_csr(nrows, ncols, rowptr, colids)
    if b < 1 or nrows % b or ncols % b:
        raise ValueError("nrows and ncols must be multiples of the block size")
    nbr, nbc = nrows // b, ncols // b
    r = entry_rows(nrows, rowptr)
    c = np.asarray(colids, dtype=np.int64)
    v = np.asarray(vals, dtype=np.float64)
    key = (r // b) * nbc + (c // b)           # block id, ordered by (block row, block column)
    blocks, inv = np.unique(key, return_inverse=True)
    bvals = np.zeros((blocks.size, b, b))
    np.add.at(bvals, (inv, r % b, c % b), v)
    brow = blocks // nbc
    bcols = blocks % nbc
    browptr = np.zeros(nbr + 1, dtype=np.int64)
    np.add.at(browptr, brow + 1, 1)
    return np.cumsum(browptr).astype(np.int32), bcols, bvals


def block_bandwidth(nbrows, browptr, bcols):
    """max |bc - br| over stored blocks (0 without blocks)."""
    if len(bcols) == 0:
        return 0
    br = entry_rows(nbrows, browptr)
    return int(np.abs(np.asarray(bcols, dtype=np.int64) - br).max())


def da_block_offsets(nbrows, browptr, bcols):
    """bc - br as int16; NoFit when the block bandwidth is 2^15 or more."""
    w = block_bandwidth(nbrows, browptr, bcols)
    if w >= INT16_LIMIT:
        raise NoFit(w)
    return (np.asarray(bcols, dtype=np.int64) - entry_rows(nbrows, browptr)).astype(np.int16)


def spmv_bsr(nbrows, nbcols, b, browptr, bidx, bvals, x, alpha=1.0, beta=0.0, y0=None,
             da=True):
    """y <- alpha*A*x + beta*y0 for BSR (da=False: bidx holds block columns)
    or DA-BSR (da=True: bidx holds block offsets).  Row br*b + i sums
    bvals[k, i, j] * x[bc_k*b + j] over the blocks k of block row br and
    j = 0..b-1, blocks in storage order, j ascending, from zero; float64.
    beta == 0 does not read y0; alpha == 0 does not read A or x."""
    nrows = nbrows * b
    if alpha != 0:
        x = np.asarray(x, dtype=np.float64)
        br = entry_rows(nbrows, browptr)
        bc = np.asarray(bidx, dtype=np.int64) + (br if da else 0)
        V = np.asarray(bvals, dtype=np.float64).reshape(-1, b, b)
        acc = np.zeros(nrows)
        for i in range(b):
            # terms of scalar row br*b + i, in (block, j) storage order
            terms = V[:, i, :] * x[bc[:, None] * b + np.arange(b)[None, :]]
            rows = np.repeat(br * b + i, b)
            acc += np.bincount(rows, weights=terms.ravel(), minlength=nrows)
        y = alpha * acc
    else:
        y = np.zeros(nrows)
    if beta != 0:
        y = y + beta * np.asarray(y0, dtype=np.float64)
    return y


def bsr_dense(nbrows, nbcols, b, browptr, bidx, bvals, da=True):
    """Dense float64 matrix of a (DA-)BSR matrix, for brute-force checks."""
    D = np.zeros((nbrows * b, nbcols * b))
    br = entry_rows(nbrows, browptr)
    bc = np.asarray(bidx, dtype=np.int64) + (br if da else 0)
    V = np.asarray(bvals, dtype=np.float64).reshape(-1, b, b)
    for k in range(len(bc)):
        D[br[k] * b:(br[k] + 1) * b, bc[k] * b:(bc[k] + 1) * b] += V[k]
    return D


def bsr_bytes(nbrows, nbcols, nnzb, b, iindex=2, scalar=8):
    """Traffic of one product: Eq. 3 with one index per block and b*b scalars
    per block, plus x read once and y written (reading R9)."""
    return 4 * (nbrows + 1) + nnzb * (iindex + b * b * scalar) + scalar * b * (nbcols + nbrows)
