"""CSR / DA-CSR storage (paper Sec. 2, Listing 1, Eq. 2, Example 1).

A matrix A of nrows x ncols is held as rowptr[nrows+1], colids[nnz],
values[nnz].  In plain CSR colids[i] is the column c_i of entry i; in DA-CSR
it is c_i - r_i, the signed distance from the diagonal (Sec. 2).  The
bandwidth w of Eq. 2 bounds every such distance, so a matrix whose w fits a
16-bit signed integer can store its column indices in int16.
"""

from __future__ import annotations

import numpy as np

# Sec. 2 / Sec. 3: 16-bit indices are used when w < 2^15 = 32768.
INT16_BANDWIDTH_LIMIT = 2**15


class BadCSR(ValueError):
    """The three arrays do not describe a valid CSR matrix."""


class NoFit(Exception):
    """An index (the bandwidth, or a column) or a value does not fit the
    storage type asked for (for int16 offsets: even after reordering)."""

    def __init__(self, w, bits=16, what="bandwidth"):
        super().__init__(f"{what} {w} does not fit int{bits} (needs < {2 ** (bits - 1)})")
        self.w = w


def check_csr(nrows, ncols, rowptr, colids):
    """Validate CSR structure.

    rowptr has nrows+1 entries, starts at 0, never decreases and ends at nnz
    (the footnote of Sec. 2 sets rowptr[nrows] = nnz); every column lies in
    [0, ncols).  Empty rows, repeated columns and unsorted rows are allowed.
    """
    rowptr = np.asarray(rowptr)
    colids = np.asarray(colids)
    if nrows < 0 or ncols < 0:
        raise BadCSR("negative dimension")
    if rowptr.shape != (nrows + 1,):
        raise BadCSR("rowptr must have nrows+1 entries")
    if rowptr[0] != 0:
        raise BadCSR("rowptr[0] must be 0")
    if nrows > 0 and np.any(np.diff(rowptr.astype(np.int64)) < 0):
        raise BadCSR("rowptr must be non-decreasing")
    if int(rowptr[-1]) != colids.shape[0]:
        raise BadCSR("rowptr[nrows] must equal nnz")
    if colids.size and (colids.min() < 0 or colids.max() >= ncols):
        raise BadCSR("column index out of range")


def entry_rows(nrows, rowptr):
    """Row index r_i of every stored entry i (int64)."""
    rl = np.diff(np.asarray(rowptr, dtype=np.int64))
    return np.repeat(np.arange(nrows, dtype=np.int64), rl)


def fit(nrows, ncols, rowptr, colids):
    """Bandwidth of Eq. 2 over all stored (pattern) entries.

    Returns (w, lo, hi, fits): w = max |c - r|, lo = max(r - c) and
    hi = max(c - r) (each at least 0; all 0 for an empty matrix), and
    fits = (w < 2^15).  Explicitly stored zeros count, as the footnote of
    Example 2 defines nnz over pattern entries.
    """
    check_csr(nrows, ncols, rowptr, colids)
    if len(colids) == 0:
        return 0, 0, 0, True
    d = np.asarray(colids, dtype=np.int64) - entry_rows(nrows, rowptr)
    hi = max(int(d.max()), 0)
    lo = max(int(-d.min()), 0)
    w = max(lo, hi)
    return w, lo, hi, w < INT16_BANDWIDTH_LIMIT


def da_offsets(nrows, rowptr, colids):
    """The DA transform: colids[i] <- c_i - r_i, as int16 (Sec. 2).

    The caller must have checked that the bandwidth fits.
    """
    d = np.asarray(colids, dtype=np.int64) - entry_rows(nrows, rowptr)
    assert d.size == 0 or (d.min() > -INT16_BANDWIDTH_LIMIT and d.max() < INT16_BANDWIDTH_LIMIT)
    return d.astype(np.int16)


def da_columns(nrows, rowptr, offsets):
    """Inverse of the DA transform: c_i = r_i + offset_i (int64)."""
    return entry_rows(nrows, rowptr) + np.asarray(offsets, dtype=np.int64)


def permute_symmetric(n, rowptr, colids, vals, perm):
    """P A P^T for a permutation given new -> old.

    New row i is old row perm[i]; a column c is relabelled inv[c] where
    inv[perm[i]] = i.  Within each new row the entries are ordered by new
    column, and entries with equal new column keep their old relative order.
    """
    perm = np.asarray(perm, dtype=np.int64)
    inv = np.empty(n, dtype=np.int64)
    inv[perm] = np.arange(n, dtype=np.int64)
    rowptr = np.asarray(rowptr, dtype=np.int64)
    rl = np.diff(rowptr)
    new_rl = rl[perm]
    new_rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(new_rl, out=new_rowptr[1:])
    # gather the old rows in new order (entries of a row stay in old order)
    nnz = int(new_rowptr[-1])
    src = np.repeat(rowptr[perm] - new_rowptr[:-1], new_rl) + np.arange(nnz, dtype=np.int64)
    new_rows = np.repeat(np.arange(n, dtype=np.int64), new_rl)
    new_cols = inv[np.asarray(colids, dtype=np.int64)[src]]
    order = np.lexsort((new_cols, new_rows))  # lexsort is stable
    src = src[order]
    return (
        new_rowptr.astype(np.int32),
        new_cols[order].astype(np.int32),
        np.asarray(vals)[src],
    )


def encode(nrows, ncols, rowptr, colids, vals, allow_rcm=True):
    """Turn int32 CSR into DA-CSR with int16 offsets.

    If the natural order fits (w < 2^15) the entries keep their order and
    values, and only the column indices are rewritten (Sec. 2).  Otherwise,
    when reordering is allowed and the matrix is square, the reverse
    Cuthill-McKee permutation is applied first (Sec. 2, Example 2; Sec. 3),
    refined by midpoint sweeps (rcm.midpoint_refine) when the RCM order alone
    does not fit, and the fit is checked again.  Raises NoFit when no fitting
    form is found.

    Returns a dict with rowptr, off (int16), vals, perm (new -> old; the
    identity if not permuted), permuted and w (bandwidth of the result).
    """
    from .rcm import midpoint_refine, rcm

    w, lo, hi, fits = fit(nrows, ncols, rowptr, colids)
    if fits:
        return {
            "rowptr": np.asarray(rowptr, dtype=np.int32).copy(),
            "off": da_offsets(nrows, rowptr, colids),
            "vals": np.asarray(vals).copy(),
            "perm": np.arange(nrows, dtype=np.int32),
            "permuted": False,
            "w": w,
        }
    if not allow_rcm or nrows != ncols:
        raise NoFit(w)
    perm = rcm(nrows, rowptr, colids)
    perm, w_perm, _ = midpoint_refine(nrows, rowptr, colids, perm)
    if w_perm >= INT16_BANDWIDTH_LIMIT:
        raise NoFit(w_perm)
    rp, cols, v = permute_symmetric(nrows, rowptr, colids, vals, perm)
    w2, _, _, fits2 = fit(nrows, ncols, rp, cols)
    if not fits2:
        raise NoFit(w2)
    return {
        "rowptr": rp,
        "off": da_offsets(nrows, rp, cols),
        "vals": v,
        "perm": perm.astype(np.int32),
        "permuted": True,
        "w": w2,
    }


# ---------------------------------------------------------------------------
# The storage grid of Fig. 3: column indices of 32, 16 or 8 bits and scalars
# of 64, 32 or 16 bits.  DA formats hold offsets c_i - r_i (Sec. 2), CSR
# formats absolute columns c_i.
# ---------------------------------------------------------------------------

# format name -> (index bytes, holds DA offsets)
INDEX_FORMATS = {"da16": (2, True), "csr32": (4, False), "da8": (1, True), "csr16": (2, False)}
_INT_TYPES = {1: np.int8, 2: np.int16, 4: np.int32}
VALUE_TYPES = {"f64": np.float64, "f32": np.float32, "f16": np.float16}


def index_limit(nbytes):
    """A signed index of nbytes holds values of magnitude below 2^(8 nbytes - 1):
    the rule w < 2^15 of Sec. 2 applied to any width, so the most negative
    value of the type is never emitted."""
    return 2 ** (8 * nbytes - 1)


def encode_index(fmt, nrows, ncols, rowptr, colids):
    """Column indices of int32 CSR in format fmt, entry order unchanged.

    DA formats store c_i - r_i and need w below index_limit (Eq. 2); CSR
    formats store c_i and need every stored column below it (a direct
    representation with narrower column indices, as the remark closing
    Sec. 4 counts them).  Raises NoFit otherwise.
    """
    nbytes, is_da = INDEX_FORMATS[fmt]
    check_csr(nrows, ncols, rowptr, colids)
    lim = index_limit(nbytes)
    c = np.asarray(colids, dtype=np.int64)
    if is_da:
        d = c - entry_rows(nrows, rowptr)
        w = int(np.abs(d).max()) if d.size else 0
        if w >= lim:
            raise NoFit(w, 8 * nbytes)
        return d.astype(_INT_TYPES[nbytes])
    m = int(c.max()) if c.size else 0
    if m >= lim:
        raise NoFit(m, 8 * nbytes, "column")
    return c.astype(_INT_TYPES[nbytes])


def store_values(vals, vtype):
    """Values as a matrix of scalar type vtype holds them: IEEE 754 binary64
    to binary32 / binary16 with round to nearest, ties to even, in one step
    from the float64 value (never through float32 first).  A finite value
    that rounds to infinity raises NoFit."""
    v = np.asarray(vals, dtype=np.float64)
    with np.errstate(over="ignore"):
        out = v.astype(VALUE_TYPES[vtype])
    bad = np.isfinite(v) & ~np.isfinite(out)
    if np.any(bad):
        raise NoFit(float(v[bad][0]), 8 * out.itemsize, "value")
    return out
