"""Seeded sparse matrices and vectors (int32 CSR, float64 values).

Every generator takes an explicit seed and is deterministic for it.  Rows
are in natural order and the column indices of a row are ascending unless a
generator says otherwise.  Nothing here computes a bandwidth, an offset or
a product: those belong to the code under test and to the oracle.
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass
class CSR:
    """A sparse matrix in CSR form: rowptr[nrows+1], colids[nnz], vals[nnz]."""

    nrows: int
    ncols: int
    rowptr: np.ndarray  # int32
    colids: np.ndarray  # int32
    vals: np.ndarray  # float64
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def rowlen(self) -> np.ndarray:
        return np.diff(self.rowptr.astype(np.int64))


def _finish(nrows, ncols, rowlen, colids, vals, name) -> CSR:
    rowptr = np.zeros(nrows + 1, dtype=np.int64)
    np.cumsum(rowlen, out=rowptr[1:])
    if rowptr[-1] >= 2**31:
        raise ValueError("matrix does not fit int32 CSR")
    return CSR(
        nrows,
        ncols,
        rowptr.astype(np.int32),
        np.ascontiguousarray(colids, dtype=np.int32),
        np.ascontiguousarray(vals, dtype=np.float64),
        name,
    )


def _grid_stencil(dims, offsets, values_fn, name) -> CSR:
    """Build a stencil matrix on an nx*ny*nz grid, x fastest.

    offsets: list of (dx, dy, dz).  values_fn(valid, k_diag) returns an
    (n, K) float64 array of entry values (ignored where not valid).
    """
    nx, ny, nz = dims
    n = nx * ny * nz
    # sort the stencil by linear column offset, so each row comes out with
    # ascending column indices
    lin = [dx + nx * (dy + ny * dz) for (dx, dy, dz) in offsets]
    order = sorted(range(len(offsets)), key=lambda k: lin[k])
    offsets = [offsets[k] for k in order]
    K = len(offsets)
    idx = np.arange(n, dtype=np.int64)
    gx = idx % nx
    gy = (idx // nx) % ny
    gz = idx // (nx * ny)
    valid = np.empty((n, K), dtype=bool)
    cols = np.empty((n, K), dtype=np.int32)
    k_diag = -1
    for k, (dx, dy, dz) in enumerate(offsets):
        if (dx, dy, dz) == (0, 0, 0):
            k_diag = k
        valid[:, k] = (
            (gx + dx >= 0) & (gx + dx < nx)
            & (gy + dy >= 0) & (gy + dy < ny)
            & (gz + dz >= 0) & (gz + dz < nz)
        )
        cols[:, k] = (idx + (dx + nx * (dy + ny * dz))).astype(np.int32, copy=False)
    del gx, gy, gz, idx
    vals = values_fn(valid, k_diag)
    rowlen = valid.sum(axis=1, dtype=np.int64)
    colids = cols[valid]
    del cols
    v = vals[valid]
    return _finish(n, n, rowlen, colids, v, name)


def laplace_2d_5pt(N: int) -> CSR:
    """2D 5-point Laplacian on an N x N grid: 4 on the diagonal, -1 off."""
    offsets = [(0, -1, 0), (-1, 0, 0), (0, 0, 0), (1, 0, 0), (0, 1, 0)]

    def values(valid, kd):
        v = np.full(valid.shape, -1.0)
        v[:, kd] = 4.0
        return v

    return _grid_stencil((N, N, 1), offsets, values, f"laplace2d_5pt_{N}x{N}")


def poisson_3d_7pt(nx: int, ny: int, nz: int) -> CSR:
    """3D 7-point Poisson operator on an nx*ny*nz grid: 6 on the diagonal, -1 off."""
    offsets = [(0, 0, -1), (0, -1, 0), (-1, 0, 0), (0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1)]

    def values(valid, kd):
        v = np.full(valid.shape, -1.0)
        v[:, kd] = 6.0
        return v

    return _grid_stencil((nx, ny, nz), offsets, values, f"poisson3d_7pt_{nx}x{ny}x{nz}")


def stencil_3d_27pt(N: int, seed: int) -> CSR:
    """3D 27-point stencil on an N^3 grid.

    Off-diagonal values uniform on [-1, 1]; the diagonal is 1 plus the sum of
    the absolute off-diagonal values of its row (strict diagonal dominance).
    """
    A = stencil_3d_27pt_box(N, N, N, seed)
    A.name = f"stencil3d_27pt_{N}^3"
    return A


def stencil_3d_27pt_box(nx: int, ny: int, nz: int, seed: int) -> CSR:
    """The 27-point stencil of stencil_3d_27pt on an nx*ny*nz box (x
    fastest); its bandwidth is 1 + nx + nx*ny."""
    offsets = [(dx, dy, dz) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]

    def values(valid, kd):
        rng = np.random.default_rng(seed)
        v = rng.uniform(-1.0, 1.0, size=valid.shape)
        v[~valid] = 0.0
        v[:, kd] = 0.0
        v[:, kd] = 1.0 + np.abs(v).sum(axis=1)
        return v

    return _grid_stencil((nx, ny, nz), offsets, values, f"stencil3d_27pt_{nx}x{ny}x{nz}")


def block_stencil_27pt(N: int, b: int, seed: int) -> CSR:
    """A block matrix of the kind finite elements give with b unknowns per
    node: the 27-point stencil pattern on an N^3 grid of nodes, each node
    pair coupled by a dense b x b block (so every block is stored).

    Values uniform on [-1, 1]; each diagonal entry is 1 plus the sum of the
    absolute values of its row.  Scalar rows come in node order, the b
    unknowns of a node adjacent; within a row, entries by block then column.
    """
    P = stencil_3d_27pt(N, seed)
    nbr, nnzb = P.nrows, P.nnz
    rp = P.rowptr.astype(np.int64)
    bc = P.colids.astype(np.int64)
    rl = np.diff(rp)
    br = np.repeat(np.arange(nbr, dtype=np.int64), rl)
    kk = np.arange(nnzb, dtype=np.int64) - rp[br]        # block position in its block row
    i = np.arange(b, dtype=np.int64)[None, :, None]
    j = np.arange(b, dtype=np.int64)[None, None, :]
    # position of entry (k, i, j): row br*b + i starts at rp[br]*b*b + i*rl[br]*b
    pos = (rp[br] * b * b)[:, None, None] + i * (rl[br] * b)[:, None, None] + kk[:, None, None] * b + j
    rows = (br * b)[:, None, None] + i + 0 * j
    cols = (bc * b)[:, None, None] + j + 0 * i
    rng = np.random.default_rng(seed + 7919 * b)
    vals_kij = rng.uniform(-1.0, 1.0, size=(nnzb, b, b))
    nnz = nnzb * b * b
    colids = np.empty(nnz, dtype=np.int64)
    vals = np.empty(nnz)
    rowof = np.empty(nnz, dtype=np.int64)
    colids[pos.ravel()] = cols.ravel()
    vals[pos.ravel()] = vals_kij.ravel()
    rowof[pos.ravel()] = rows.ravel()
    diag = rowof == colids
    vals[diag] = 0.0
    rowsum = np.bincount(rowof, weights=np.abs(vals), minlength=nbr * b)
    vals[diag] = 1.0 + rowsum[rowof[diag]]
    rowlen = np.repeat(rl * b, b)
    return _finish(nbr * b, nbr * b, rowlen, colids.astype(np.int32), vals,
                   f"block{b}_stencil27_{N}^3")


def random_banded(
    n: int,
    seed: int,
    half_band: int = 20000,
    mean_len: float = 12.0,
    sigma: float = 0.8,
    max_len: int = 200,
    ncols: int | None = None,
) -> CSR:
    """Random banded matrix, n x ncols (ncols = n by default).

    Row lengths are lognormal with the given mean and shape sigma, rounded
    and clipped to [1, max_len] (and to the row's window).  The columns of a
    row are distinct, uniform over
    [max(0, r-half_band), min(ncols-1, r+half_band)], sorted ascending (a row
    whose window is empty, in a tall matrix, stays empty); values are
    standard normal.
    """
    m = n if ncols is None else ncols
    rng = np.random.default_rng(seed)
    mu = math.log(mean_len) - 0.5 * sigma * sigma
    rowlen = np.clip(np.rint(rng.lognormal(mu, sigma, n)), 1, max_len).astype(np.int64)
    r = np.arange(n, dtype=np.int64)
    lo = np.maximum(r - half_band, 0)
    window = np.maximum(np.minimum(r + half_band, m - 1) - lo + 1, 0)
    rowlen = np.minimum(rowlen, window)
    del r
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(rowlen, out=rowptr[1:])
    nnz = int(rowptr[-1])
    rows = np.repeat(np.arange(n, dtype=np.int64), rowlen)
    cols = lo[rows] + rng.integers(0, window[rows], dtype=np.int64)
    key = rows * m + cols
    key.sort()
    cols = key - rows * m
    del key
    # redraw repeated columns until every row's columns are distinct
    while True:
        dup = np.flatnonzero(cols[1:] == cols[:-1]) + 1
        dup = dup[rows[dup] == rows[dup - 1]]
        if dup.size == 0:
            break
        dr = rows[dup]
        cols[dup] = lo[dr] + rng.integers(0, window[dr], dtype=np.int64)
        for rr in np.unique(dr):
            s, e = rowptr[rr], rowptr[rr + 1]
            cols[s:e].sort()
    del rows
    vals = rng.standard_normal(nnz)
    name = f"banded_n{n}_hb{half_band}" if m == n else f"banded_{n}x{m}_hb{half_band}"
    return _finish(n, m, rowlen, cols.astype(np.int32), vals, name)


def scramble_symmetric(A: CSR, seed: int) -> CSR:
    """Return Q A Q^T for a seeded random permutation Q (square matrices).

    New row i is old row q[i]; an old column c becomes the position of c in q.
    Each new row is sorted by new column; ties keep their old order.
    """
    if A.nrows != A.ncols:
        raise ValueError("symmetric scrambling needs a square matrix")
    n = A.nrows
    rng = np.random.default_rng(seed)
    q = rng.permutation(n).astype(np.int64)
    pos = np.empty(n, dtype=np.int64)
    pos[q] = np.arange(n, dtype=np.int64)
    rl = A.rowlen()
    rows_old = np.repeat(np.arange(n, dtype=np.int64), rl)
    key = pos[rows_old] * n + pos[A.colids.astype(np.int64)]
    del rows_old
    order = np.argsort(key, kind="stable")
    newcols = (key[order] % n).astype(np.int32)
    del key
    vals = A.vals[order]
    del order
    return _finish(n, n, rl[q], newcols, vals, A.name + "_scrambled")


def random_csr(
    nrows: int,
    ncols: int,
    seed: int,
    mean_len: float = 4.0,
    band: int | None = None,
    empty_frac: float = 0.1,
    dup_frac: float = 0.0,
    zero_frac: float = 0.0,
    shuffle_rows: bool = False,
    int_values: bool = False,
) -> CSR:
    """Small irregular CSR for edge-case tests.

    Poisson row lengths (mean_len) with a fraction of forced-empty rows;
    columns uniform over [0, ncols) or, if band is given, within `band` of the
    row (clipped to the matrix).  Optional repeated columns within a row,
    explicit zero values and unsorted rows.  int_values draws small integers
    (exact products and sums in float64).
    """
    rng = np.random.default_rng(seed)
    rowlen = rng.poisson(mean_len, nrows).astype(np.int64)
    rowlen[rng.random(nrows) < empty_frac] = 0
    if ncols == 0:
        rowlen[:] = 0
    nnz = int(rowlen.sum())
    rows = np.repeat(np.arange(nrows, dtype=np.int64), rowlen)
    if band is None:
        cols = rng.integers(0, max(ncols, 1), nnz, dtype=np.int64)
    else:
        lo = np.clip(rows - band, 0, max(ncols - 1, 0))
        hi = np.clip(rows + band, 0, max(ncols - 1, 0))
        cols = lo + (rng.random(nnz) * (hi - lo + 1)).astype(np.int64)
        cols = np.minimum(cols, hi)
    if dup_frac > 0 and nnz > 1:
        # copy the previous entry's column within the same row
        pick = np.flatnonzero(rng.random(nnz) < dup_frac)
        pick = pick[pick > 0]
        pick = pick[rows[pick] == rows[pick - 1]]
        cols[pick] = cols[pick - 1]
    key = rows * max(ncols, 1) + cols
    order = np.argsort(key, kind="stable")
    cols = cols[order]
    if shuffle_rows:
        perm = np.lexsort((rng.random(nnz), rows))
        cols = cols[perm]
    if int_values:
        vals = rng.integers(-8, 9, nnz).astype(np.float64)
    else:
        vals = rng.uniform(-1.0, 1.0, nnz)
    if zero_frac > 0:
        vals[rng.random(nnz) < zero_frac] = 0.0
    return _finish(nrows, ncols, rowlen, cols.astype(np.int32), vals, f"random_{nrows}x{ncols}_s{seed}")


def uniform_vector(n: int, seed: int, nrhs: int | None = None, dtype=np.float64) -> np.ndarray:
    """Vector (or n x nrhs row-major block) uniform on [-1, 1]."""
    rng = np.random.default_rng(seed)
    shape = (n,) if nrhs is None else (n, nrhs)
    return rng.uniform(-1.0, 1.0, size=shape).astype(dtype)


BATCH_KINDS = ("laplace2d", "poisson3d", "stencil27", "banded")


def batch_member(seed: int, index: int, n_lo: float = 1e3, n_hi: float = 2e5):
    """Descriptor of one matrix of the batched / selector family.

    n log-uniform on [n_lo, n_hi]; kind uniform over BATCH_KINDS; nrhs uniform
    on 1..8; banded half-bandwidth log-uniform on [8, min(30000, n-1)].
    """
    rng = np.random.default_rng([seed, index])
    n = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
    kind = BATCH_KINDS[int(rng.integers(0, len(BATCH_KINDS)))]
    nrhs = int(rng.integers(1, 9))
    hb_hi = min(30000, n - 1)
    half_band = int(round(math.exp(rng.uniform(math.log(8), math.log(hb_hi)))))
    mseed = int(rng.integers(0, 2**31 - 1))
    return {"kind": kind, "n": n, "nrhs": nrhs, "half_band": half_band, "seed": mseed}


def batch_matrix(desc) -> CSR:
    kind, n = desc["kind"], desc["n"]
    if kind == "laplace2d":
        return laplace_2d_5pt(max(3, int(round(math.sqrt(n)))))
    if kind == "poisson3d":
        N = max(3, int(round(n ** (1.0 / 3.0))))
        return poisson_3d_7pt(N, N, N)
    if kind == "stencil27":
        return stencil_3d_27pt(max(3, int(round(n ** (1.0 / 3.0)))), desc["seed"])
    return random_banded(n, desc["seed"], half_band=desc["half_band"])


def batch_family(count: int, seed: int):
    """List of `count` (descriptor, CSR) pairs from the batched family."""
    out = []
    for i in range(count):
        d = batch_member(seed, i)
        out.append((d, batch_matrix(d)))
    return out
