"""The oracle's DA-BSR (Sec. 1: diagonal addressing applied to BSR).

Pins: Example 1 (Sec. 2) cut into 2 x 2 blocks by hand; Kronecker products
A (x) K whose block structure is A's pattern (block bandwidth = w(A), block
offsets = A's DA offsets); block size 1 reducing to CSR; dense brute force;
integer closed forms; the traffic model at b = 1 against Eq. 3.
"""

import numpy as np
import pytest

from conftest import golden
from oracle import blocks as B
from oracle import spmv as S
from oracle import storage as O
from oracle import traffic as T
from workloads import laplace_2d_5pt, random_csr


def test_example1_blocks_by_hand():
    g = golden("example1.json")
    e = [1.0, 2.0, 3.0, 4.0, 5.0]
    rp, cols, vals = B.bsr_from_csr(4, 4, g["rowptr"], g["csr_colids"], e, 2)
    assert rp.tolist() == [0, 2, 4]
    assert cols.tolist() == [0, 1, 0, 1]
    assert B.da_block_offsets(2, rp, cols).tolist() == [0, 1, -1, 0]
    # entry (0,0) -> block (0,0)[0][0]; (1,2) -> block (0,1)[1][0];
    # (2,1) -> block (1,0)[0][1]; (2,3) -> (1,1)[0][1]; (3,3) -> (1,1)[1][1]
    want = np.array([[[1, 0], [0, 0]], [[0, 0], [2, 0]], [[0, 3], [0, 0]], [[0, 4], [0, 5]]],
                    dtype=float)
    assert np.array_equal(vals, want)
    assert B.block_bandwidth(2, rp, cols) == 1


def _kron(A, K):
    """A (x) K as int32 CSR (K dense b x b, every entry stored)."""
    b = K.shape[0]
    D = np.kron(S.dense(A.nrows, A.ncols, A.rowptr, A.colids, A.vals), np.ones((b, b)))
    pat = D != 0
    D = np.kron(S.dense(A.nrows, A.ncols, A.rowptr, A.colids, A.vals), K)
    r, c = np.nonzero(pat)
    rowptr = np.concatenate([[0], np.cumsum(np.bincount(r, minlength=D.shape[0]))]).astype(np.int32)
    return D.shape[0], D.shape[1], rowptr, c.astype(np.int32), D[r, c]


@pytest.mark.parametrize("b", [2, 3, 4])
def test_kronecker_block_structure(b):
    A = laplace_2d_5pt(7)
    K = np.arange(1, b * b + 1, dtype=float).reshape(b, b)
    n, m, rp, c, v = _kron(A, K)
    brp, bcols, bvals = B.bsr_from_csr(n, m, rp, c, v, b)
    assert np.array_equal(brp, A.rowptr)
    assert np.array_equal(bcols, A.colids)
    assert B.block_bandwidth(A.nrows, brp, bcols) == 7  # w of the 2D 5-point Laplacian on 7x7
    assert np.array_equal(B.da_block_offsets(A.nrows, brp, bcols),
                          O.da_offsets(A.nrows, A.rowptr, A.colids))
    assert np.array_equal(bvals, A.vals[:, None, None] * K[None])


def test_block_size_one_is_csr():
    A = laplace_2d_5pt(9)
    brp, bcols, bvals = B.bsr_from_csr(A.nrows, A.ncols, A.rowptr, A.colids, A.vals, 1)
    assert np.array_equal(brp, A.rowptr) and np.array_equal(bcols, A.colids)
    assert np.array_equal(bvals.ravel(), A.vals)


@pytest.mark.parametrize("b", [1, 2, 3, 5])
@pytest.mark.parametrize("seed", [0, 1])
def test_spmv_matches_dense_brute_force(b, seed):
    A = random_csr(20 * b, 30 * b, seed, mean_len=4, dup_frac=0.2, zero_frac=0.1)
    brp, bcols, bvals = B.bsr_from_csr(A.nrows, A.ncols, A.rowptr, A.colids, A.vals, b)
    Dref = S.dense(A.nrows, A.ncols, A.rowptr, A.colids, A.vals)
    nbr, nbc = A.nrows // b, A.ncols // b
    off = B.da_block_offsets(nbr, brp, bcols)
    assert np.array_equal(B.bsr_dense(nbr, nbc, b, brp, off, bvals), Dref)
    assert np.array_equal(B.bsr_dense(nbr, nbc, b, brp, bcols, bvals, da=False), Dref)
    rng = np.random.default_rng(seed)
    x, y0 = rng.uniform(-1, 1, A.ncols), rng.uniform(-1, 1, A.nrows)
    for alpha, beta in ((1.0, 0.0), (-0.5, 2.0), (0.0, 3.0)):
        y = B.spmv_bsr(nbr, nbc, b, brp, off, bvals, x, alpha, beta, y0)
        assert np.allclose(y, alpha * (Dref @ x) + beta * y0, rtol=0, atol=1e-12)
        assert np.array_equal(y, B.spmv_bsr(nbr, nbc, b, brp, bcols, bvals, x, alpha, beta, y0,
                                            da=False))


def test_beta_zero_ignores_nan_and_alpha_zero_ignores_x():
    A = laplace_2d_5pt(4)
    brp, bc, bv = B.bsr_from_csr(16, 16, A.rowptr, A.colids, A.vals, 2)
    off = B.da_block_offsets(8, brp, bc)
    y = B.spmv_bsr(8, 8, 2, brp, off, bv, np.ones(16), 1.0, 0.0, np.full(16, np.nan))
    assert np.all(np.isfinite(y))
    y = B.spmv_bsr(8, 8, 2, brp, off, bv, np.full(16, np.nan), 0.0, 2.0, np.ones(16))
    assert np.all(y == 2.0)


def test_kronecker_identity_closed_form():
    # (Laplacian (x) I_3) times kron(i^2 + j^2, 1): every component of an
    # interior block row is -4, exactly
    N = 12
    A = laplace_2d_5pt(N)
    n, m, rp, c, v = _kron(A, np.eye(3))
    keep = v != 0
    rows = O.entry_rows(n, rp)[keep]
    rp2 = np.concatenate([[0], np.cumsum(np.bincount(rows, minlength=n))]).astype(np.int32)
    brp, bcols, bvals = B.bsr_from_csr(n, m, rp2, c[keep], v[keep], 3)
    i, j = np.meshgrid(np.arange(N), np.arange(N), indexing="xy")
    x = np.repeat((i.ravel() ** 2 + j.ravel() ** 2).astype(float), 3)
    y = B.spmv_bsr(N * N, N * N, 3, brp, B.da_block_offsets(N * N, brp, bcols), bvals, x)
    interior = np.repeat(((i > 0) & (i < N - 1) & (j > 0) & (j < N - 1)).ravel(), 3)
    assert np.all(y[interior] == -4.0)


def test_rejects_sizes_not_multiple_of_block():
    A = laplace_2d_5pt(3)
    with pytest.raises(ValueError):
        B.bsr_from_csr(A.nrows, A.ncols, A.rowptr, A.colids, A.vals, 2)


def test_block_offset_fit_boundary():
    # one block at block distance 32767 fits, 32768 does not
    for d, fits in ((32767, True), (32768, False)):
        nb = d + 1
        brp = np.zeros(nb + 1, dtype=np.int32)
        brp[1:] = 1
        if fits:
            assert B.da_block_offsets(nb, brp, [d]).tolist() == [d]
        else:
            with pytest.raises(O.NoFit):
                B.da_block_offsets(nb, brp, [d])


def test_traffic_b1_matches_eq3():
    # block size 1: one 2-byte offset and one scalar per entry, as DA-CSR
    assert B.bsr_bytes(1000, 1000, 5000, 1) == T.spmv_bytes(1000, 1000, 5000, 2, 8)
    # b = 3: 2/9 bytes of index per entry against 4/9 for int32 block columns
    db = B.bsr_bytes(1000, 1000, 5000, 3, 2) - 4 * 1001 - 8 * 3 * 2000
    cb = B.bsr_bytes(1000, 1000, 5000, 3, 4) - 4 * 1001 - 8 * 3 * 2000
    assert (db, cb) == (5000 * (2 + 72), 5000 * (4 + 72))
