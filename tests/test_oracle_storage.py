"""Pins of the oracle's storage functions (fit, DA transform, permutation)
against the paper's Example 1, closed-form bandwidths and brute force."""

import numpy as np
import pytest

from conftest import golden
from oracle import storage as S
from oracle.spmv import dense
from workloads import laplace_2d_5pt, poisson_3d_7pt, stencil_3d_27pt, random_csr


def test_example1_fit_and_da_colids():
    g = golden("example1.json")
    rp = np.array(g["rowptr"], dtype=np.int32)
    c = np.array(g["csr_colids"], dtype=np.int32)
    w, lo, hi, fits = S.fit(g["nrows"], g["ncols"], rp, c)
    assert w == g["w"] and fits
    off = S.da_offsets(g["nrows"], rp, c)
    assert off.dtype == np.int16
    assert off.tolist() == g["da_colids"]
    # Example 1: DA colids cover exactly [-w, w]
    assert set(off.tolist()) == set(range(-w, w + 1))
    assert (lo, hi) == (1, 1)
    # the (row, col) positions drawn in Fig. 1
    rows = S.entry_rows(4, rp)
    assert [[int(r), int(cc)] for r, cc in zip(rows, c)] == g["entries_rc"]


def test_example1_encode_keeps_order_and_values():
    g = golden("example1.json")
    vals = np.array([1.0, 2.0, 3.0, 4.0, 5.0])
    e = S.encode(4, 4, np.array(g["rowptr"]), np.array(g["csr_colids"]), vals)
    assert not e["permuted"]
    assert e["rowptr"].tolist() == g["rowptr"]
    assert e["off"].tolist() == g["da_colids"]
    assert e["vals"].tolist() == vals.tolist()
    assert e["perm"].tolist() == [0, 1, 2, 3]


@pytest.mark.parametrize("N", [3, 5, 16, 64])
def test_bandwidth_2d_5pt_is_N(N):
    A = laplace_2d_5pt(N)
    assert S.fit(A.nrows, A.ncols, A.rowptr, A.colids)[0] == N


@pytest.mark.parametrize("N", [3, 7, 20])
def test_bandwidth_3d_7pt_is_N2(N):
    A = poisson_3d_7pt(N, N, N)
    assert S.fit(A.nrows, A.ncols, A.rowptr, A.colids)[0] == N * N


@pytest.mark.parametrize("N", [3, 6, 12])
def test_bandwidth_3d_27pt_is_N2_N_1(N):
    A = stencil_3d_27pt(N, 7)
    assert S.fit(A.nrows, A.ncols, A.rowptr, A.colids)[0] == N * N + N + 1


def test_bandwidth_27pt_128_closed_form():
    # the 128^3 27-point workload: w = 128^2 + 128 + 1 = 16513, nnz = 382^3
    assert 128 * 128 + 128 + 1 == 16513
    A = stencil_3d_27pt(10, 1)
    assert A.nnz == (3 * 10 - 2) ** 3


def test_stencil_entry_counts():
    assert laplace_2d_5pt(64).nnz == 20224
    assert poisson_3d_7pt(4, 5, 6).nnz == 7 * 120 - 2 * (5 * 6 + 4 * 6 + 4 * 5)


@pytest.mark.parametrize("d,fits", [(32767, True), (32768, False)])
def test_int16_boundary_upper(d, fits):
    rp = np.array([0, 1, 1], dtype=np.int32)
    c = np.array([d], dtype=np.int32)
    w, lo, hi, f = S.fit(2, d + 1, rp, c)
    assert (w, lo, hi, f) == (d, 0, d, fits)


@pytest.mark.parametrize("d,fits", [(32767, True), (32768, False)])
def test_int16_boundary_lower(d, fits):
    n = d + 1
    rp = np.zeros(n + 1, dtype=np.int32)
    rp[n] = 1  # single entry in the last row, column 0
    c = np.array([0], dtype=np.int32)
    w, lo, hi, f = S.fit(n, 1, rp, c)
    assert (w, lo, hi, f) == (d, d, 0, fits)
    if fits:
        off = S.da_offsets(n, rp, c)
        assert off.tolist() == [-d]


def test_empty_matrix_fit():
    assert S.fit(0, 0, np.array([0]), np.array([], dtype=np.int32)) == (0, 0, 0, True)
    assert S.fit(3, 5, np.array([0, 0, 0, 0]), np.array([], dtype=np.int32)) == (0, 0, 0, True)


def test_explicit_zeros_count_in_bandwidth():
    # footnote of Example 2: pattern entries include stored zeros
    rp = np.array([0, 2, 3])
    c = np.array([0, 1, 1])
    # row 0 holds a stored zero at column 1: bandwidth counts it
    w = S.fit(2, 2, rp, c)[0]
    assert w == 1


@pytest.mark.parametrize("bad", [
    dict(rowptr=[1, 1, 2], colids=[0, 1]),          # rowptr[0] != 0
    dict(rowptr=[0, 2, 1], colids=[0]),             # decreasing
    dict(rowptr=[0, 1, 3], colids=[0, 1]),          # rowptr[n] != nnz
    dict(rowptr=[0, 1, 2], colids=[0, 2]),          # column out of range
    dict(rowptr=[0, 1, 2], colids=[0, -1]),         # negative column
    dict(rowptr=[0, 1], colids=[0]),                # wrong length
])
def test_bad_csr_rejected(bad):
    with pytest.raises(S.BadCSR):
        S.fit(2, 2, np.array(bad["rowptr"]), np.array(bad["colids"]))


@pytest.mark.parametrize("seed", range(6))
def test_round_trip_random(seed):
    A = random_csr(60, 45, seed, band=15, dup_frac=0.2, zero_frac=0.1, shuffle_rows=seed % 2 == 1)
    e = S.encode(A.nrows, A.ncols, A.rowptr, A.colids, A.vals, allow_rcm=False)
    assert np.array_equal(S.da_columns(A.nrows, e["rowptr"], e["off"]), A.colids)
    assert np.array_equal(e["vals"], A.vals)


def test_example1_permuted_by_hand():
    # P A P^T with perm = (3, 2, 1, 0), worked by hand from Fig. 1:
    # new row 0 = old row 3 (entry e5 at old col 3 -> new col 0)
    # new row 1 = old row 2 (e3 at old col 1 -> 2, e4 at old col 3 -> 0)
    # new row 2 = old row 1 (e2 at old col 2 -> 1); new row 3 = old row 0 (e1)
    g = golden("example1.json")
    vals = np.array([1.0, 2.0, 3.0, 4.0, 5.0])
    rp, c, v = S.permute_symmetric(4, np.array(g["rowptr"]), np.array(g["csr_colids"]), vals,
                                   np.array([3, 2, 1, 0]))
    assert rp.tolist() == [0, 1, 3, 4, 5]
    assert c.tolist() == [0, 0, 2, 1, 3]
    assert v.tolist() == [5.0, 4.0, 3.0, 2.0, 1.0]
    assert S.da_offsets(4, rp, c).tolist() == [0, -1, 1, -1, 0]


@pytest.mark.parametrize("seed", range(4))
def test_permute_matches_dense_brute_force(seed):
    A = random_csr(40, 40, seed, mean_len=5, dup_frac=0.1, shuffle_rows=True)
    perm = np.random.default_rng(seed).permutation(40)
    rp, c, v = S.permute_symmetric(40, A.rowptr, A.colids, A.vals, perm)
    D = dense(40, 40, A.rowptr, A.colids, A.vals)
    Dp = dense(40, 40, rp, c, v)
    assert np.allclose(Dp, D[np.ix_(perm, perm)], rtol=0, atol=1e-15)
    # rows of the result are sorted by column, repeated columns keep their order
    rows = S.entry_rows(40, rp)
    assert np.all((np.diff(rows) > 0) | (np.diff(c) >= 0))


def test_encode_no_fit_without_rcm():
    n = 40000
    rp = np.arange(n + 1, dtype=np.int32)
    c = np.arange(n, dtype=np.int32)[::-1].copy()  # anti-diagonal: w = n-1
    with pytest.raises(S.NoFit) as ei:
        S.encode(n, n, rp, c, np.ones(n), allow_rcm=False)
    assert ei.value.w == n - 1


def test_encode_rectangular_no_fit_is_not_reordered():
    rp = np.array([0, 1], dtype=np.int32)
    c = np.array([40000], dtype=np.int32)
    with pytest.raises(S.NoFit):
        S.encode(1, 40001, rp, c, np.ones(1), allow_rcm=True)


def test_encode_antidiagonal_with_rcm_fits():
    # the anti-diagonal pattern is a perfect matching; RCM pairs each i with
    # n-1-i, so the reordered bandwidth is 1
    n = 40000
    rp = np.arange(n + 1, dtype=np.int32)
    c = np.arange(n, dtype=np.int32)[::-1].copy()
    e = S.encode(n, n, rp, c, np.arange(n, dtype=np.float64), allow_rcm=True)
    assert e["permuted"] and e["w"] == 1
    perm = e["perm"].astype(np.int64)
    assert np.array_equal(np.sort(perm), np.arange(n))
