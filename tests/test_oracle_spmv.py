"""Pins of the oracle's products: brute-force dense products, integer-exact
stencil closed forms, and the beta / alpha conventions."""

import numpy as np
import pytest

from oracle import spmv as S
from oracle import storage as ST
from workloads import laplace_2d_5pt, poisson_3d_7pt, random_csr, stencil_3d_27pt, uniform_vector


def _shapes():
    yield 64, 64, dict(mean_len=5)
    yield 200, 80, dict(mean_len=4, band=30)     # tall
    yield 80, 200, dict(mean_len=7, band=60)     # wide
    yield 300, 300, dict(mean_len=3, dup_frac=0.3, zero_frac=0.2, shuffle_rows=True)
    yield 512, 512, dict(mean_len=10, empty_frac=0.4)


@pytest.mark.parametrize("shape", list(_shapes()), ids=lambda s: f"{s[0]}x{s[1]}")
@pytest.mark.parametrize("alpha,beta", [(1.0, 0.0), (-2.5, 0.75), (0.0, 3.0)])
def test_spmv_matches_dense_product(shape, alpha, beta):
    nrows, ncols, kw = shape
    A = random_csr(nrows, ncols, 7, **kw)
    D = S.dense(nrows, ncols, A.rowptr, A.colids, A.vals)
    x = uniform_vector(ncols, 1)
    y0 = uniform_vector(nrows, 2)
    want = alpha * (D @ x) + beta * y0
    got = S.spmv_csr(nrows, ncols, A.rowptr, A.colids, A.vals, x, alpha, beta, y0)
    assert np.allclose(got, want, rtol=1e-13, atol=1e-13)
    w, _, _, fits = ST.fit(nrows, ncols, A.rowptr, A.colids)
    if fits:
        off = ST.da_offsets(nrows, A.rowptr, A.colids)
        got_da = S.spmv_da(nrows, ncols, A.rowptr, off, A.vals, x, alpha, beta, y0)
        assert np.array_equal(got_da, got)


def test_integer_values_exact():
    # integer entries and vectors: every order of summation is exact
    A = random_csr(300, 250, 3, mean_len=8, band=100, int_values=True, dup_frac=0.2)
    D = S.dense(300, 250, A.rowptr, A.colids, A.vals)
    x = np.random.default_rng(0).integers(-5, 6, 250).astype(np.float64)
    off = ST.da_offsets(300, A.rowptr, A.colids)
    assert np.array_equal(S.spmv_da(300, 250, A.rowptr, off, A.vals, x), D @ x)


def test_laplace_2d_times_ones_gives_row_sums():
    N = 16
    A = laplace_2d_5pt(N)
    y = S.spmv_csr(A.nrows, A.ncols, A.rowptr, A.colids, A.vals, np.ones(A.ncols))
    g = y.reshape(N, N)
    assert g[1:-1, 1:-1].max() == 0 and g[1:-1, 1:-1].min() == 0
    assert g[0, 0] == g[0, -1] == g[-1, 0] == g[-1, -1] == 2
    assert np.all(g[0, 1:-1] == 1) and np.all(g[1:-1, 0] == 1)


def test_laplace_2d_times_quadratic_gives_minus_four_inside():
    N = 20
    A = laplace_2d_5pt(N)
    j, i = np.indices((N, N))
    f = (i ** 2 + j ** 2).astype(np.float64).ravel()
    off = ST.da_offsets(A.nrows, A.rowptr, A.colids)
    y = S.spmv_da(A.nrows, A.ncols, A.rowptr, off, A.vals, f).reshape(N, N)
    assert np.all(y[1:-1, 1:-1] == -4.0)
    # boundary row i = 0: the missing neighbour (-1, j) adds 1 + j^2
    assert np.array_equal(y[1:-1, 0], -4.0 + 1.0 + np.arange(1, N - 1) ** 2)


def test_poisson_3d_times_quadratic_gives_minus_six_inside():
    A = poisson_3d_7pt(7, 8, 9)
    k, j, i = np.indices((9, 8, 7))
    f = (i ** 2 + j ** 2 + k ** 2).astype(np.float64).ravel()
    y = S.spmv_csr(A.nrows, A.ncols, A.rowptr, A.colids, A.vals, f).reshape(9, 8, 7)
    assert np.all(y[1:-1, 1:-1, 1:-1] == -6.0)


def test_27pt_diagonal_dominance_row_sum():
    A = stencil_3d_27pt(6, 1)
    absA = S.spmv_csr(A.nrows, A.ncols, A.rowptr, A.colids, np.abs(A.vals), np.ones(A.ncols))
    diag = A.vals[A.colids == ST.entry_rows(A.nrows, A.rowptr)]
    # diagonal = 1 + sum |off-diagonal|  =>  sum |row| = 2 diag - 1
    assert np.allclose(absA, 2 * diag - 1, rtol=0, atol=1e-12)


def test_beta_zero_ignores_nan_y0():
    A = random_csr(40, 40, 1)
    y0 = np.full(40, np.nan)
    y = S.spmv_csr(40, 40, A.rowptr, A.colids, A.vals, np.ones(40), 1.0, 0.0, y0)
    assert np.all(np.isfinite(y))


def test_alpha_zero_does_not_read_x():
    A = random_csr(40, 40, 1)
    y0 = uniform_vector(40, 3)
    y = S.spmv_csr(40, 40, A.rowptr, A.colids, A.vals, np.full(40, np.nan), 0.0, 2.0, y0)
    assert np.array_equal(y, 2.0 * y0)


def test_empty_rows_give_beta_y0():
    rp = np.array([0, 0, 2, 2])
    c = np.array([0, 1])
    y0 = np.array([1.5, 2.5, -3.0])
    y = S.spmv_csr(3, 2, rp, c, np.array([1.0, 1.0]), np.array([1.0, 2.0]), 1.0, 2.0, y0)
    assert y.tolist() == [3.0, 8.0, -6.0]


def test_spmm_is_columnwise_spmv():
    A = random_csr(90, 70, 5, mean_len=6, band=20)
    D = S.dense(90, 70, A.rowptr, A.colids, A.vals)
    X = uniform_vector(70, 4, 5)
    Y0 = uniform_vector(90, 5, 5)
    off = ST.da_offsets(90, A.rowptr, A.colids)
    Y = S.spmm_da(90, 70, A.rowptr, off, A.vals, X, 0.5, -1.0, Y0)
    assert np.allclose(Y, 0.5 * D @ X - Y0, rtol=1e-13, atol=1e-13)


def test_abs_products_brute_force():
    A = random_csr(30, 30, 2, mean_len=4)
    x = uniform_vector(30, 9)
    D = S.dense(30, 30, A.rowptr, A.colids, np.abs(A.vals))
    assert np.allclose(S.abs_products(30, A.rowptr, A.colids, A.vals, x), D @ np.abs(x),
                       rtol=1e-14, atol=1e-15)
