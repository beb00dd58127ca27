"""The oracle's DA-COO (Sec. 1: diagonal addressing applied to one index
vector of COO).  Pins: Example 1 (Sec. 2) as coordinates by hand; the int16
boundary; dense brute force; the integer Laplacian closed form; traffic
against Eq. 3's per-entry bytes."""

import numpy as np
import pytest

from conftest import golden
from oracle import coo as OC
from oracle import spmv as S
from oracle import storage as O
from workloads import laplace_2d_5pt, random_csr


def test_example1_coordinates_by_hand():
    g = golden("example1.json")
    rows, off = OC.coo_from_csr(4, 4, g["rowptr"], g["csr_colids"])
    assert rows.tolist() == [0, 1, 2, 2, 3]
    assert off.dtype == np.int16 and off.tolist() == g["da_colids"]
    rows, cols = OC.coo_from_csr(4, 4, g["rowptr"], g["csr_colids"], da=False)
    assert cols.tolist() == g["csr_colids"]


@pytest.mark.parametrize("d,fits", [(32767, True), (32768, False)])
def test_int16_boundary(d, fits):
    n = d + 1
    rp = np.zeros(n + 1, dtype=np.int32)
    rp[1:] = 1
    col = np.array([d], dtype=np.int32)
    if fits:
        assert OC.coo_from_csr(n, n, rp, col)[1].tolist() == [d]
    else:
        with pytest.raises(O.NoFit):
            OC.coo_from_csr(n, n, rp, col)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_matches_dense_brute_force(seed):
    A = random_csr(90, 70, seed, mean_len=5, empty_frac=0.3, dup_frac=0.2, zero_frac=0.1,
                   shuffle_rows=True)
    D = S.dense(A.nrows, A.ncols, A.rowptr, A.colids, A.vals)
    rng = np.random.default_rng(seed)
    x, y0 = rng.uniform(-1, 1, A.ncols), rng.uniform(-1, 1, A.nrows)
    for da in (True, False):
        rows, idx = OC.coo_from_csr(A.nrows, A.ncols, A.rowptr, A.colids, da)
        for alpha, beta in ((1.0, 0.0), (2.0, -0.5), (0.0, 1.0)):
            y = OC.spmv_coo(A.nrows, A.ncols, rows, idx, A.vals, x, alpha, beta, y0, da)
            assert np.allclose(y, alpha * (D @ x) + beta * y0, rtol=0, atol=1e-12)


def test_same_sums_as_csr_bit_for_bit():
    A = random_csr(200, 200, 7, mean_len=9, dup_frac=0.1)
    x = np.random.default_rng(8).uniform(-1, 1, 200)
    rows, off = OC.coo_from_csr(A.nrows, A.ncols, A.rowptr, A.colids)
    assert np.array_equal(OC.spmv_coo(A.nrows, A.ncols, rows, off, A.vals, x),
                          S.spmv_csr(A.nrows, A.ncols, A.rowptr, A.colids, A.vals, x))


def test_laplacian_closed_form():
    N = 10
    A = laplace_2d_5pt(N)
    rows, off = OC.coo_from_csr(A.nrows, A.ncols, A.rowptr, A.colids)
    i, j = np.meshgrid(np.arange(N), np.arange(N), indexing="xy")
    y = OC.spmv_coo(A.nrows, A.ncols, rows, off, A.vals, (i ** 2 + j ** 2).ravel().astype(float))
    interior = ((i > 0) & (i < N - 1) & (j > 0) & (j < N - 1)).ravel()
    assert np.all(y[interior] == -4.0)


def test_beta_zero_ignores_nan():
    A = laplace_2d_5pt(3)
    rows, off = OC.coo_from_csr(A.nrows, A.ncols, A.rowptr, A.colids)
    y = OC.spmv_coo(9, 9, rows, off, A.vals, np.ones(9), 1.0, 0.0, np.full(9, np.nan))
    assert np.all(np.isfinite(y))


def test_traffic_per_entry():
    # 14 bytes per entry for DA-COO (4 + 2 + 8) against 10 for DA-CSR's
    # entries, which pay 4 bytes per row instead
    t = OC.coo_bytes(1000, 1000, 5000)
    assert t == 5000 * 14 + 8 * 1000 + 8 * 1000
    assert OC.coo_bytes(1000, 1000, 5000, 4) - t == 5000 * 2
