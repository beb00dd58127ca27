"""Host-side DA-COO / COO encoding and upload validation (no GPU),
bit-exact against the oracle."""

import ctypes as C

import numpy as np
import pytest

import paper_2307_06305_amd as D
from oracle import coo as OC
from workloads import laplace_2d_5pt, random_banded, random_csr


def _mats():
    yield laplace_2d_5pt(9)
    yield random_banded(4000, 5, half_band=500)
    yield random_csr(300, 200, 2, mean_len=6, empty_frac=0.3, dup_frac=0.2, shuffle_rows=True)
    yield random_csr(0, 4, 1)


@pytest.mark.parametrize("A", list(_mats()), ids=lambda A: A.name)
@pytest.mark.parametrize("fmt", [D.FORMAT_DACOO16, D.FORMAT_COO32])
def test_coo_encode_matches_oracle(A, fmt):
    da = fmt == D.FORMAT_DACOO16
    r_ref, i_ref = OC.coo_from_csr(A.nrows, A.ncols, A.rowptr, A.colids, da)
    rows, idx = D.coo_encode(A.nrows, A.ncols, A.rowptr, A.colids, fmt)
    assert np.array_equal(rows, r_ref)
    assert idx.dtype == i_ref.dtype and np.array_equal(idx, i_ref)


def test_coo_encode_no_fit():
    n = 40000
    rp = np.zeros(n + 1, dtype=np.int32)
    rp[1:] = 1
    col = np.array([32768], dtype=np.int32)
    with pytest.raises(D.NoFit) as e:
        D.coo_encode(n, n, rp, col)
    assert e.value.w == 32768
    assert D.coo_encode(n, n, rp, col, D.FORMAT_COO32)[1].tolist() == [32768]


def _status(fmt, nrows, ncols, rows, idx, store=D.F64):
    h = C.c_void_p()
    v = np.ones(len(rows))
    return D.lib.damn_coo_create(C.byref(h), fmt, nrows, ncols, len(rows),
                                 rows.ctypes.data_as(C.POINTER(C.c_int32)),
                                 idx.ctypes.data_as(C.c_void_p), v.ctypes.data_as(C.c_void_p),
                                 D.F64, store, None)


def test_coo_create_host_validation():
    i16 = lambda *a: np.array(a, dtype=np.int16)  # noqa: E731
    r32 = lambda *a: np.array(a, dtype=np.int32)  # noqa: E731
    assert _status(D.FORMAT_DACOO16, 3, 3, r32(1, 0), i16(0, 0)) == -2        # rows out of order
    assert _status(D.FORMAT_DACOO16, 3, 3, r32(0, 3), i16(0, 0)) == -2        # row out of range
    assert _status(D.FORMAT_DACOO16, 3, 3, r32(0, 2), i16(0, 1)) == -2        # column 3 >= ncols
    assert _status(D.FORMAT_COO32, 3, 3, r32(0, 1), r32(0, -1)) == -2         # column < 0
    assert _status(D.FORMAT_DACOO16, 3, 3, r32(0), i16(0), D.F16) == -6       # float16 values
    assert _status(D.FORMAT_DA16, 3, 3, r32(0), i16(0)) == -1                 # not coordinates
