"""Host-side BSR / DA-BSR encoding (no GPU): bit-exact against the oracle
(block structure, offsets, summed values), the fit boundary and errors."""

import ctypes as C

import numpy as np
import pytest

import paper_2307_06305_amd as D
from oracle import blocks as OB
from oracle import storage as OS
from workloads import laplace_2d_5pt, random_csr, stencil_3d_27pt


def _mats():
    yield 2, laplace_2d_5pt(8)
    yield 3, stencil_3d_27pt(6, 2)
    yield 4, random_csr(80, 120, 3, mean_len=6, dup_frac=0.3, zero_frac=0.1, shuffle_rows=True)
    yield 6, random_csr(120, 60, 4, mean_len=5, band=30, dup_frac=0.2)
    yield 2, random_csr(0, 0, 1)
    yield 3, random_csr(9, 6, 5, mean_len=0.5, empty_frac=0.6)


@pytest.mark.parametrize("b,A", list(_mats()), ids=lambda v: getattr(v, "name", str(v)))
@pytest.mark.parametrize("fmt", [D.FORMAT_DABSR16, D.FORMAT_BSR32])
def test_bsr_encode_matches_oracle_bit_exact(b, A, fmt):
    rp, bc, bv = OB.bsr_from_csr(A.nrows, A.ncols, A.rowptr, A.colids, A.vals, b)
    e = D.bsr_encode(A.nrows, A.ncols, A.rowptr, A.colids, A.vals, b, fmt)
    assert np.array_equal(e["browptr"], rp)
    nbr = A.nrows // b
    want = OB.da_block_offsets(nbr, rp, bc) if fmt == D.FORMAT_DABSR16 else bc.astype(np.int32)
    assert e["bidx"].dtype == want.dtype and np.array_equal(e["bidx"], want)
    assert np.array_equal(e["bvals"].view(np.uint64), bv.view(np.uint64))  # bit for bit
    assert e["wb"] == OB.block_bandwidth(nbr, rp, bc)


def test_bsr_example1_by_hand():
    rp = np.array([0, 1, 2, 4, 5], dtype=np.int32)
    c = np.array([0, 2, 1, 3, 3], dtype=np.int32)
    e = D.bsr_encode(4, 4, rp, c, np.arange(1.0, 6.0), 2)
    assert e["browptr"].tolist() == [0, 2, 4]
    assert e["bidx"].tolist() == [0, 1, -1, 0]
    assert e["bvals"].reshape(4, 4).tolist() == [[1, 0, 0, 0], [0, 0, 2, 0], [0, 3, 0, 0],
                                                 [0, 4, 0, 5]]


@pytest.mark.parametrize("d,fits", [(32767, True), (32768, False)])
def test_bsr_block_offset_boundary(d, fits):
    b = 2
    nb = d + 1
    n = nb * b
    rp = np.zeros(n + 1, dtype=np.int32)
    rp[1:] = 1  # one entry in row 0, at column d*b
    col = np.array([d * b], dtype=np.int32)
    if fits:
        e = D.bsr_encode(n, n, rp, col, np.ones(1), b)
        assert e["bidx"].tolist() == [d]
    else:
        with pytest.raises(D.NoFit) as err:
            D.bsr_encode(n, n, rp, col, np.ones(1), b)
        assert err.value.w == d
        # the absolute-column form has no such limit
        assert D.bsr_encode(n, n, rp, col, np.ones(1), b, D.FORMAT_BSR32)["bidx"].tolist() == [d]


def test_bsr_rejects_sizes_not_multiple_of_block():
    A = laplace_2d_5pt(3)
    with pytest.raises(D.DamnError) as e:
        D.bsr_encode(A.nrows, A.ncols, A.rowptr, A.colids, A.vals, 2)
    assert e.value.code == -1


def _bsr_create_status(fmt, nbr, nbc, b, brp, bidx, bvals, store=D.F64):
    h = C.c_void_p()
    return D.lib.damn_bsr_create(C.byref(h), fmt, nbr, nbc, b, brp.ctypes.data_as(
        C.POINTER(C.c_int32)), bidx.ctypes.data_as(C.c_void_p), bvals.ctypes.data_as(C.c_void_p),
        D.F64, store, None)


def test_bsr_create_host_validation():
    brp = np.array([0, 1, 2], dtype=np.int32)
    v = np.ones(8)
    # block offsets leaving [0, nbcols)
    assert _bsr_create_status(D.FORMAT_DABSR16, 2, 2, 2, brp, np.array([0, 1], np.int16), v) == -2
    assert _bsr_create_status(D.FORMAT_BSR32, 2, 2, 2, brp, np.array([0, 2], np.int32), v) == -2
    # unsupported block size and float16 values
    assert _bsr_create_status(D.FORMAT_DABSR16, 2, 2, 5, brp, np.zeros(2, np.int16),
                              np.ones(50)) == -6
    assert _bsr_create_status(D.FORMAT_DABSR16, 2, 2, 2, brp, np.zeros(2, np.int16), v,
                              D.F16) == -6
    # not a block format
    assert _bsr_create_status(D.FORMAT_DA16, 2, 2, 2, brp, np.zeros(2, np.int16), v) == -1
