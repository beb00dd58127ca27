"""Host-side conversion into the storage grid of Fig. 3 (no GPU): the
library's index encoder and value rounding bit-exact against the oracle, the
fit boundaries, and the upload's host-side validation."""

import numpy as np
import pytest

import paper_2307_06305_amd as D
from oracle import storage as OS
from workloads import laplace_2d_5pt, random_banded, random_csr, stencil_3d_27pt

from test_oracle_formats import F16_CASES

FMT = {"da16": D.FORMAT_DA16, "csr32": D.FORMAT_CSR32, "da8": D.FORMAT_DA8,
       "csr16": D.FORMAT_CSR16}


def _mats():
    yield laplace_2d_5pt(17)                        # w = 17: every format
    yield stencil_3d_27pt(5, 1)                     # w = 31
    yield random_banded(3000, 2, half_band=100)     # w <= 100, ncols 3000
    yield random_banded(40000, 3, half_band=127)    # csr16 does not fit
    yield random_banded(3000, 4, half_band=600)     # da8 does not fit
    for s in range(3):
        yield random_csr(300, 200, s, band=20, dup_frac=0.2, zero_frac=0.1, shuffle_rows=True)
    yield random_csr(0, 0, 1)
    yield random_csr(4, 0, 1)


@pytest.mark.parametrize("A", list(_mats()), ids=lambda A: A.name)
@pytest.mark.parametrize("fmt", list(FMT))
def test_encode_index_matches_oracle_bit_exact(A, fmt):
    try:
        ref = OS.encode_index(fmt, A.nrows, A.ncols, A.rowptr, A.colids)
    except OS.NoFit as e:
        with pytest.raises(D.NoFit) as got:
            D.encode_index(FMT[fmt], A.nrows, A.ncols, A.rowptr, A.colids)
        assert got.value.w == e.w
        return
    idx, w = D.encode_index(FMT[fmt], A.nrows, A.ncols, A.rowptr, A.colids)
    assert idx.dtype == ref.dtype and np.array_equal(idx, ref)


@pytest.mark.parametrize("d,fits", [(126, True), (127, True), (128, False), (-127, True),
                                    (-128, False)])
def test_da8_boundary(d, fits):
    n = 300
    r = 150
    rp = np.zeros(n + 1, dtype=np.int32)
    rp[r + 1:] = 1
    col = np.array([r + d], dtype=np.int32)
    if fits:
        idx, w = D.encode_index(D.FORMAT_DA8, n, n, rp, col)
        assert int(idx[0]) == d and w == abs(d)
    else:
        with pytest.raises(D.NoFit) as e:
            D.encode_index(D.FORMAT_DA8, n, n, rp, col)
        assert e.value.w == abs(d)


@pytest.mark.parametrize("c,fits", [(32767, True), (32768, False)])
def test_csr16_boundary(c, fits):
    rp = np.array([0, 1], dtype=np.int32)
    col = np.array([c], dtype=np.int32)
    if fits:
        assert int(D.encode_index(D.FORMAT_CSR16, 1, 40000, rp, col)[0][0]) == c
    else:
        with pytest.raises(D.NoFit):
            D.encode_index(D.FORMAT_CSR16, 1, 40000, rp, col)


@pytest.mark.parametrize("v,bits", F16_CASES)
def test_f16_rounding_by_hand(v, bits):
    got = D.store_values(np.array([v, -v]), D.F16)
    assert int(got.view(np.uint16)[0]) == bits
    assert int(got.view(np.uint16)[1]) == bits ^ 0x8000  # the negated value


def _wide_values(seed, n=200_000):
    rng = np.random.default_rng(seed)
    # magnitudes from 2^-40 to 2^15.9 (subnormal, normal and near-overflow
    # float16), random signs, and exact ties
    e = rng.uniform(-40, 15.9, n)
    v = np.exp2(e) * rng.choice([-1.0, 1.0], n)
    ties = (np.arange(1, 2001, dtype=np.float64) + 0.5) * 2.0**-10  # k + 1/2 ulp in [1, 2)
    return np.concatenate([v, 1 + ties[ties < 1], [0.0, -0.0, 65504.0, -65504.0]])


@pytest.mark.parametrize("seed", [0, 1])
def test_f16_matches_oracle_bit_exact(seed):
    v = _wide_values(seed)
    got = D.store_values(v, D.F16)
    ref = OS.store_values(v, "f16")
    assert np.array_equal(got.view(np.uint16), ref.view(np.uint16))


def test_f16_from_f32_matches_oracle():
    v = _wide_values(2).astype(np.float32)
    got = D.store_values(v, D.F16)
    ref = OS.store_values(v.astype(np.float64), "f16")
    assert np.array_equal(got.view(np.uint16), ref.view(np.uint16))


def test_f32_matches_oracle_bit_exact():
    v = np.random.default_rng(4).standard_normal(100_000) * np.exp2(
        np.random.default_rng(5).uniform(-140, 120, 100_000))
    got = D.store_values(v, D.F32)
    assert np.array_equal(got.view(np.uint32), OS.store_values(v, "f32").view(np.uint32))


@pytest.mark.parametrize("v,dt", [(65520.0, D.F16), (-1e5, D.F16), (1e39, D.F32)])
def test_value_overflow_is_no_fit(v, dt):
    with pytest.raises(D.NoFit):
        D.store_values(np.array([1.0, v]), dt)


def test_store_values_rejects_widening():
    import ctypes as C

    src = np.zeros(1, np.float32)
    dst = np.zeros(1, np.float64)
    st = D.lib.damn_store_values(1, src.ctypes.data_as(C.c_void_p), D.F32, D.F64,
                                 dst.ctypes.data_as(C.c_void_p))
    assert st == -6


def _create_status(fmt, nrows, ncols, rp, idx, vals):
    """damn_create_format called directly (null stream): host validation
    returns before any device work."""
    import ctypes as C

    h = C.c_void_p()
    return D.lib.damn_create_format(C.byref(h), fmt, nrows, ncols,
                                    rp.ctypes.data_as(C.POINTER(C.c_int32)),
                                    idx.ctypes.data_as(C.c_void_p),
                                    vals.ctypes.data_as(C.c_void_p), D.F64, D.F64, None)


def test_create_format_rejects_columns_outside_x_on_the_host():
    rp = np.array([0, 1, 2], dtype=np.int32)
    assert _create_status(D.FORMAT_DA8, 2, 2, rp, np.array([-1, 0], np.int8), np.ones(2)) == -2
    assert _create_status(D.FORMAT_DA8, 2, 2, rp, np.array([0, 1], np.int8), np.ones(2)) == -2
    assert _create_status(D.FORMAT_CSR16, 2, 2, rp, np.array([0, 2], np.int16), np.ones(2)) == -2
    assert _create_status(D.FORMAT_CSR16, 2, 2, rp, np.array([-1, 0], np.int16), np.ones(2)) == -2


def test_create_format_rejects_unknown_format_and_bad_rowptr():
    rp = np.array([0, 1], dtype=np.int32)
    assert _create_status(7, 1, 1, rp, np.zeros(1, np.int16), np.ones(1)) == -1
    assert _create_status(D.FORMAT_DA16, 1, 1, np.array([1, 1], np.int32), np.zeros(1, np.int16),
                          np.ones(1)) == -2
