"""The oracle's storage grid of Fig. 3: 8/16/32-bit column indices (DA
offsets or absolute columns) and 64/32/16-bit scalars.

Pins: Example 1 (Sec. 2) in every index width; the fit boundaries derived
from the signed range of each width; IEEE 754 binary16 / binary32 encodings
worked out by hand from the format's definition (sign, 5-bit exponent with
bias 15, 10-bit fraction; subnormal step 2^-24); brute-force dense products
of the rounded values.
"""

import numpy as np
import pytest

from oracle import spmv as S
from oracle import storage as O
from workloads.matrices import random_csr

from conftest import golden


def _example1():
    g = golden("example1.json")
    return g["nrows"], g["ncols"], np.array(g["rowptr"]), np.array(g["csr_colids"])


@pytest.mark.parametrize("fmt,dtype", [("da16", np.int16), ("da8", np.int8)])
def test_example1_da_offsets_every_width(fmt, dtype):
    n, m, rp, c = _example1()
    off = O.encode_index(fmt, n, m, rp, c)
    assert off.dtype == dtype
    assert off.tolist() == golden("example1.json")["da_colids"]


@pytest.mark.parametrize("fmt,dtype", [("csr32", np.int32), ("csr16", np.int16)])
def test_example1_csr_columns_every_width(fmt, dtype):
    n, m, rp, c = _example1()
    col = O.encode_index(fmt, n, m, rp, c)
    assert col.dtype == dtype and col.tolist() == c.tolist()


def _one_entry(nrows, ncols, r, c):
    rp = np.zeros(nrows + 1, dtype=np.int32)
    rp[r + 1:] = 1
    return rp, np.array([c], dtype=np.int32)


@pytest.mark.parametrize("r,c,fits", [(0, 127, True), (0, 128, False), (127, 0, True),
                                      (128, 0, False), (300, 173, True), (300, 172, False)])
def test_int8_offset_boundary(r, c, fits):
    # int8 holds -128..127; the symmetric rule admits |c - r| <= 127 only
    rp, col = _one_entry(400, 400, r, c)
    if fits:
        off = O.encode_index("da8", 400, 400, rp, col)
        assert off.dtype == np.int8 and int(off[0]) == c - r
    else:
        with pytest.raises(O.NoFit) as e:
            O.encode_index("da8", 400, 400, rp, col)
        assert e.value.w == abs(c - r)


@pytest.mark.parametrize("c,fits", [(0, True), (32767, True), (32768, False), (39999, False)])
def test_int16_column_boundary(c, fits):
    rp, col = _one_entry(3, 40000, 1, c)
    if fits:
        assert int(O.encode_index("csr16", 3, 40000, rp, col)[0]) == c
    else:
        with pytest.raises(O.NoFit):
            O.encode_index("csr16", 3, 40000, rp, col)


def test_index_limits():
    assert [O.index_limit(b) for b in (1, 2, 4)] == [128, 32768, 2**31]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_da8_round_trip_banded(seed):
    rng = np.random.default_rng(seed)
    n = 500
    rows, cols = [], []
    for r in range(n):
        k = rng.integers(0, 9)
        lo, hi = max(0, r - 127), min(n - 1, r + 127)
        cols += sorted(rng.integers(lo, hi + 1, k).tolist())
        rows += [r] * k
    rp = np.zeros(n + 1, dtype=np.int32)
    np.add.at(rp, np.array(rows, dtype=np.int64) + 1, 1)
    rp = np.cumsum(rp).astype(np.int32)
    c = np.array(cols, dtype=np.int32)
    off = O.encode_index("da8", n, n, rp, c)
    assert np.array_equal(O.da_columns(n, rp, off), c)


# IEEE 754 binary16: bits = sign | exponent (5, bias 15) | fraction (10)
F16_CASES = [
    (1.0, 0x3C00),
    (-2.0, 0xC000),
    (1.0 / 3.0, 0x3555),           # 1365/4096 = 0.333251953125 (1366/4096 is further away)
    (65504.0, 0x7BFF),             # largest finite
    (65519.99, 0x7BFF),            # below the midpoint 65520
    (2.0**-24, 0x0001),            # smallest subnormal
    (2.0**-25, 0x0000),            # tie between 0 and 2^-24: even is 0
    (3 * 2.0**-25, 0x0002),        # tie between 1 and 2 ulps: even is 2
    (2.0**-14, 0x0400),            # smallest normal
    (1 + 2.0**-11, 0x3C00),        # tie between 0x3C00 and 0x3C01: even
    (1 + 3 * 2.0**-11, 0x3C02),    # tie between 0x3C01 and 0x3C02: even
    (1 + 2.0**-11 + 2.0**-40, 0x3C01),  # just above the tie: up (float32 first would give 0x3C00)
    (0.0, 0x0000),
]


@pytest.mark.parametrize("v,bits", F16_CASES)
def test_binary16_rounding_by_hand(v, bits):
    got = O.store_values([v], "f16")
    assert got.dtype == np.float16
    assert int(got.view(np.uint16)[0]) == bits


def test_binary16_value_of_one_third():
    # 0x3555: exponent 13 - 15 = -2, fraction 0x155 = 341: (1 + 341/1024) / 4
    assert float(O.store_values([1 / 3], "f16")[0]) == (1 + 341 / 1024) / 4


@pytest.mark.parametrize("v", [65520.0, -65520.0, 1e6, 1e300])
def test_binary16_overflow_is_no_fit(v):
    with pytest.raises(O.NoFit):
        O.store_values([1.0, v], "f16")


def test_binary16_infinite_inputs_stay_infinite():
    got = O.store_values([np.inf, -np.inf], "f16")
    assert np.isinf(got).all()


@pytest.mark.parametrize("v,bits", [
    (1.0, 0x3F800000),
    (1 + 2.0**-24, 0x3F800000),            # tie: even
    (1 + 2.0**-24 + 2.0**-50, 0x3F800001),  # above the tie
    (1 + 3 * 2.0**-24, 0x3F800002),        # tie between ...01 and ...02: even
    (2.0**-149, 0x00000001),               # smallest subnormal
])
def test_binary32_rounding_by_hand(v, bits):
    got = O.store_values([v], "f32")
    assert int(got.view(np.uint32)[0]) == bits


def test_binary64_is_identity():
    v = np.random.default_rng(3).standard_normal(100)
    assert np.array_equal(O.store_values(v, "f64"), v)


@pytest.mark.parametrize("fmt", ["da16", "csr32", "da8", "csr16"])
@pytest.mark.parametrize("vt", ["f64", "f32", "f16"])
def test_grid_product_matches_dense_brute_force(fmt, vt):
    """Every index format with every scalar type against the dense product
    of the rounded values (float64 arithmetic on the stored operands)."""
    seed = 10 * ["da16", "csr32", "da8", "csr16"].index(fmt) + ["f64", "f32", "f16"].index(vt)
    A = random_csr(120, 100, seed, mean_len=6.0, dup_frac=0.1, zero_frac=0.05)
    # keep the bandwidth well inside int8 for da8: drop entries with |c - r| > 60
    rows = O.entry_rows(A.nrows, A.rowptr)
    keep = np.abs(A.colids.astype(np.int64) - rows) <= 60
    rl = np.bincount(rows[keep], minlength=A.nrows)
    rp = np.concatenate([[0], np.cumsum(rl)]).astype(np.int32)
    c = A.colids[keep]
    v = O.store_values(A.vals[keep], vt)
    idx = O.encode_index(fmt, A.nrows, A.ncols, rp, c)
    x = np.random.default_rng(5).uniform(-1, 1, A.ncols).astype(np.float32 if vt != "f64" else np.float64)
    D = S.dense(A.nrows, A.ncols, rp, c, v)
    if O.INDEX_FORMATS[fmt][1]:
        y = S.spmv_da(A.nrows, A.ncols, rp, idx, v, x)
    else:
        y = S.spmv_csr(A.nrows, A.ncols, rp, idx, v, x)
    assert np.allclose(y, D @ x.astype(np.float64), rtol=0, atol=1e-12)
