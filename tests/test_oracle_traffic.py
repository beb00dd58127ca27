"""Pins of the traffic model against the numbers the paper prints (Example 3,
Fig. 3, the multi-precision remark and the 6/5 target of Sec. 4)."""

from fractions import Fraction

import pytest

from conftest import golden
from oracle import traffic as T

MiB = 2 ** 20


def test_example3_sizes():
    g = golden("example3.json")
    n, nnz = g["n"], g["nnz"]
    m = g["mib_rounded"]
    assert round((n + 1) * 4 / MiB) == m["rowptr_int32"]
    assert round(nnz * 4 / MiB) == m["colids_int32"]
    assert round(nnz * 2 / MiB) == m["colids_int16"]
    assert round(nnz * 8 / MiB) == m["values_f64"]
    assert round(nnz * 4 / MiB) == m["values_f32"]
    assert g["w"] < 2 ** 15


def test_example3_percentages_from_rounded_sizes():
    g = golden("example3.json")
    m = g["mib_rounded"]
    book = 1 - (m["rowptr_int32"] + m["colids_int16"]) / (m["rowptr_int32"] + m["colids_int32"])
    assert round(100 * book, 1) == g["bookkeeping_reduction_pct"]
    f64 = 1 - ((m["rowptr_int32"] + m["colids_int16"] + m["values_f64"])
               / (m["rowptr_int32"] + m["colids_int32"] + m["values_f64"]))
    f32 = 1 - ((m["rowptr_int32"] + m["colids_int16"] + m["values_f32"])
               / (m["rowptr_int32"] + m["colids_int32"] + m["values_f32"]))
    assert round(100 * f64, 1) == g["matrix_reduction_pct_f64"]
    assert round(100 * f32, 1) == g["matrix_reduction_pct_f32"]


def test_example3_with_the_model():
    g = golden("example3.json")
    n, nnz = g["n"], g["nnz"]
    csr = T.matrix_bytes(n, nnz, 4, 4, 8)
    da = T.matrix_bytes(n, nnz, 4, 2, 8)
    assert abs((1 - da / csr) * 100 - g["matrix_reduction_pct_f64"]) < 0.1
    book_csr = T.matrix_bytes(n, nnz, 4, 4, 0)
    book_da = T.matrix_bytes(n, nnz, 4, 2, 0)
    assert round(book_csr / nnz, 2) == g["bytes_per_nnz_int32"]
    assert round(book_da / nnz, 2) == g["bytes_per_nnz_int16"]


def test_example3_row_pointers_ignored():
    g = golden("example3.json")
    r64 = 1 - T.per_nnz_ratio(4, 8, 2, 8)
    r32 = 1 - T.per_nnz_ratio(4, 4, 2, 4)
    assert r64 == Fraction(*g["approx_reduction_f64"])
    assert r32 == Fraction(*g["approx_reduction_f32"])


def test_fig3_grid():
    g = golden("fig3.json")
    sc = list(g["scalars"].values())
    for name, steps in g["scalar_steps"].items():
        ix = g["indices"][name]
        for k, (p, q) in enumerate(steps):
            assert T.per_nnz_ratio(ix, sc[k], ix, sc[k + 1]) == Fraction(p, q), (name, k)
    ix = g["indices"]
    for k, (p, q) in enumerate(g["index_steps"]["int32_to_int16"]):
        assert T.per_nnz_ratio(ix["int32"], sc[k], ix["int16"], sc[k]) == Fraction(p, q)
    for k, (p, q) in enumerate(g["index_steps"]["int16_to_int8"]):
        assert T.per_nnz_ratio(ix["int16"], sc[k], ix["int8"], sc[k]) == Fraction(p, q)


def test_multi_precision_speedups():
    g = golden("fig3.json")["multi_precision_speedups"]
    assert 1 / T.per_nnz_ratio(4, 8, 4, 4) == Fraction(*g["csr_int32"])
    assert 1 / T.per_nnz_ratio(2, 8, 2, 4) == Fraction(*g["da_int16"])
    assert 1 / T.per_nnz_ratio(0, 8, 0, 4) == Fraction(*g["dense"])
    assert 1 / T.per_nnz_ratio(4, 8, 2, 8) == Fraction(*golden("fig3.json")
                                                     ["int32_to_int16_speedup_f64"]["value"])


def test_work_and_uplift_fraction():
    assert T.work_flops(10, 100) == 220
    assert T.work_flops(10, 100, nrhs=3) == 660
    # the abstract's 87.5%: a measured +17.5% against a predicted +20%
    assert T.uplift_fraction(1.175, 1.0, 1.2, 1.0) == pytest.approx(0.875)


def test_spmv_bytes_workloads():
    # 128^3 27-point: n = 2^21, nnz = 382^3
    n, nnz = 128 ** 3, 382 ** 3
    assert T.spmv_bytes(n, n, nnz, 4, 8) == 4 * (n + 1) + 12 * nnz + 16 * n
    assert T.spmv_bytes(n, n, nnz, 2, 8) == 4 * (n + 1) + 10 * nnz + 16 * n
    assert T.spmv_bytes(n, n, nnz, 2, 8, beta_nonzero=True) == 4 * (n + 1) + 10 * nnz + 24 * n
    assert T.spmv_bytes(5, 3, 7, 2, 8, nrhs=4) == 24 + 70 + 96 + 160
