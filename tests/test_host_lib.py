"""Host-side library calls (no GPU): exported symbols, fit check, RCM and
encode bit-exact against the oracle, and error paths."""

import ctypes as C
import os
import re

import numpy as np
import pytest

import paper_2307_06305_amd as D
from conftest import ROOT, golden
from oracle import rcm as OR
from oracle import storage as OS
from workloads import (config_matrix, laplace_2d_5pt, poisson_3d_7pt, random_banded, random_csr,
                       scramble_symmetric, stencil_3d_27pt)


def _header_symbols():
    syms = set()
    for name in os.listdir(os.path.join(ROOT, "include")):
        if name.endswith(".h"):
            text = open(os.path.join(ROOT, "include", name)).read()
            syms |= set(re.findall(r"\b(damn_[a-z0-9_]+)\s*\(", text))
    return syms


def test_library_exports_every_declared_symbol():
    syms = _header_symbols()
    assert "damn_spmv" in syms and "damn_encode" in syms
    lib = C.CDLL(D.library_path())
    missing = [s for s in sorted(syms) if not hasattr(lib, s)]
    assert not missing, missing


def test_status_strings_and_version():
    assert D.version().startswith("damn")
    assert D.status_string(0) == "ok"
    assert "16-bit" in D.status_string(-3)


def _mats():
    yield laplace_2d_5pt(17)
    yield poisson_3d_7pt(5, 6, 7)
    yield stencil_3d_27pt(9, 3)
    yield random_banded(5000, 4, half_band=300)
    for s in range(4):
        yield random_csr(200, 150, s, band=40, dup_frac=0.2, zero_frac=0.1, shuffle_rows=s % 2 == 1)
    yield random_csr(0, 0, 1)
    yield random_csr(5, 0, 1)
    yield random_csr(0, 7, 1)


@pytest.mark.parametrize("A", list(_mats()), ids=lambda A: A.name)
def test_fit_check_matches_oracle(A):
    assert D.fit_check(A.nrows, A.ncols, A.rowptr, A.colids) == OS.fit(A.nrows, A.ncols, A.rowptr,
                                                                       A.colids)


def test_fit_check_example1():
    g = golden("example1.json")
    assert D.fit_check(4, 4, g["rowptr"], g["csr_colids"]) == (1, 1, 1, True)


@pytest.mark.parametrize("d,fits", [(32767, True), (32768, False)])
def test_fit_boundary(d, fits):
    assert D.fit_check(2, d + 1, [0, 1, 1], [d]) == (d, 0, d, fits)


@pytest.mark.parametrize("A", list(_mats()), ids=lambda A: A.name)
def test_encode_natural_matches_oracle_bit_exact(A):
    e = D.encode(A.nrows, A.ncols, A.rowptr, A.colids, A.vals, allow_rcm=False)
    o = OS.encode(A.nrows, A.ncols, A.rowptr, A.colids, A.vals, allow_rcm=False)
    assert not e["permuted"] and e["w"] == o["w"]
    assert np.array_equal(e["rowptr"], o["rowptr"])
    assert np.array_equal(e["off"], o["off"]) and e["off"].dtype == np.int16
    assert np.array_equal(e["vals"].view(np.uint64), o["vals"].view(np.uint64))
    assert np.array_equal(e["perm"], np.arange(A.nrows))


def test_encode_example1():
    g = golden("example1.json")
    e = D.encode(4, 4, g["rowptr"], g["csr_colids"], np.arange(5.0))
    assert e["off"].tolist() == g["da_colids"]


def _rcm_cases():
    yield "example1", 4, np.array([0, 1, 2, 4, 5]), np.array([0, 2, 1, 3, 3])
    for s in range(5):
        A = random_csr(300, 300, s, mean_len=2.0 + s, empty_frac=0.2, dup_frac=0.1)
        yield f"random{s}", 300, A.rowptr, A.colids
    G = scramble_symmetric(laplace_2d_5pt(30), 5)
    yield "grid30", G.nrows, G.rowptr, G.colids
    B = scramble_symmetric(random_banded(40000, 8, half_band=1500), 6)
    yield "banded40k", B.nrows, B.rowptr, B.colids


@pytest.mark.parametrize("case", list(_rcm_cases()), ids=lambda c: c[0])
def test_rcm_matches_oracle_bit_exact(case):
    _, n, rp, c = case
    assert np.array_equal(D.rcm(n, rp, c), OR.rcm(n, rp, c))


def test_encode_permuted_matches_oracle_bit_exact():
    # anti-diagonal plus diagonal: natural bandwidth n-1, RCM brings it to 1
    n = 40000
    rows = np.repeat(np.arange(n), 2)
    cols = np.stack([np.arange(n), np.arange(n)[::-1]], axis=1)
    cols.sort(axis=1)
    cols = cols.ravel()
    rp = np.arange(0, 2 * n + 1, 2, dtype=np.int32)
    vals = np.random.default_rng(0).standard_normal(2 * n)
    e = D.encode(n, n, rp, cols, vals, allow_rcm=True)
    o = OS.encode(n, n, rp, cols, vals, allow_rcm=True)
    assert e["permuted"] and o["permuted"] and e["w"] == o["w"] == 1
    for k in ("rowptr", "off", "perm"):
        assert np.array_equal(e[k], o[k]), k
    assert np.array_equal(e["vals"].view(np.uint64), o["vals"].view(np.uint64))
    del rows


def test_encode_no_fit_reports_bandwidth():
    n = 40000
    rp = np.arange(n + 1, dtype=np.int32)
    c = np.arange(n, dtype=np.int32)[::-1].copy()
    with pytest.raises(D.NoFit) as ei:
        D.encode(n, n, rp, c, np.ones(n), allow_rcm=False)
    assert ei.value.w == n - 1


def test_encode_rectangular_wide_band_no_fit():
    with pytest.raises(D.NoFit):
        D.encode(1, 40001, [0, 1], [40000], [1.0], allow_rcm=True)


@pytest.mark.parametrize("rowptr,colids,code", [
    ([1, 1, 2], [0, 1], -2),
    ([0, 2, 1], [0], -2),
    ([0, 1, 3], [0, 1], -2),
    ([0, 1, 2], [0, 2], -2),
    ([0, 1, 2], [0, -1], -2),
])
def test_bad_csr_status(rowptr, colids, code):
    with pytest.raises(D.DamnError) as ei:
        D.fit_check(2, 2, rowptr, colids)
    assert ei.value.code == code


def test_rcm_rejects_bad_input():
    with pytest.raises(D.DamnError) as ei:
        D.rcm(2, [0, 1, 2], [0, 5])
    assert ei.value.code == -2


def test_null_pointer_status():
    lib = D.lib
    w = C.c_int32()
    st = lib.damn_fit_check(2, 2, None, None, C.byref(w), None, None, None)
    assert st == -1
    assert lib.damn_rcm(3, (C.c_int32 * 4)(0, 0, 0, 0), None, None) == -1


@pytest.mark.slow
def test_rcm_full_size_banded_scrambled_matches_oracle():
    Q = config_matrix(2, scrambled=True)
    assert np.array_equal(D.rcm(Q.nrows, Q.rowptr, Q.colids), OR.rcm(Q.nrows, Q.rowptr, Q.colids))


def test_refine_by_hand_through_the_library():
    # path 0-1-2-3 ordered [1, 0, 3, 2] -> one sweep gives [0, 2, 1, 3], w 2
    rp = [0, 1, 3, 5, 6]
    c = [1, 0, 2, 1, 3, 2]
    perm, w, fits = D.refine_bandwidth(4, rp, c, [1, 0, 3, 2], limit=3)
    assert perm.tolist() == [0, 2, 1, 3] and w == 2 and fits


@pytest.mark.parametrize("limit", [2600, 3000, 100000])
def test_refine_matches_oracle_bit_exact(limit):
    B = scramble_symmetric(random_banded(60000, 9, half_band=2000), 3)
    n = B.nrows
    start = OR.rcm(n, B.rowptr, B.colids)
    p_lib, w_lib, fits = D.refine_bandwidth(n, B.rowptr, B.colids, start, limit=limit)
    p_or, w_or, _ = OR.midpoint_refine(n, B.rowptr, B.colids, start, limit=limit)
    assert np.array_equal(p_lib, p_or) and w_lib == w_or
    assert fits == (w_or < limit)


def test_refine_rejects_non_permutation():
    with pytest.raises(D.DamnError) as ei:
        D.refine_bandwidth(3, [0, 1, 2, 3], [0, 1, 2], [0, 0, 1])
    assert ei.value.code == -1


def test_encode_refined_banded_matches_oracle_bit_exact():
    # a scrambled random band of half-width 20000: RCM alone comes back too
    # wide for int16, the refinement sweeps make it fit
    A = config_matrix(2, scrambled=True, scale=0.05)
    n = A.nrows
    assert D.fit_check(n, n, A.rowptr, A.colids)[0] > 100000
    rcm_w = OS.fit(n, n, *OS.permute_symmetric(n, A.rowptr, A.colids, A.vals,
                                              OR.rcm(n, A.rowptr, A.colids))[:2])[0]
    assert rcm_w >= 32768
    e = D.encode(n, n, A.rowptr, A.colids, A.vals, allow_rcm=True)
    o = OS.encode(n, n, A.rowptr, A.colids, A.vals, allow_rcm=True)
    assert e["permuted"] and e["w"] == o["w"] and e["w"] < 32768
    for k in ("rowptr", "off", "perm"):
        assert np.array_equal(e[k], o[k]), k
    assert np.array_equal(e["vals"].view(np.uint64), o["vals"].view(np.uint64))


@pytest.mark.slow
def test_encode_full_size_banded_scrambled_matches_oracle():
    Q = config_matrix(2, scrambled=True)
    n = Q.nrows
    e = D.encode(n, n, Q.rowptr, Q.colids, Q.vals, allow_rcm=True)
    o = OS.encode(n, n, Q.rowptr, Q.colids, Q.vals, allow_rcm=True)
    assert e["w"] == o["w"] < 32768
    for k in ("rowptr", "off", "perm"):
        assert np.array_equal(e[k], o[k]), k
