"""The native CPU baseline (OpenMP DA-CSR / CSR SpMV, used by the benchmark
for comparison only) against the oracle, within the rounding bound of the
GPU parity tests; thread counts do not change its result."""

import numpy as np
import pytest

from gpu_util import U64, assert_within, error_bound
from oracle import spmv as OS
from oracle import storage as OST
from paper_2307_06305_amd import cpu
from workloads import laplace_2d_5pt, random_banded, random_csr, stencil_3d_27pt


@pytest.mark.parametrize("A", [laplace_2d_5pt(30), stencil_3d_27pt(14, 2),
                               random_banded(20000, 3, half_band=500),
                               random_csr(500, 400, 4, mean_len=7, empty_frac=0.3, dup_frac=0.2,
                                          shuffle_rows=True)], ids=lambda A: A.name)
def test_cpu_baseline_matches_oracle(A):
    x = np.random.default_rng(1).uniform(-1, 1, A.ncols)
    ref = OS.spmv_csr(A.nrows, A.ncols, A.rowptr, A.colids, A.vals, x)
    bnd = error_bound(A.nrows, A.rowptr, A.colids, A.vals, x, 1.0, 0.0, None, U64)
    off = OST.encode_index("da16", A.nrows, A.ncols, A.rowptr, A.colids)
    outs = []
    for threads in (1, 4):
        rp, o, v, xx = cpu.arrays(A.rowptr, off, A.vals, x, np.int16)
        y = np.full(A.nrows, np.nan)
        cpu.spmv_da(A.nrows, rp, o, v, xx, y, threads)
        assert_within(y, ref, bnd, f"da {threads}")
        rp, c, v, xx = cpu.arrays(A.rowptr, A.colids, A.vals, x, np.int32)
        yc = np.full(A.nrows, np.nan)
        cpu.spmv_csr(A.nrows, rp, c, v, xx, yc, threads)
        assert_within(yc, ref, bnd, f"csr {threads}")
        outs.append((y, yc))
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])
