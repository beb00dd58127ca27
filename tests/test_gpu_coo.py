"""GPU parity of the DA-COO and COO products (diagonal addressing applied to
one index vector of COO, Sec. 1) against the CPU oracle, through the C ABI:
rows cut by chunk edges, rows running through several chunks, empty rows
(also long runs of them before, between and after the rows with entries),
both scalar types; a closed form bit-exact."""

import numpy as np
import pytest

import paper_2307_06305_amd as D
from gpu_util import U32, U64, assert_within, dev, error_bound, host, torch_or_skip
from oracle import coo as OC
from oracle import storage as OST
from workloads import laplace_2d_5pt, random_banded, random_csr, stencil_3d_27pt, uniform_vector
from workloads.matrices import CSR


def _runs():
    # rows of 1..7000 entries: some end exactly on a 2048-entry chunk edge,
    # some run through several chunks, empty rows between
    rng = np.random.default_rng(3)
    rl = np.array([2048, 0, 2048, 5000, 1, 0, 7000, 3, 2047, 1, 4096, 0, 17, 6000, 2, 0],
                  dtype=np.int64)
    ncols = 9000
    rp = np.concatenate([[0], np.cumsum(rl)])
    cols = np.concatenate([np.sort(rng.choice(ncols, size=k, replace=False)) for k in rl])
    return CSR(rl.size, ncols, rp.astype(np.int32), cols.astype(np.int32),
               rng.uniform(-1, 1, int(rp[-1])), "long_runs")


def _gaps():
    # long runs of empty rows before, between and after the rows with
    # entries (rows without entries get beta*y from the chunk that follows
    # them, or from the last chunk), rows of 1023..1025 entries next to the
    # 1024-entry chunk edges
    rng = np.random.default_rng(4)
    nrows, ncols = 20000, 30000
    rl = np.zeros(nrows, dtype=np.int64)
    rl[3000:3100] = rng.integers(0, 60, 100)
    rl[9000:9003] = [1023, 1024, 1025]
    rl[15000:15050] = rng.integers(1, 40, 50)
    rp = np.concatenate([[0], np.cumsum(rl)])
    cols = np.concatenate([np.sort(rng.choice(np.arange(max(0, r - 20000), min(ncols, r + 20000)),
                                              size=int(k), replace=False))
                           for r, k in enumerate(rl) if k])
    return CSR(nrows, ncols, rp.astype(np.int32), cols.astype(np.int32),
               rng.uniform(-1, 1, int(rp[-1])), "empty_gaps")


CASES = [laplace_2d_5pt(30), stencil_3d_27pt(12, 4), random_banded(30000, 6, half_band=2000),
         random_csr(900, 600, 7, mean_len=6, empty_frac=0.4, dup_frac=0.2, zero_frac=0.1,
                    shuffle_rows=True),
         random_csr(300, 800, 8, mean_len=9, band=400), _runs(), _gaps()]

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("store", ["f64", "f32"])
@pytest.mark.parametrize("fmt", [D.FORMAT_DACOO16, D.FORMAT_COO32])
@pytest.mark.parametrize("A", CASES, ids=lambda A: A.name)
def test_coo_matches_oracle(A, fmt, store):
    torch = torch_or_skip()
    print(f"case {A.name} {fmt} {store}", flush=True)
    da = fmt == D.FORMAT_DACOO16
    rows, idx = D.coo_encode(A.nrows, A.ncols, A.rowptr, A.colids, fmt)
    f64 = store == "f64"
    vals = A.vals if f64 else OST.store_values(A.vals, "f32")
    M = D.Matrix.coo_create(fmt, A.nrows, A.ncols, rows, idx, A.vals,
                            store=D.F64 if f64 else D.F32)
    tdt = torch.float64 if f64 else torch.float32
    x = uniform_vector(A.ncols, 41)
    y0 = uniform_vector(A.nrows, 42)
    if not f64:
        x, y0 = x.astype(np.float32), y0.astype(np.float32)
    xd = dev(x, tdt)
    for alpha, beta in ((1.0, 0.0), (0.75, -1.25), (0.0, 2.0)):
        ref = OC.spmv_coo(A.nrows, A.ncols, rows, idx, vals, x, alpha, beta, y0, da)
        bnd = error_bound(A.nrows, A.rowptr, A.colids, vals, x, alpha, beta, y0,
                          U64 if f64 else U32)
        yd = dev(y0, tdt)
        M.apply(xd, yd, alpha, beta)
        assert_within(host(yd), ref, bnd, f"{A.name} {fmt} {store} alpha={alpha} beta={beta}")
    # the result does not depend on scheduling: two runs agree bit for bit
    y1 = dev(y0, tdt)
    y2 = dev(y0, tdt)
    M.apply(xd, y1, 1.0, 0.5)
    M.apply(xd, y2, 1.0, 0.5)
    assert np.array_equal(host(y1), host(y2))
    M.destroy()


def test_coo_laplacian_closed_form_and_nan_y():
    torch = torch_or_skip()
    N = 40
    A = laplace_2d_5pt(N)
    i, j = np.meshgrid(np.arange(N), np.arange(N), indexing="xy")
    x = (i.ravel() ** 2 + j.ravel() ** 2).astype(np.float64)
    rows, off = D.coo_encode(A.nrows, A.ncols, A.rowptr, A.colids)
    ref = OC.spmv_coo(A.nrows, A.ncols, rows, off, A.vals, x)
    M = D.Matrix.coo_create(D.FORMAT_DACOO16, A.nrows, A.ncols, rows, off, A.vals)
    y = torch.full((A.nrows,), np.nan, dtype=torch.float64, device="cuda")
    M.spmv(dev(x), y)  # beta = 0 does not read the NaNs
    assert np.array_equal(host(y), ref)
    M.destroy()


def test_coo_empty_and_refused():
    torch = torch_or_skip()
    M = D.Matrix.coo_create(D.FORMAT_DACOO16, 5, 4, np.zeros(0, np.int32), np.zeros(0, np.int16),
                            np.zeros(0))
    y = torch.full((5,), 3.0, dtype=torch.float64, device="cuda")
    M.spmv(torch.ones(4, dtype=torch.float64, device="cuda"), y, 1.0, 2.0)
    assert np.all(host(y) == 6.0)
    with pytest.raises(D.DamnError) as e:
        M.csr_spmv(torch.ones(4, dtype=torch.float64, device="cuda"), y)
    assert e.value.code == -1
    X = torch.ones(4, 2, dtype=torch.float64, device="cuda")
    Y = torch.zeros(5, 2, dtype=torch.float64, device="cuda")
    with pytest.raises(D.DamnError) as e:
        M.spmm(X, Y)
    assert e.value.code == -6
    M.destroy()
