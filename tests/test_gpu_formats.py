"""GPU parity of every cell of the storage grid of Fig. 3 (DA offsets of 8
and 16 bits, CSR columns of 16 and 32 bits; float64, float32 and float16
values) against the CPU oracle, through the C ABI, in every launch
configuration; closed forms bit-exact; the calls each format refuses."""

import numpy as np
import pytest

import paper_2307_06305_amd as D
from gpu_util import U32, U64, assert_within, dev, error_bound, host, torch_or_skip
from oracle import spmv as OS
from oracle import storage as OST
from paper_2307_06305_amd.tuning import candidates_for, config_name
from workloads import laplace_2d_5pt, random_banded, random_csr, stencil_3d_27pt, uniform_vector
from workloads.matrices import CSR, stencil_3d_27pt_box

pytestmark = pytest.mark.gpu

FMT = {"da16": D.FORMAT_DA16, "csr32": D.FORMAT_CSR32, "da8": D.FORMAT_DA8,
       "csr16": D.FORMAT_CSR16}
VT = {"f64": D.F64, "f32": D.F32, "f16": D.F16}


def _long_rows():
    # rows longer than every tile cap (up to 4096), within 16-bit columns
    rng = np.random.default_rng(6)
    ncols = 9000
    rl = np.array([0, 5000, 2, 0, 4500, 3, 7] * 3 + [4200], dtype=np.int64)
    rp = np.concatenate([[0], np.cumsum(rl)])
    cols = np.concatenate([np.sort(rng.choice(ncols, size=k, replace=False)) for k in rl])
    return CSR(rl.size, ncols, rp.astype(np.int32), cols.astype(np.int32),
               rng.uniform(-1, 1, int(rp[-1])), "long_rows")


def _matrices():
    yield laplace_2d_5pt(40)                                  # w 40, every format
    yield stencil_3d_27pt(6, 5)                               # w 43
    yield random_banded(20000, 7, half_band=120)              # lognormal rows, w <= 120
    yield random_csr(600, 500, 8, mean_len=7, band=100, empty_frac=0.2, dup_frac=0.1,
                     zero_frac=0.1, shuffle_rows=True)        # tall
    yield random_csr(400, 900, 9, mean_len=9, band=110, empty_frac=0.2, dup_frac=0.1)  # wide
    yield _long_rows()                                        # no DA8 form


MATS = list(_matrices())


def _oracle_form(fmt, vt, A):
    """The oracle's own encoding and rounding, or None if the cell does not fit."""
    try:
        idx = OST.encode_index(fmt, A.nrows, A.ncols, A.rowptr, A.colids)
        vals = OST.store_values(A.vals, vt)
    except OST.NoFit:
        return None
    return idx, vals


def _upload(fmt, vt, A):
    idx, _ = D.encode_index(FMT[fmt], A.nrows, A.ncols, A.rowptr, A.colids)
    return D.Matrix.create_format(FMT[fmt], A.nrows, A.ncols, A.rowptr, idx, A.vals,
                                  store=VT[vt])


def _oracle(fmt, A, idx, vals, x, alpha, beta, y0):
    if OST.INDEX_FORMATS[fmt][1]:
        return OS.spmv_da(A.nrows, A.ncols, A.rowptr, idx, vals, x, alpha, beta, y0)
    return OS.spmv_csr(A.nrows, A.ncols, A.rowptr, idx, vals, x, alpha, beta, y0)


@pytest.mark.parametrize("vt", list(VT))
@pytest.mark.parametrize("fmt", list(FMT))
@pytest.mark.parametrize("A", MATS, ids=lambda A: A.name)
def test_grid_all_configs_match_oracle(A, fmt, vt):
    torch = torch_or_skip()
    print(f"case {A.name} {fmt} {vt}", flush=True)
    form = _oracle_form(fmt, vt, A)
    if form is None:
        with pytest.raises(D.NoFit):
            D.encode_index(FMT[fmt], A.nrows, A.ncols, A.rowptr, A.colids)
        return
    idx, vals = form
    f64 = vt == "f64"
    tdt = torch.float64 if f64 else torch.float32
    x = uniform_vector(A.ncols, 91)
    y0 = uniform_vector(A.nrows, 92)
    if not f64:
        x, y0 = x.astype(np.float32), y0.astype(np.float32)
    M = _upload(fmt, vt, A)
    xd = dev(x, tdt)
    u = U64 if f64 else U32
    cols = OST.da_columns(A.nrows, A.rowptr, idx) if OST.INDEX_FORMATS[fmt][1] else idx
    for alpha, beta in ((1.0, 0.0), (0.5, -2.0)):
        ref = _oracle(fmt, A, idx, vals, x, alpha, beta, y0)
        bnd = error_bound(A.nrows, A.rowptr, cols, vals, x, alpha, beta, y0, u)
        for cfg in candidates_for(M):
            yd = dev(y0, tdt)
            M.set_config(*cfg)
            M.apply(xd, yd, alpha, beta)
            assert_within(host(yd), ref, bnd, f"{A.name} {fmt} {vt} {config_name(cfg)} "
                                              f"alpha={alpha} beta={beta}")
    M.destroy()


@pytest.mark.parametrize("vt", list(VT))
@pytest.mark.parametrize("fmt", list(FMT))
def test_grid_laplacian_closed_form_bit_exact(fmt, vt):
    """4 on the diagonal, -1 off, times x = i^2 + j^2: every product and sum
    is an integer below 2^14, exact in float16 values and float32 sums, so
    every launch gives -4 on interior rows exactly (Sec. 4's product)."""
    torch = torch_or_skip()
    N = 48
    A = laplace_2d_5pt(N)
    i, j = np.meshgrid(np.arange(N), np.arange(N), indexing="xy")
    x = (i.ravel() ** 2 + j.ravel() ** 2).astype(np.float64)
    ref = OS.spmv_csr(A.nrows, A.ncols, A.rowptr, A.colids, A.vals, x)
    interior = ((i > 0) & (i < N - 1) & (j > 0) & (j < N - 1)).ravel()
    assert np.all(ref[interior] == -4.0)
    tdt = torch.float64 if vt == "f64" else torch.float32
    M = _upload(fmt, vt, A)
    xd = dev(x, tdt)
    for cfg in candidates_for(M):
        yd = torch.full((A.nrows,), np.nan, dtype=tdt, device="cuda")
        M.set_config(*cfg)
        M.apply(xd, yd)  # beta = 0: the NaNs in y are not read
        assert np.array_equal(host(yd).astype(np.float64), ref), config_name(cfg)
    M.destroy()


@pytest.mark.parametrize("fmt", list(FMT))
def test_grid_empty_shapes_and_alpha_zero(fmt):
    torch = torch_or_skip()
    for nrows, ncols in ((0, 0), (0, 5), (5, 0), (3, 3)):
        rp = np.zeros(nrows + 1, dtype=np.int32)
        idx = np.zeros(0, dtype=D.FORMATS[FMT[fmt]][0])
        M = D.Matrix.create_format(FMT[fmt], nrows, ncols, rp, idx, np.zeros(0), store=D.F16)
        y = torch.full((nrows,), 3.0, dtype=torch.float32, device="cuda")
        x = torch.ones(ncols, dtype=torch.float32, device="cuda")
        M.apply(x, y, 1.0, 0.5)
        assert np.all(host(y) == 1.5)
        M.destroy()
    A = laplace_2d_5pt(8)
    M = _upload(fmt, "f16", A)
    y = torch.full((A.nrows,), 2.0, dtype=torch.float32, device="cuda")
    M.apply(torch.full((A.ncols,), np.nan, dtype=torch.float32, device="cuda"), y, 0.0, -1.0)
    assert np.all(host(y) == -2.0)  # alpha = 0 reads neither A nor x
    M.destroy()


def test_grid_refused_calls():
    torch = torch_or_skip()
    A = laplace_2d_5pt(10)
    x = torch.ones(A.ncols, dtype=torch.float32, device="cuda")
    y = torch.zeros(A.nrows, dtype=torch.float32, device="cuda")
    M8 = _upload("da8", "f32", A)
    C16 = _upload("csr16", "f32", A)
    with pytest.raises(D.DamnError) as e:
        M8.csr_spmv(x, y)
    assert e.value.code == -1
    with pytest.raises(D.DamnError) as e:
        C16.spmv(x, y)
    assert e.value.code == -1
    M64 = _upload("da8", "f64", A)
    X = torch.ones(A.ncols, 2, dtype=torch.float64, device="cuda")
    Y = torch.zeros(A.nrows, 2, dtype=torch.float64, device="cuda")
    with pytest.raises(D.DamnError) as e:
        M64.spmm(X, Y)
    assert e.value.code == -6
    b = torch.ones(A.nrows, dtype=torch.float64, device="cuda")
    with pytest.raises(D.DamnError) as e:
        D.cg(M64, b, torch.zeros_like(b))
    assert e.value.code == -6
    for M in (M8, C16, M64):
        M.destroy()


def test_grid_value_overflow_refused_at_upload():
    torch_or_skip()
    A = laplace_2d_5pt(4)
    vals = A.vals.copy()
    vals[3] = 1e5
    idx, _ = D.encode_index(D.FORMAT_DA16, A.nrows, A.ncols, A.rowptr, A.colids)
    with pytest.raises(D.DamnError) as e:
        D.Matrix.create_format(D.FORMAT_DA16, A.nrows, A.ncols, A.rowptr, idx, vals, store=D.F16)
    assert e.value.code == -3


@pytest.mark.timeout(600)
@pytest.mark.parametrize("fmt,vt", [("da8", "f64"), ("da8", "f32"), ("da8", "f16"),
                                    ("da16", "f16"), ("csr32", "f16")])
def test_grid_full_size_box_every_row(fmt, vt):
    """The 27-point stencil on the 10 x 10 x 20972 box (n 2,097,200, w 111),
    the workload the grid is measured on: every row of y against the
    oracle's full product on the same rounded values, in every
    configuration; y starts as NaN before each product."""
    torch = torch_or_skip()
    A = stencil_3d_27pt_box(10, 10, 20972, 1009)
    sv = OST.store_values(A.vals, vt)
    f64 = vt == "f64"
    x = uniform_vector(A.ncols, 2009)
    if not f64:
        x = x.astype(np.float32)
    ref = OS.spmv_csr(A.nrows, A.ncols, A.rowptr, A.colids, sv, x)
    bnd = error_bound(A.nrows, A.rowptr, A.colids, sv, x, 1.0, 0.0, None, U64 if f64 else U32)
    M = _upload(fmt, vt, A)
    tdt = torch.float64 if f64 else torch.float32
    xd = dev(x, tdt)
    yd = torch.empty(A.nrows, dtype=tdt, device="cuda")
    for cfg in candidates_for(M):
        print(f"case box {fmt} {vt} {config_name(cfg)}", flush=True)
        yd.fill_(float("nan"))
        M.set_config(*cfg)
        M.apply(xd, yd)
        assert_within(host(yd), ref, bnd, f"{fmt} {vt} {config_name(cfg)}")
    M.destroy()
