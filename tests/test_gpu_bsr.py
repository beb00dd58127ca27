"""GPU parity of the DA-BSR and BSR products (diagonal addressing applied to
block storage, Sec. 1) against the CPU oracle, through the C ABI: every
block size, scalar type and launch configuration; a closed form bit-exact;
the calls block handles refuse."""

import numpy as np
import pytest

import paper_2307_06305_amd as D
from gpu_util import U32, U64, assert_within, dev, error_bound, host, torch_or_skip
from oracle import blocks as OB
from oracle import storage as OST
from paper_2307_06305_amd.tuning import candidates_for, config_name
from workloads import laplace_2d_5pt, random_csr, uniform_vector
from workloads.matrices import CSR, block_stencil_27pt

pytestmark = pytest.mark.gpu


def _long_block_rows(b):
    # a block row with far more blocks than any tile holds, among short ones
    rng = np.random.default_rng(b)
    nbc = 3000
    rl = np.array([0, 2500, 3, 1, 0, 1800, 2], dtype=np.int64)
    rows, cols = [], []
    for br, k in enumerate(rl):
        for bc in np.sort(rng.choice(nbc, size=k, replace=False)):
            i, j = rng.integers(0, b, 2)
            rows.append(br * b + i)
            cols.append(bc * b + j)
    rows, cols = np.array(rows), np.array(cols)
    order = np.lexsort((cols, rows))
    rows, cols = rows[order], cols[order]
    n = rl.size * b
    rp = np.concatenate([[0], np.cumsum(np.bincount(rows, minlength=n))])
    return CSR(n, nbc * b, rp.astype(np.int32), cols.astype(np.int32),
               rng.uniform(-1, 1, rows.size), f"long_block_rows_b{b}")


def _cases():
    for b in (2, 3, 4, 6):
        yield b, block_stencil_27pt(5, b, 3)
        yield b, random_csr(60 * b, 40 * b, b, mean_len=5, dup_frac=0.2, zero_frac=0.1,
                            empty_frac=0.3)                         # tall, empty block rows
        yield b, random_csr(30 * b, 70 * b, 10 + b, mean_len=7, band=50 * b)  # wide
        yield b, _long_block_rows(b)


CASES = list(_cases())


def _scalar_form(nbr, b, brp, bcols, bvals):
    """The blocks as scalar CSR (every stored block value an entry), for the
    rounding-error bound."""
    nnzb = len(bcols)
    br = OST.entry_rows(nbr, brp)
    rows = (br[:, None, None] * b + np.arange(b)[None, :, None] + 0 * np.arange(b)).ravel()
    cols = (bcols[:, None, None] * b + np.arange(b)[None, None, :] + 0 * np.arange(b)[:, None]
            ).ravel()
    order = np.lexsort((np.repeat(np.arange(nnzb), b * b), rows))
    rp = np.concatenate([[0], np.cumsum(np.bincount(rows, minlength=nbr * b))]).astype(np.int32)
    return rp, cols[order], np.asarray(bvals, dtype=np.float64).ravel()[order]


@pytest.mark.parametrize("store", ["f64", "f32"])
@pytest.mark.parametrize("fmt", [D.FORMAT_DABSR16, D.FORMAT_BSR32])
@pytest.mark.parametrize("b,A", CASES, ids=[f"b{b}-{A.name}" for b, A in CASES])
def test_bsr_all_configs_match_oracle(b, A, fmt, store):
    torch = torch_or_skip()
    print(f"case {A.name} b={b} fmt={fmt} {store}", flush=True)
    brp, bcols, bvals = OB.bsr_from_csr(A.nrows, A.ncols, A.rowptr, A.colids, A.vals, b)
    nbr, nbc = A.nrows // b, A.ncols // b
    f64 = store == "f64"
    bv = bvals if f64 else OST.store_values(bvals, "f32")
    e = D.bsr_encode(A.nrows, A.ncols, A.rowptr, A.colids, A.vals, b, fmt)
    M = D.Matrix.bsr_create(fmt, nbr, nbc, b, e["browptr"], e["bidx"], e["bvals"],
                            store=D.F64 if f64 else D.F32)
    tdt = torch.float64 if f64 else torch.float32
    x = uniform_vector(A.ncols, 31)
    y0 = uniform_vector(A.nrows, 32)
    if not f64:
        x, y0 = x.astype(np.float32), y0.astype(np.float32)
    xd = dev(x, tdt)
    srp, scols, svals = _scalar_form(nbr, b, brp, bcols, bv)
    for alpha, beta in ((1.0, 0.0), (-1.5, 0.25)):
        ref = OB.spmv_bsr(nbr, nbc, b, brp, bcols, bv, x, alpha, beta, y0, da=False)
        bnd = error_bound(A.nrows, srp, scols, svals, x, alpha, beta, y0, U64 if f64 else U32)
        for cfg in candidates_for(M):
            yd = dev(y0, tdt)
            M.set_config(*cfg)
            M.apply(xd, yd, alpha, beta)
            assert_within(host(yd), ref, bnd, f"{A.name} b={b} {fmt} {store} "
                                              f"{config_name(cfg)} alpha={alpha} beta={beta}")
    M.destroy()


@pytest.mark.parametrize("b", [2, 3, 4, 6])
def test_bsr_kronecker_laplacian_closed_form(b):
    """(2D Laplacian (x) I_b) times kron(i^2 + j^2, 1): -4 on every interior
    component, exactly, in every configuration and both scalar types."""
    torch = torch_or_skip()
    N = 20
    A = laplace_2d_5pt(N)
    nbr = A.nrows
    bvals = A.vals[:, None, None] * np.eye(b)[None]
    off, _ = D.encode_index(D.FORMAT_DA16, A.nrows, A.ncols, A.rowptr, A.colids)
    i, j = np.meshgrid(np.arange(N), np.arange(N), indexing="xy")
    x = np.repeat((i.ravel() ** 2 + j.ravel() ** 2).astype(float), b)
    ref = OB.spmv_bsr(nbr, nbr, b, A.rowptr, off, bvals, x)
    interior = np.repeat(((i > 0) & (i < N - 1) & (j > 0) & (j < N - 1)).ravel(), b)
    assert np.all(ref[interior] == -4.0)
    for store, tdt in ((D.F64, torch.float64), (D.F32, torch.float32)):
        M = D.Matrix.bsr_create(D.FORMAT_DABSR16, nbr, nbr, b, A.rowptr, off, bvals, store=store)
        xd = dev(x, tdt)
        for cfg in candidates_for(M):
            yd = torch.full((nbr * b,), np.nan, dtype=tdt, device="cuda")
            M.set_config(*cfg)
            M.apply(xd, yd)
            assert np.array_equal(host(yd).astype(np.float64), ref), config_name(cfg)
        M.destroy()


def test_bsr_refused_calls_and_alpha_zero():
    torch = torch_or_skip()
    A = block_stencil_27pt(3, 2, 1)
    e = D.bsr_encode(A.nrows, A.ncols, A.rowptr, A.colids, A.vals, 2)
    M = D.Matrix.bsr_create(D.FORMAT_DABSR16, A.nrows // 2, A.ncols // 2, 2, e["browptr"],
                            e["bidx"], e["bvals"])
    x = torch.ones(A.ncols, dtype=torch.float64, device="cuda")
    y = torch.full((A.nrows,), 4.0, dtype=torch.float64, device="cuda")
    with pytest.raises(D.DamnError) as err:
        M.csr_spmv(x, y)
    assert err.value.code == -1
    X = torch.ones(A.ncols, 2, dtype=torch.float64, device="cuda")
    Y = torch.zeros(A.nrows, 2, dtype=torch.float64, device="cuda")
    with pytest.raises(D.DamnError) as err:
        M.spmm(X, Y)
    assert err.value.code == -6
    with pytest.raises(D.DamnError) as err:
        D.cg(M, x, torch.zeros_like(x))
    assert err.value.code == -6
    with pytest.raises(D.DamnError):
        D.Batch([M], [X[:, :1].contiguous()], [Y[:, :1].contiguous()], 1.0, 0.0)
    M.spmv(torch.full((A.ncols,), np.nan, dtype=torch.float64, device="cuda"), y, 0.0, 0.5)
    assert np.all(host(y) == 2.0)
    M.destroy()


@pytest.mark.timeout(600)
@pytest.mark.parametrize("fmt", [D.FORMAT_DABSR16, D.FORMAT_BSR32])
def test_bsr_full_size_every_row(fmt):
    """The block workload the bench measures (3 x 3 blocks on the 27-point
    pattern of a 64^3 node grid, 786,432 rows): every row of y against the
    oracle's full product, in every configuration; y starts as NaN."""
    torch = torch_or_skip()
    b = 3
    A = block_stencil_27pt(64, b, 1010)
    e = D.bsr_encode(A.nrows, A.ncols, A.rowptr, A.colids, A.vals, b, fmt)
    nbr = A.nrows // b
    M = D.Matrix.bsr_create(fmt, nbr, nbr, b, e["browptr"], e["bidx"], e["bvals"])
    x = uniform_vector(A.ncols, 2010)
    from oracle import spmv as OS
    ref = OS.spmv_csr(A.nrows, A.ncols, A.rowptr, A.colids, A.vals, x)
    bnd = error_bound(A.nrows, A.rowptr, A.colids, A.vals, x, 1.0, 0.0, None, U64)
    xd = dev(x)
    yd = torch.empty(A.nrows, dtype=torch.float64, device="cuda")
    for cfg in candidates_for(M):
        print(f"case block3 {fmt} {config_name(cfg)}", flush=True)
        yd.fill_(float("nan"))
        M.set_config(*cfg)
        M.apply(xd, yd)
        assert_within(host(yd), ref, bnd, config_name(cfg))
    M.destroy()
