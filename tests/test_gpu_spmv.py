"""GPU parity of the HIP SpMV / SpMM kernels against the CPU oracle, through
the C ABI.  Every launch configuration the library accepts is checked."""

import numpy as np
import pytest

import paper_2307_06305_amd as D
from gpu_util import U32, U64, assert_within, dev, error_bound, host, torch_or_skip
from oracle import spmv as OS
from oracle import storage as OST
from paper_2307_06305_amd.tuning import candidates_for, config_name
from workloads import (config_matrix, laplace_2d_5pt, poisson_3d_7pt, random_banded, random_csr,
                       stencil_3d_27pt, uniform_vector)

pytestmark = pytest.mark.gpu


def _long_rows():
    # rows far longer than any tile cap, mixed with empty and short rows
    rng = np.random.default_rng(5)
    ncols = 9000
    rl = np.array([0, 5000, 1, 0, 7000, 3] * 6 + [4100, 0], dtype=np.int64)
    nrows = rl.size
    rp = np.zeros(nrows + 1, dtype=np.int64)
    np.cumsum(rl, out=rp[1:])
    cols = np.concatenate([np.sort(rng.choice(ncols, size=k, replace=False)) for k in rl])
    from workloads.matrices import CSR
    return CSR(nrows, ncols, rp.astype(np.int32), cols.astype(np.int32),
               rng.uniform(-1, 1, int(rp[-1])), "long_rows")


def _matrices():
    yield config_matrix(0)                                   # 2D 5-point 64x64
    yield stencil_3d_27pt(20, 11)                            # 27-point, 8000 rows
    yield random_banded(30000, 12, half_band=3000)           # lognormal rows
    yield random_csr(700, 300, 3, mean_len=6, band=250, empty_frac=0.2, dup_frac=0.1,
                     zero_frac=0.1, shuffle_rows=True)        # tall
    yield random_csr(300, 700, 4, mean_len=9, band=500, empty_frac=0.2, dup_frac=0.1)  # wide
    yield _long_rows()


MATS = list(_matrices())


def _encode(A):
    e = D.encode(A.nrows, A.ncols, A.rowptr, A.colids, A.vals, allow_rcm=False)
    return e


@pytest.mark.parametrize("fmt", ["da", "csr"])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("A", MATS, ids=lambda A: A.name)
def test_spmv_all_configs_match_oracle(A, dtype, fmt):
    torch = torch_or_skip()
    print(f"case {A.name} {dtype} {fmt}", flush=True)
    f32 = dtype == "f32"
    vals = A.vals.astype(np.float32) if f32 else A.vals
    x = uniform_vector(A.ncols, 77)
    y0 = uniform_vector(A.nrows, 78)
    if f32:
        x, y0 = x.astype(np.float32), y0.astype(np.float32)
    store = D.F32 if f32 else D.F64
    if fmt == "da":
        e = _encode(A)
        M = D.Matrix.create(A.nrows, A.ncols, e["rowptr"], e["off"], vals, store=store)
    else:
        M = D.Matrix.csr_create(A.nrows, A.ncols, A.rowptr, A.colids, vals, store=store)
    tdt = torch.float32 if f32 else torch.float64
    xd = dev(x, tdt)
    u = U32 if f32 else U64
    for alpha, beta in ((1.0, 0.0), (-0.75, 1.5)):
        ref = OS.spmv_csr(A.nrows, A.ncols, A.rowptr, A.colids, vals, x, alpha, beta, y0)
        bnd = error_bound(A.nrows, A.rowptr, A.colids, vals, x, alpha, beta, y0, u)
        for cfg in candidates_for(M):
            yd = dev(y0, tdt)
            M.set_config(*cfg)
            M.apply(xd, yd, alpha, beta)
            assert_within(host(yd), ref, bnd, f"{A.name} {fmt} {dtype} {config_name(cfg)} "
                                              f"alpha={alpha} beta={beta}")
    M.destroy()


def _grid_quadratic(shape):
    idx = np.indices(shape[::-1])[::-1]  # x fastest
    return sum(a.astype(np.float64) ** 2 for a in idx).ravel(), idx


def _ghost_sum(shape, idx):
    """Sum over missing (off-grid) neighbours of the quadratic's values."""
    out = np.zeros(int(np.prod(shape)))
    for axis, n in enumerate(shape):
        for step in (-1, 1):
            coords = [a.ravel().astype(np.float64) for a in idx]
            c = coords[axis] + step
            missing = (c < 0) | (c >= n)
            coords[axis] = c
            val = sum(v ** 2 for v in coords)
            out += np.where(missing, val, 0.0)
    return out


@pytest.mark.parametrize("fmt", ["da", "csr"])
def test_laplace_2d_closed_forms_bit_exact(fmt):
    torch = torch_or_skip()
    N = 64
    A = laplace_2d_5pt(N)
    e = _encode(A)
    M = (D.Matrix.create(A.nrows, A.ncols, e["rowptr"], e["off"], A.vals) if fmt == "da"
         else D.Matrix.csr_create(A.nrows, A.ncols, A.rowptr, A.colids, A.vals))
    # stencil times ones = row sums: 0 inside, 1 on edges, 2 in corners
    idx = np.indices((N, N))[::-1]
    on_edge = (idx[0] == 0).astype(int) + (idx[0] == N - 1) + (idx[1] == 0) + (idx[1] == N - 1)
    expect_ones = on_edge.ravel().astype(np.float64)
    f, idx2 = _grid_quadratic((N, N))
    expect_quad = -4.0 + _ghost_sum((N, N), idx2)
    for cfg in candidates_for(M):
        M.set_config(*cfg)
        for vec, expect in ((np.ones(N * N), expect_ones), (f, expect_quad)):
            yd = dev(np.zeros(N * N))
            M.apply(dev(vec), yd)
            assert np.array_equal(host(yd), expect), config_name(cfg)
    M.destroy()


@pytest.mark.parametrize("fmt", ["da", "csr"])
def test_poisson_3d_quadratic_bit_exact(fmt):
    torch = torch_or_skip()
    shape = (12, 10, 14)
    A = poisson_3d_7pt(*shape)
    e = _encode(A)
    M = (D.Matrix.create(A.nrows, A.ncols, e["rowptr"], e["off"], A.vals) if fmt == "da"
         else D.Matrix.csr_create(A.nrows, A.ncols, A.rowptr, A.colids, A.vals))
    f, idx = _grid_quadratic(shape)
    expect = -6.0 + _ghost_sum(shape, idx)
    for cfg in candidates_for(M):
        M.set_config(*cfg)
        yd = dev(np.zeros(A.nrows))
        M.apply(dev(f), yd)
        assert np.array_equal(host(yd), expect), config_name(cfg)
    M.destroy()


def test_beta_zero_ignores_nan_and_alpha_zero_scales():
    torch = torch_or_skip()
    A = stencil_3d_27pt(8, 2)
    e = _encode(A)
    M = D.Matrix.create(A.nrows, A.ncols, e["rowptr"], e["off"], A.vals)
    x = uniform_vector(A.ncols, 1)
    ref = OS.spmv_csr(A.nrows, A.ncols, A.rowptr, A.colids, A.vals, x)
    bnd = error_bound(A.nrows, A.rowptr, A.colids, A.vals, x, 1.0, 0.0, None, U64)
    y0 = uniform_vector(A.nrows, 2)
    for cfg in candidates_for(M):
        M.set_config(*cfg)
        yd = dev(np.full(A.nrows, np.nan))
        M.spmv(dev(x), yd, 1.0, 0.0)
        assert_within(host(yd), ref, bnd, config_name(cfg))
        # alpha = 0: y <- beta*y exactly, x not read (NaN x is harmless)
        yd = dev(y0)
        M.spmv(dev(np.full(A.ncols, np.nan)), yd, 0.0, 2.0)
        assert np.array_equal(host(yd), 2.0 * y0)
        yd = dev(y0)
        M.spmv(dev(x), yd, 0.0, 0.0)
        assert np.array_equal(host(yd), np.zeros(A.nrows))
    M.destroy()


def test_empty_shapes():
    torch = torch_or_skip()
    # nnz = 0 with rows: y = beta*y0 exactly; zero rows: nothing to do
    for nrows, ncols in ((50, 20), (0, 10), (10, 0)):
        rp = np.zeros(nrows + 1, dtype=np.int32)
        M = D.Matrix.create(nrows, ncols, rp, np.zeros(0, np.int16), np.zeros(0))
        C = D.Matrix.csr_create(nrows, ncols, rp, np.zeros(0, np.int32), np.zeros(0))
        y0 = uniform_vector(nrows, 3)
        for cfg in candidates_for(M):
            for mat in (M, C):
                mat.set_config(*cfg)
                yd = dev(y0)
                mat.apply(dev(np.ones(ncols)), yd, 1.0, 0.5)
                assert np.array_equal(host(yd), 0.5 * y0)
        M.destroy()
        C.destroy()


def _runs_matrix(ncols, seed):
    """Rows of runs of neighbouring columns, for the paired gathers: runs of
    every length 1..70 starting at column 0, at column 1, ending at the last
    column and at a random column; rows of short runs with gaps; single
    entries at the first and last columns; a pair ending at the last
    column; empty rows.  Columns stay within 32767 of the row (DA16)."""
    from workloads.matrices import CSR
    rng = np.random.default_rng(seed)
    rows = []
    for L in range(1, min(71, ncols + 1)):
        for start in {0, min(1, ncols - L), ncols - L, int(rng.integers(0, ncols - L + 1))}:
            rows.append(np.arange(start, start + L))
    for _ in range(200):
        starts = rng.integers(0, max(ncols - 4, 1), int(rng.integers(1, 12)))
        c = np.concatenate([np.arange(a, a + int(rng.integers(1, 5))) for a in starts])
        rows.append(np.unique(c[c < ncols]))
    rows += [np.array([0]), np.array([ncols - 1]), np.array([], dtype=np.int64)]
    if ncols >= 2:
        rows.append(np.array([ncols - 2, ncols - 1]))
    order = rng.permutation(len(rows))
    rows = [rows[i] for i in order]
    rl = np.array([r.size for r in rows], dtype=np.int64)
    rp = np.zeros(len(rows) + 1, dtype=np.int64)
    np.cumsum(rl, out=rp[1:])
    cols = np.concatenate(rows).astype(np.int32)
    return CSR(len(rows), ncols, rp.astype(np.int32), cols, rng.uniform(-1, 1, cols.size),
               f"runs_{ncols}")


@pytest.mark.parametrize("ncols", [600, 2, 1])
def test_paired_gathers_on_runs_and_edges(ncols):
    """Paired gathers (stream unroll 2) against the oracle on rows made of
    runs, including the last column (the load address is clamped there) and
    matrices with two columns and one column (which take the interleaved
    kernel), for every lane count and tile, DA16 and CSR32, float64 and
    float32 (Sec. 4's product)."""
    torch = torch_or_skip()
    A = _runs_matrix(ncols, 31 + ncols)
    e = _encode(A)
    for f32 in (False, True):
        vals = A.vals.astype(np.float32) if f32 else A.vals
        x = uniform_vector(A.ncols, 79)
        y0 = uniform_vector(A.nrows, 80)
        if f32:
            x, y0 = x.astype(np.float32), y0.astype(np.float32)
        store, tdt, u = (D.F32, torch.float32, U32) if f32 else (D.F64, torch.float64, U64)
        for fmt in ("da", "csr"):
            M = (D.Matrix.create(A.nrows, A.ncols, e["rowptr"], e["off"], vals, store=store)
                 if fmt == "da" else
                 D.Matrix.csr_create(A.nrows, A.ncols, A.rowptr, A.colids, vals, store=store))
            xd = dev(x, tdt)
            for alpha, beta in ((1.0, 0.0), (-0.5, 2.0)):
                ref = OS.spmv_csr(A.nrows, A.ncols, A.rowptr, A.colids, vals, x, alpha, beta, y0)
                bnd = error_bound(A.nrows, A.rowptr, A.colids, vals, x, alpha, beta, y0, u)
                for cfg in [c for c in candidates_for(M) if c[0] == D.VAR_STREAM and c[2] == 2]:
                    M.set_config(*cfg)
                    yd = dev(y0, tdt)
                    M.apply(xd, yd, alpha, beta)
                    assert_within(host(yd), ref, bnd, f"{A.name} {fmt} f32={f32} "
                                                      f"{config_name(cfg)} alpha={alpha}")
            M.destroy()


def test_paired_gathers_ignore_values_they_do_not_use():
    """A paired load also brings x[c + 1] (or x[c - 1] at the last column);
    where that column is not in the row its value is not used: infinities
    and NaNs there leave y finite and equal to the oracle's product."""
    torch = torch_or_skip()
    from workloads.matrices import CSR
    rng = np.random.default_rng(41)
    ncols = 401                      # the last column, 400, is even
    rows = [np.sort(rng.choice(np.arange(0, ncols, 2), size=int(rng.integers(0, 30)),
                               replace=False)) for _ in range(300)]
    rows.append(np.array([ncols - 1]))
    rl = np.array([r.size for r in rows])
    rp = np.concatenate([[0], np.cumsum(rl)]).astype(np.int32)
    A = CSR(len(rows), ncols, rp, np.concatenate(rows).astype(np.int32),
            rng.uniform(-1, 1, int(rp[-1])), "even_columns")
    x = uniform_vector(ncols, 81)
    ref = OS.spmv_csr(A.nrows, A.ncols, A.rowptr, A.colids, A.vals, x)
    bnd = error_bound(A.nrows, A.rowptr, A.colids, A.vals, x, 1.0, 0.0, None, U64)
    x[1::4] = np.inf                 # odd columns: never in a row
    x[3::4] = np.nan
    e = _encode(A)
    for M in (D.Matrix.create(A.nrows, A.ncols, e["rowptr"], e["off"], A.vals),
              D.Matrix.csr_create(A.nrows, A.ncols, A.rowptr, A.colids, A.vals)):
        for cfg in [c for c in candidates_for(M) if c[0] == D.VAR_STREAM and c[2] == 2]:
            M.set_config(*cfg)
            yd = dev(np.full(A.nrows, np.nan))
            M.apply(dev(x), yd)
            assert_within(host(yd), ref, bnd, config_name(cfg))
        M.destroy()


def test_paired_gathers_need_a_scalar_cell():
    """unroll 2 is taken by the stream configurations of every scalar cell
    (with either cache policy where the cell has both) and gives the
    oracle's product there; block formats and other unroll values are
    rejected, and the tuner offers paired candidates only where they apply."""
    torch_or_skip()
    A = stencil_3d_27pt(6, 3)
    e = _encode(A)
    M = D.Matrix.create(A.nrows, A.ncols, e["rowptr"], e["off"], A.vals)
    x = dev(uniform_vector(A.ncols, 5))
    ref = OS.spmv_csr(A.nrows, A.ncols, A.rowptr, A.colids, A.vals, host(x))
    bnd = error_bound(A.nrows, A.rowptr, A.colids, A.vals, host(x), 1.0, 0.0, None, U64)
    for cache in (D.CACHE_NT, D.CACHE_PLAIN):
        M.set_config(D.VAR_STREAM, 4, 2, 2048, cache=cache)
        assert M.get_config()["unroll"] == 2 and M.takes_paired
        yd = dev(np.full(A.nrows, np.nan))
        M.spmv(x, yd)
        assert_within(host(yd), ref, bnd, f"paired cache={cache}")
    with pytest.raises(D.DamnError) as err:
        M.set_config(D.VAR_STREAM, 4, 3, 2048)
    assert err.value.code == -1  # DAMN_ERR_INVALID_ARG
    M.destroy()
    # int8 offsets take paired gathers too
    idx, _ = D.encode_index(D.FORMAT_DA8, A.nrows, A.ncols, A.rowptr, A.colids)
    M8 = D.Matrix.create_format(D.FORMAT_DA8, A.nrows, A.ncols, A.rowptr, idx, A.vals)
    assert M8.takes_paired
    M8.set_config(D.VAR_STREAM, 2, 2, 1024)
    yd = dev(np.full(A.nrows, np.nan))
    M8.spmv(x, yd)
    assert_within(host(yd), ref, bnd, "paired DA8")
    M8.destroy()
    # a block format does not
    from workloads.matrices import block_stencil_27pt
    B = block_stencil_27pt(4, 2, 3)
    eb = D.bsr_encode(B.nrows, B.ncols, B.rowptr, B.colids, B.vals, 2, D.FORMAT_DABSR16)
    MB = D.Matrix.bsr_create(D.FORMAT_DABSR16, B.nrows // 2, B.ncols // 2, 2, eb["browptr"],
                             eb["bidx"], eb["bvals"])
    assert not MB.takes_paired
    assert all(c[2] == 1 for c in candidates_for(MB) if c[0] == D.VAR_STREAM)
    with pytest.raises(D.DamnError) as err:
        MB.set_config(D.VAR_STREAM, 4, 2, 2048)
    assert err.value.code == -6  # DAMN_ERR_UNSUPPORTED
    MB.destroy()


def test_tuner_sets_its_choice_and_times_every_candidate():
    """The two-stage tuner: every candidate timed, the choice set on the
    handle and among the candidates, and the product with it correct."""
    torch = torch_or_skip()
    from paper_2307_06305_amd.tuning import autotune
    A = stencil_3d_27pt(16, 9)
    e = _encode(A)
    M = D.Matrix.create(A.nrows, A.ncols, e["rowptr"], e["off"], A.vals)
    x = uniform_vector(A.ncols, 12)
    xd = dev(x)
    yd = torch.zeros(A.nrows, dtype=torch.float64, device="cuda")
    best, times = autotune(M, xd, yd, reps=3, sustained_s=0.002)
    assert set(times) == set(candidates_for(M)) and best in times
    assert all(np.isfinite(t) and t > 0 for t in times.values())
    cfg = M.get_config()
    assert (cfg["variant"], cfg["lanes"], cfg["unroll"]) == best[:3]
    if best[0] == D.VAR_STREAM:
        assert cfg["tile"] == best[3]
    ref = OS.spmv_csr(A.nrows, A.ncols, A.rowptr, A.colids, A.vals, x)
    bnd = error_bound(A.nrows, A.rowptr, A.colids, A.vals, x, 1.0, 0.0, None, U64)
    yd = dev(np.full(A.nrows, np.nan))
    M.spmv(xd, yd)
    assert_within(host(yd), ref, bnd, config_name(best))
    M.destroy()


SPMM_CFGS = ([(D.VAR_VECTOR, lanes, 2048) for lanes in (1, 4, 8, 32, 64)]
             + [(D.VAR_STREAM, lanes, tile) for lanes in (1, 2, 4, 8, 16, 32, 64)
                for tile in (1024, 4096)])


def _dev_offset(a, offset):
    """A contiguous device copy of a whose data starts `offset` float64 past
    an allocation's start (offset 1: 8-byte but not 16-byte aligned)."""
    import torch

    flat = torch.zeros(a.size + offset, dtype=torch.float64, device="cuda")
    flat[offset:] = torch.from_numpy(np.ascontiguousarray(a).ravel()).to("cuda")
    return flat[offset:].view(*a.shape)


@pytest.mark.parametrize("fmt", ["da", "csr"])
@pytest.mark.parametrize("A", MATS, ids=lambda A: A.name)
def test_spmm_matches_oracle(A, fmt):
    """Both SpMM variants, every lane count, two tile sizes, aligned and
    unaligned operands (16-byte pairs or single values)."""
    torch_or_skip()
    print(f"case {A.name} {fmt}", flush=True)
    e = _encode(A)
    M = (D.Matrix.create(A.nrows, A.ncols, e["rowptr"], e["off"], A.vals) if fmt == "da"
         else D.Matrix.csr_create(A.nrows, A.ncols, A.rowptr, A.colids, A.vals))
    for nrhs in range(1, 9):
        X = uniform_vector(A.ncols, 10 + nrhs, nrhs)
        Y0 = uniform_vector(A.nrows, 20 + nrhs, nrhs)
        for alpha, beta in ((1.0, 0.0), (2.0, -1.0)):
            ref = OS.spmm_csr(A.nrows, A.ncols, A.rowptr, A.colids, A.vals, X, alpha, beta, Y0)
            bnds = [error_bound(A.nrows, A.rowptr, A.colids, A.vals, X[:, j], alpha, beta,
                                Y0[:, j], U64) for j in range(nrhs)]
            for variant, lanes, tile in SPMM_CFGS:
                for offset in ((0, 1) if nrhs % 2 == 0 else (0,)):
                    M.set_config(variant, lanes, 1, tile)
                    Yd = _dev_offset(Y0, offset)
                    M.spmm(_dev_offset(X, offset), Yd, alpha, beta)
                    Y = host(Yd)
                    for j in range(nrhs):
                        assert_within(Y[:, j], ref[:, j], bnds[j],
                                      f"{A.name} nrhs={nrhs} v={variant} lanes={lanes} "
                                      f"tile={tile} offset={offset}")
    M.destroy()


def test_spmm_alpha_zero_reads_neither_matrix_nor_x():
    torch = torch_or_skip()
    A = MATS[1]
    e = _encode(A)
    M = D.Matrix.create(A.nrows, A.ncols, e["rowptr"], e["off"], A.vals)
    X = torch.full((A.ncols, 3), float("nan"), dtype=torch.float64, device="cuda")
    for variant in (D.VAR_VECTOR, D.VAR_STREAM):
        M.set_config(variant, 2, 1, 2048)
        Y = torch.full((A.nrows, 3), 2.0, dtype=torch.float64, device="cuda")
        M.spmm(X, Y, 0.0, -0.5)
        assert np.all(host(Y) == -1.0)
    M.destroy()


def test_invalid_calls_return_status():
    torch = torch_or_skip()
    A = laplace_2d_5pt(8)
    e = _encode(A)
    M = D.Matrix.create(A.nrows, A.ncols, e["rowptr"], e["off"], A.vals)
    C = D.Matrix.csr_create(A.nrows, A.ncols, A.rowptr, A.colids, A.vals)
    x, y = dev(np.ones(64)), dev(np.zeros(64))
    with pytest.raises(D.DamnError):
        M.csr_spmv(x, y)          # DA handle through the CSR entry point
    with pytest.raises(D.DamnError):
        C.spmv(x, y)              # and the reverse
    X, Y = dev(np.ones((64, 9))), dev(np.zeros((64, 9)))
    with pytest.raises(D.DamnError) as ei:
        M.spmm(X, Y)
    assert ei.value.code == -6
    with pytest.raises(D.DamnError):
        M.set_config(0, 3, 1, 2048)  # lanes not a power of two
    with pytest.raises(D.DamnError):
        M.set_config(1, 8, 1, 100)   # tile too small
    # offsets that would read outside x are refused at upload
    with pytest.raises(D.DamnError) as ei:
        D.Matrix.create(2, 2, [0, 1, 2], np.array([1, 1], np.int16), np.ones(2))
    assert ei.value.code == -2
    M.destroy()
    C.destroy()


@pytest.mark.timeout(600)
def test_full_size_27pt_every_row():
    """The 128^3 27-point matrix in every configuration: every row of y
    against the oracle's full product.  y starts as NaN before each product,
    so a row no workgroup writes fails too."""
    torch = torch_or_skip()
    A = config_matrix(1)
    e = _encode(A)
    assert e["w"] == 16513
    M = D.Matrix.create(A.nrows, A.ncols, e["rowptr"], e["off"], A.vals)
    C = D.Matrix.csr_create(A.nrows, A.ncols, A.rowptr, A.colids, A.vals)
    x = uniform_vector(A.ncols, 2001)
    xd = dev(x)
    ref = OS.spmv_csr(A.nrows, A.ncols, A.rowptr, A.colids, A.vals, x)
    bnd = error_bound(A.nrows, A.rowptr, A.colids, A.vals, x, 1.0, 0.0, None, U64)
    yd = torch.empty(A.nrows, dtype=torch.float64, device="cuda")
    for mat in (M, C):
        for cfg in candidates_for(mat):
            print(f"case 27pt128 {mat.format} {config_name(cfg)}", flush=True)
            yd.fill_(float("nan"))
            mat.set_config(*cfg)
            mat.apply(xd, yd)
            assert_within(host(yd), ref, bnd, f"{mat.format} {config_name(cfg)}")
    M.destroy()
    C.destroy()


def test_first_product_of_a_fresh_handle_is_graph_capturable():
    """Create builds the tiles, so the first product call on a new handle only
    launches kernels: it is captured into a HIP graph, and every replay
    (with eager work and synchronisations between them) matches the oracle.
    Covers DA-CSR and CSR SpMV and a three-column SpMM."""
    torch = torch_or_skip()
    A = stencil_3d_27pt(20, 11)
    e = _encode(A)
    x = uniform_vector(A.ncols, 77)
    X = np.stack([uniform_vector(A.ncols, 78 + j) for j in range(3)], axis=1)
    ref = OS.spmv_csr(A.nrows, A.ncols, A.rowptr, A.colids, A.vals, x)
    bnd = error_bound(A.nrows, A.rowptr, A.colids, A.vals, x, 1.0, 0.0, None, U64)
    refX = OS.spmm_csr(A.nrows, A.ncols, A.rowptr, A.colids, A.vals, X)
    xd, Xd = dev(x), dev(X)
    for kind in ("da", "csr", "spmm"):
        if kind == "csr":
            M = D.Matrix.csr_create(A.nrows, A.ncols, A.rowptr, A.colids, A.vals)
        else:
            M = D.Matrix.create(A.nrows, A.ncols, e["rowptr"], e["off"], A.vals)
        out = torch.full((A.nrows, 3) if kind == "spmm" else (A.nrows,), float("nan"),
                         dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            if kind == "spmm":
                M.spmm(Xd, out)
            else:
                M.apply(xd, out)
        for rep in range(3):
            out.fill_(float("nan"))
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            got = host(out)
            if kind == "spmm":
                for j in range(3):
                    bj = error_bound(A.nrows, A.rowptr, A.colids, A.vals, X[:, j], 1.0, 0.0,
                                     None, U64)
                    assert_within(got[:, j], refX[:, j], bj, f"spmm replay {rep} rhs {j}")
            else:
                assert_within(got, ref, bnd, f"{kind} replay {rep}")
            # eager work between replays
            (xd * 2.0).sum().item()
        del g
        M.destroy()


def test_probes_read_what_they_claim():
    """The measurement probes: the read probe's checksums cover every byte
    of the buffer on every pass (a buffer of ones folds to a known value
    per workgroup), and the gather probe reads per_row values per row
    (x = 1 sums to rows * per_row; half-width 0 reads x[r] per_row times)."""
    torch = torch_or_skip()
    sink = torch.zeros(65536, dtype=torch.float64, device="cuda")
    # gather probe
    n, per_row = 100_003, 12
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    D.gather_read(x, sink, n, per_row, halfwidth=20000)
    assert host(sink)[: (n + 255) // 256].sum() == n * per_row
    sink.zero_()
    x = torch.arange(n, dtype=torch.float64, device="cuda")
    D.gather_read(x, sink, n, per_row, halfwidth=0)
    assert host(sink)[: (n + 255) // 256].sum() == per_row * (n - 1) * n // 2
    # stencil offsets: x[r + d] clipped to [0, n)
    offs = np.array([-300, -1, 0, 1, 300], dtype=np.int32)
    sink.zero_()
    D.gather_read(x, sink, n, offs.size, offs=dev(offs))
    r = np.arange(n)
    want = sum(np.clip(r + d, 0, n - 1).sum() for d in offs)
    assert host(sink)[: (n + 255) // 256].sum() == want
    # read probe, register and LDS paths, one and several passes: a buffer
    # whose 16-byte pieces are (1, 0, 0, 0) words folds to XOR = 1 per odd
    # number of pieces a workgroup reads
    buf = torch.zeros(1 << 22, dtype=torch.int32, device="cuda")
    buf[0::4] = 1
    for mode in (D.READ_NT, D.READ_PLAIN, D.READ_LDS_NT, D.READ_LDS_PLAIN):
        for passes in (1, 3):
            sink.fill_(-1.0)
            D.stream_read(buf, sink, mode, 8192, passes=passes)
            s = host(sink)
            # every workgroup wrote its checksum (0 or 1: an even or odd
            # count of pieces), none is left at -1
            assert np.all((s == 0.0) | (s == 1.0) | (s == -1.0))
            if mode in (D.READ_LDS_NT, D.READ_LDS_PLAIN):
                tiles = (buf.numel() * 4) // 8192
                assert np.all(s[: tiles * passes] >= 0.0)
