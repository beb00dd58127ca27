"""Full-size parity on the GPU for the measured workloads other than the
27-point matrix (whose every-row test is in test_gpu_spmv.py): every row of
every product against the oracle's full product, or properties that hold at
any size, in every configuration the autotuner may pick.  Outputs start as
NaN, so a row that no workgroup writes fails too.

- random band, n = 4,000,000, natural order: every row, DA-CSR and CSR;
- its scrambled copy, reordered by the library's RCM + refinement: the
  permuted product equals the original product permuted, every row;
- CG on the 7-point operator of the 128 x 128 x 1024 box: the oracle's
  recomputed true residual of both solutions is below 1e-10;
- the batch of 512 matrices: every row of every matrix, every RHS.
"""

import numpy as np
import pytest

import paper_2307_06305_amd as D
from gpu_util import U64, assert_within, dev, error_bound, host, torch_or_skip
from oracle import spmv as OS
from paper_2307_06305_amd.tuning import candidates_for, config_name
from workloads import config_matrix, config_vector
from workloads.matrices import batch_matrix, batch_member

pytestmark = pytest.mark.gpu


@pytest.mark.timeout(600)
def test_banded_full_size_every_row():
    torch = torch_or_skip()
    A = config_matrix(2)
    print(f"case {A.name} nnz={A.nnz}", flush=True)
    e = D.encode(A.nrows, A.ncols, A.rowptr, A.colids, A.vals, allow_rcm=False)
    M = D.Matrix.create(A.nrows, A.ncols, e["rowptr"], e["off"], e["vals"])
    C = D.Matrix.csr_create(A.nrows, A.ncols, A.rowptr, A.colids, A.vals)
    x = config_vector(2, A.ncols)
    ref = OS.spmv_csr(A.nrows, A.ncols, A.rowptr, A.colids, A.vals, x)
    bnd = error_bound(A.nrows, A.rowptr, A.colids, A.vals, x, 1.0, 0.0, None, U64)
    xd = dev(x)
    yd = torch.empty(A.nrows, dtype=torch.float64, device="cuda")
    for mat in (M, C):
        for cfg in candidates_for(mat):
            print(f"case band {mat.format} {config_name(cfg)}", flush=True)
            yd.fill_(float("nan"))
            mat.set_config(*cfg)
            mat.apply(xd, yd)
            assert_within(host(yd), ref, bnd, f"{mat.format} {config_name(cfg)}")
    M.destroy()
    C.destroy()


@pytest.mark.timeout(600)
def test_scrambled_band_reordered_product_every_row():
    torch = torch_or_skip()
    Q = config_matrix(2, scrambled=True)
    assert not D.fit_check(Q.nrows, Q.ncols, Q.rowptr, Q.colids)[3]
    e = D.encode(Q.nrows, Q.ncols, Q.rowptr, Q.colids, Q.vals, allow_rcm=True)
    assert e["permuted"] and e["w"] < 2**15
    perm = e["perm"].astype(np.int64)
    assert np.array_equal(np.sort(perm), np.arange(Q.nrows))
    M = D.Matrix.create(Q.nrows, Q.ncols, e["rowptr"], e["off"], e["vals"])
    x = config_vector(2, Q.ncols, salt=1)
    # y_p = (P A P^T) x_p with x_p[i] = x[perm[i]] must give y_p[i] = (A x)[perm[i]]:
    # the oracle's product of the scrambled matrix in its own order, permuted
    ref = OS.spmv_csr(Q.nrows, Q.ncols, Q.rowptr, Q.colids, Q.vals, x)[perm]
    bnd = error_bound(Q.nrows, Q.rowptr, Q.colids, Q.vals, x, 1.0, 0.0, None, U64)[perm]
    xd = dev(x[perm])
    yd = torch.empty(Q.nrows, dtype=torch.float64, device="cuda")
    for cfg in candidates_for(M):
        print(f"case scrambled band {config_name(cfg)}", flush=True)
        yd.fill_(float("nan"))
        M.set_config(*cfg)
        M.spmv(xd, yd)
        assert_within(host(yd), ref, bnd, config_name(cfg))
    M.destroy()


def test_cg_full_size_true_residual():
    """Both solvers on n = 16,777,216: the oracle recomputes r = b - A x in
    float64 for each returned x; both are below 1e-10 relative."""
    torch = torch_or_skip()
    A = config_matrix(3)
    e = D.encode(A.nrows, A.ncols, A.rowptr, A.colids, A.vals, allow_rcm=False)
    A64 = D.Matrix.create(A.nrows, A.ncols, e["rowptr"], e["off"], e["vals"], store=D.F64)
    A32 = D.Matrix.create(A.nrows, A.ncols, e["rowptr"], e["off"], e["vals"], store=D.F32)
    b = config_vector(3, A.nrows)
    bd = dev(b)
    nb = np.linalg.norm(b)
    sols = {}
    for name, a32 in (("fp64", None), ("mixed", A32)):
        xd = torch.zeros_like(bd)
        info = D.cg(A64, bd, xd, A32=a32, tol=1e-10, inner_tol=1e-5, max_iter=20000,
                    check_every=32)
        assert info["converged"], (name, info)
        x = host(xd)
        r = b - OS.spmv_csr(A.nrows, A.ncols, A.rowptr, A.colids, A.vals, x)
        rel = np.linalg.norm(r) / nb
        print(name, info, "oracle residual", rel, flush=True)
        assert rel <= 1.05e-10, (name, rel)
        sols[name] = x
    # reported, not pinned: the two solutions agree to the conditioning bound
    err = np.linalg.norm(sols["mixed"] - sols["fp64"]) / np.linalg.norm(sols["fp64"])
    print("mixed vs fp64 relative difference", err, flush=True)
    assert err < 1e-5
    A64.destroy()
    A32.destroy()


@pytest.mark.timeout(900)
def test_batch_full_size_every_row():
    """The 512-matrix batch the bench measures (seed 1004), one graph launch:
    every row of every matrix, for every right-hand side, against the
    oracle's full products; Y starts as NaN."""
    torch = torch_or_skip()
    rng = np.random.default_rng(5)
    mats, Xs, Ys, data = [], [], [], []
    for i in range(512):
        d = batch_member(1004, i)
        A = batch_matrix(d)
        e = D.encode(A.nrows, A.ncols, A.rowptr, A.colids, A.vals, allow_rcm=False)
        M = D.Matrix.create(A.nrows, A.ncols, e["rowptr"], e["off"], e["vals"])
        k = d["nrhs"]
        X = rng.uniform(-1, 1, (A.ncols, k))
        mats.append(M)
        Xs.append(dev(X))
        Ys.append(torch.full((A.nrows, k), float("nan"), dtype=torch.float64, device="cuda"))
        data.append((A, X))
    print("case batch512: built", flush=True)
    B = D.Batch(mats, Xs, Ys, 1.0, 0.0)
    B.run(use_graph=True)
    torch.cuda.synchronize()
    for i, (A, X) in enumerate(data):
        got = host(Ys[i])
        ref = OS.spmm_csr(A.nrows, A.ncols, A.rowptr, A.colids, A.vals, X)
        for j in range(X.shape[1]):
            bnd = error_bound(A.nrows, A.rowptr, A.colids, A.vals, X[:, j], 1.0, 0.0, None, U64)
            assert_within(got[:, j], ref[:, j], bnd, f"matrix {i} rhs {j}")
    B.destroy()
    for M in mats:
        M.destroy()
