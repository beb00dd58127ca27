"""Batched persistent SpMM on the GPU: per-matrix parity with the oracle,
every tile processed exactly once (beta != 0 would expose a repeat or a
skip), and graph replays checked one by one against the oracle."""

import numpy as np
import pytest

import paper_2307_06305_amd as D
from gpu_util import U64, assert_within, dev, error_bound, host, torch_or_skip
from oracle import spmv as OS
from workloads.matrices import batch_matrix, batch_member, uniform_vector

pytestmark = pytest.mark.gpu


def _family(count, seed):
    out = []
    for i in range(count):
        d = batch_member(seed, i, n_lo=60, n_hi=30000)
        out.append((d, batch_matrix(d)))
    return out


def _setup(torch, count, seed):
    fam = _family(count, seed)
    mats, Xs, Ys, Y0s, data = [], [], [], [], []
    rng = np.random.default_rng(seed)
    for i, (d, A) in enumerate(fam):
        e = D.encode(A.nrows, A.ncols, A.rowptr, A.colids, A.vals, allow_rcm=False)
        M = D.Matrix.create(A.nrows, A.ncols, e["rowptr"], e["off"], e["vals"])
        M.set_config(D.VAR_STREAM, int(rng.choice([1, 2, 4, 8, 16])), 1, 2048)
        k = d["nrhs"]
        X = uniform_vector(A.ncols, 100 + i, k)
        Y0 = uniform_vector(A.nrows, 200 + i, k)
        mats.append(M)
        Xs.append(dev(X))
        Ys.append(dev(Y0))
        Y0s.append(Y0)
        data.append((A, e, X))
    return mats, Xs, Ys, Y0s, data


def _expect(A, e, X, Yprev, alpha, beta):
    Y = OS.spmm_da(A.nrows, A.ncols, e["rowptr"], e["off"], e["vals"], X, alpha, beta, Yprev)
    bounds = [error_bound(A.nrows, A.rowptr, A.colids, A.vals, X[:, j], alpha, beta, Yprev[:, j],
                          U64) for j in range(X.shape[1])]
    return Y, bounds


@pytest.mark.parametrize("workgroups", [0, 37, 1024])
def test_batch_direct_matches_oracle(workgroups):
    torch = torch_or_skip()
    alpha, beta = 1.5, -0.5
    mats, Xs, Ys, Y0s, data = _setup(torch, 48, 7)
    B = D.Batch(mats, Xs, Ys, alpha, beta, workgroups=workgroups)
    info = B.info()
    assert info["ntiles"] > 0
    # 0: one workgroup per tile; else a persistent grid of that size
    assert info["workgroups"] == (workgroups or info["ntiles"])
    B.run(use_graph=False)
    for i, (A, e, X) in enumerate(data):
        Y, bounds = _expect(A, e, X, Y0s[i], alpha, beta)
        got = host(Ys[i])
        for j in range(X.shape[1]):
            assert_within(got[:, j], Y[:, j], bounds[j], f"matrix {i} rhs {j}")
    B.destroy()


@pytest.mark.parametrize("workgroups", [0, 256])
def test_batch_graph_replays_match_oracle(workgroups):
    torch = torch_or_skip()
    alpha, beta = 0.75, 0.5
    mats, Xs, Ys, Y0s, data = _setup(torch, 24, 11)
    B = D.Batch(mats, Xs, Ys, alpha, beta, workgroups=workgroups)
    prev = [y.copy() for y in Y0s]
    scratch = torch.randn(512, 512, device="cuda", dtype=torch.float32)
    for replay in range(3):
        B.run(use_graph=True)
        torch.cuda.synchronize()
        for i, (A, e, X) in enumerate(data):
            Y, bounds = _expect(A, e, X, prev[i], alpha, beta)
            got = host(Ys[i])
            for j in range(X.shape[1]):
                assert_within(got[:, j], Y[:, j], bounds[j], f"replay {replay} matrix {i} rhs {j}")
            prev[i] = got
        # eager work of the program between replays
        scratch = (scratch @ scratch.T) * 1e-3
        torch.cuda.synchronize()
    B.destroy()


def test_batch_rejects_bad_inputs():
    torch = torch_or_skip()
    A = batch_matrix(batch_member(3, 0, n_lo=100, n_hi=200))
    e = D.encode(A.nrows, A.ncols, A.rowptr, A.colids, A.vals, allow_rcm=False)
    M = D.Matrix.create(A.nrows, A.ncols, e["rowptr"], e["off"], e["vals"])
    Cm = D.Matrix.csr_create(A.nrows, A.ncols, A.rowptr, A.colids, A.vals)
    X = dev(np.ones((A.ncols, 9)))
    Y = dev(np.zeros((A.nrows, 9)))
    with pytest.raises(D.DamnError) as ei:
        D.Batch([M], [X], [Y])
    assert ei.value.code == -6
    X1, Y1 = dev(np.ones((A.ncols, 1))), dev(np.zeros((A.nrows, 1)))
    with pytest.raises(D.DamnError) as ei:
        D.Batch([Cm], [X1], [Y1])
    assert ei.value.code == -1
    M.destroy()
    Cm.destroy()
