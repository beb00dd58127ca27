"""Pins of the selector oracle: features by hand and by closed form, the
network's backward pass against central finite differences, soft targets,
the first Adam step, and the forward pass on hand-set weights."""

import math

import numpy as np
import pytest

from conftest import golden
from oracle import features as OF
from oracle import mlp as M
from workloads import laplace_2d_5pt


def test_features_example1_by_hand():
    g = golden("example1.json")
    f = OF.features(4, 4, g["rowptr"], g["csr_colids"], 3)
    # row lengths (1, 1, 2, 1); |c - r| = (0, 1, 1, 1, 0); the only pair of
    # entries in one row is (1, 3) in row 2: column step 2
    mean = 1.25
    std = math.sqrt(1.75 - mean * mean)
    want = [math.log2(5), math.log2(6), mean, std, math.log2(3), 0.0, 1.0, 0.25, 0.0, 3.0,
            math.log2(1.6), 1.0, std / mean, 0.0, math.log2(5), 0.0]
    assert np.allclose(f, want, rtol=1e-15, atol=0)


@pytest.mark.parametrize("N", [4, 9, 30])
def test_features_laplace_closed_forms(N):
    A = laplace_2d_5pt(N)
    f = OF.features(A.nrows, A.ncols, A.rowptr, A.colids, 1)
    n = N * N
    nnz = 5 * n - 4 * N
    assert f[1] == pytest.approx(math.log2(nnz + 1))
    assert f[2] == pytest.approx(nnz / n)
    assert f[6] == pytest.approx(math.log2(N + 1)) and f[7] == pytest.approx(N / n)
    assert f[11] == 1.0 and f[8] == 0.0 and f[13] == 0.0
    # adjacent pairs: rows of length L have L-1 pairs; column steps of 1 are
    # (left, centre) and (centre, right) whenever those neighbours exist
    pairs = nnz - n
    unit = 2 * (N - 1) * N
    assert f[15] == pytest.approx(unit / pairs)
    # mean |c - r|: each of the 2N(N-1) horizontal neighbours is at 1, each of
    # the 2N(N-1) vertical ones at N, the diagonal at 0
    mean_d = (2 * N * (N - 1) * 1 + 2 * N * (N - 1) * N) / nnz
    assert f[10] == pytest.approx(math.log2(mean_d + 1))


def _rand_params(K, seed):
    rng = np.random.default_rng(seed)
    flat = rng.standard_normal(M.nparams(K)) * 0.4
    P = M.unpack(flat, K)
    P["mu"] = rng.standard_normal(M.NFEAT)
    P["sigma"] = rng.uniform(0.5, 2.0, M.NFEAT)
    return P


def _batch(K, B, seed):
    rng = np.random.default_rng(seed)
    F = rng.standard_normal((B, M.NFEAT))
    times = rng.uniform(1.0, 3.0, (B, K))
    times[rng.random((B, K)) < 0.3] = np.inf
    times[:, 0] = rng.uniform(1.0, 3.0, B)  # at least one valid class
    Q, mask = M.soft_targets(times, 0.1)
    return F, mask, Q


def test_backward_matches_central_differences():
    K, B = 9, 7
    P = _rand_params(K, 1)
    F, mask, Q = _batch(K, B, 2)
    _, g = M.backward(P, F, mask, Q)
    h = 1e-6
    rng = np.random.default_rng(3)
    for name in ("W1", "b1", "W2", "b2", "W3", "b3"):
        for _ in range(6):
            idx = tuple(int(rng.integers(0, s)) for s in P[name].shape)
            old = P[name][idx]
            P[name][idx] = old + h
            lp, _ = M.loss(P, F, mask, Q)
            P[name][idx] = old - h
            lm, _ = M.loss(P, F, mask, Q)
            P[name][idx] = old
            fd = (lp - lm) / (2 * h)
            assert abs(fd - g[name][idx]) <= 1e-6 * max(1.0, abs(fd)), (name, idx)


def test_forward_hand_set_weights():
    # all weights zero: probabilities are the softmax of b3 over valid classes
    K = 4
    P = M.unpack(np.zeros(M.nparams(K)), K)
    P["sigma"] = np.ones(M.NFEAT)
    P["b3"] = np.log(np.array([1.0, 2.0, 3.0, 4.0]))
    mask = np.array([[True, True, False, True]])
    c = M.forward(P, np.zeros((1, M.NFEAT)), mask)
    assert np.allclose(c["P"], [[1 / 7, 2 / 7, 0.0, 4 / 7]], rtol=1e-15)
    assert M.select(P, np.zeros((1, M.NFEAT)), mask).tolist() == [3]


def test_soft_targets_closed_form():
    Q, valid = M.soft_targets(np.array([[1.0, 2.0, np.inf]]), 0.5)
    e = math.exp(-2.0)
    assert np.allclose(Q, [[1 / (1 + e), e / (1 + e), 0.0]], rtol=1e-15)
    assert valid.tolist() == [[True, True, False]]


def test_first_adam_step_is_a_signed_step():
    # from zero moments the bias-corrected step is lr * g / (|g| + eps)
    P = {"W": np.array([1.0, -2.0, 0.5])}
    g = {"W": np.array([0.3, -4.0, 0.0])}
    m = {"W": np.zeros(3)}
    v = {"W": np.zeros(3)}
    M.adam(P, g, m, v, 1, lr=0.01)
    assert np.allclose(P["W"], [0.99, -1.99, 0.5], rtol=0, atol=1e-9)


def test_training_on_a_separable_task_drives_loss_down():
    K, B = 5, 64
    rng = np.random.default_rng(0)
    F = rng.standard_normal((B, M.NFEAT))
    best = (F[:, 0] > 0).astype(int) + 2 * (F[:, 1] > 0)
    times = np.full((B, K), 2.0)
    times[np.arange(B), best] = 1.0
    Q, mask = M.soft_targets(times, 0.05)
    P = _rand_params(K, 4)
    P["mu"], P["sigma"] = np.zeros(M.NFEAT), np.ones(M.NFEAT)
    m = {k: np.zeros_like(P[k]) for k, _ in M.shapes(K)}
    v = {k: np.zeros_like(P[k]) for k, _ in M.shapes(K)}
    l0, _ = M.loss(P, F, mask, Q)
    for t in range(1, 301):
        _, g = M.backward(P, F, mask, Q)
        M.adam(P, g, m, v, t, lr=0.01)
    l1, _ = M.loss(P, F, mask, Q)
    assert l1 < 0.2 * l0
    assert np.mean(M.select(P, F, mask) == best) > 0.9
