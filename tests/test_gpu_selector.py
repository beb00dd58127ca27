"""The kernel selector on the GPU: network gradients and inference against
the float64 oracle, training, the autotuner, and what the shipped network
gains over the library's default configuration on matrices it never saw."""

import os

import numpy as np
import pytest

import paper_2307_06305_amd as D
from gpu_util import dev, torch_or_skip
from oracle import mlp as OM
from paper_2307_06305_amd import selector as S
from paper_2307_06305_amd.tuning import candidates
from workloads.matrices import batch_matrix, batch_member

pytestmark = pytest.mark.gpu

K = D.NCLASS
S0 = D.CLASS_SPMM  # first SpMM class


def _mask(F):
    spmm = F[:, 9] > 1.5
    cls = np.arange(K)
    return np.where(spmm[:, None], cls[None, :] >= S0, cls[None, :] < S0)


def _params(seed):
    rng = np.random.default_rng(seed)
    net = D.Mlp(seed=seed)
    p = net.params()
    net.destroy()
    p[OM.nparams(K) - 32:OM.nparams(K) - 16] = rng.standard_normal(16)           # mu
    p[OM.nparams(K) - 16:] = rng.uniform(0.5, 2.0, 16)                           # sigma
    p[:OM.nparams(K) - 32] += rng.standard_normal(OM.nparams(K) - 32) * 0.05
    return p.astype(np.float32)


def _batch(B, seed):
    rng = np.random.default_rng(seed)
    F = rng.standard_normal((B, 16)).astype(np.float32)
    F[:, 9] = rng.choice([1.0, 4.0], B)
    times = rng.uniform(1.0, 2.0, (B, K))
    times[~_mask(F)] = np.inf
    Q, _ = OM.soft_targets(times, 0.1)
    return F, Q.astype(np.float32)


def test_gradients_match_oracle():
    torch_or_skip()
    p = _params(3)
    F, Q = _batch(40, 4)
    net = D.Mlp(p)
    loss, g = net.grad(F, Q)
    net.destroy()
    P = OM.unpack(p.astype(np.float64), K)
    lref, gref = OM.backward(P, F.astype(np.float64), _mask(F), Q.astype(np.float64))
    assert abs(loss - lref) <= 1e-4 * abs(lref)
    off = 0
    for name, shp in OM.shapes(K):
        size = int(np.prod(shp))
        got = g[off:off + size].reshape(shp)
        ref = gref[name]
        scale = np.abs(ref).max()
        assert np.abs(got - ref).max() <= 1e-4 * scale + 1e-7, name
        off += size
    assert np.all(g[off:] == 0)


def test_select_matches_oracle_argmax():
    torch_or_skip()
    p = _params(5)
    F, _ = _batch(300, 6)
    net = D.Mlp(p)
    got = net.select(F)
    net.destroy()
    P = OM.unpack(p.astype(np.float64), K)
    mask = _mask(F)
    ref = OM.select(P, F.astype(np.float64), mask)
    Z = np.where(mask, OM.forward(P, F.astype(np.float64), mask)["Z"], -np.inf)
    top2 = np.sort(Z, axis=1)[:, -2:]
    clear = top2[:, 1] - top2[:, 0] > 1e-3
    assert clear.sum() > 250
    assert np.array_equal(got[clear], ref[clear])
    assert np.all(mask[np.arange(len(F)), got])


def test_training_reduces_loss():
    torch_or_skip()
    rng = np.random.default_rng(0)
    N = 2048
    F = rng.standard_normal((N, 16)).astype(np.float32)
    F[:, 9] = 1.0
    best = (F[:, 0] > 0).astype(int) * 3 + (F[:, 1] > 0).astype(int) * 21
    T = np.full((N, K), 2.0, dtype=np.float32)
    T[:, S0:] = np.inf
    T[np.arange(N), best] = 1.0
    net = D.Mlp(seed=2)
    losses = net.train(F, T, epochs=40, batch=128, lr=3e-3, tau=0.05, seed=3)
    acc = np.mean(net.select(F) == best)
    net.destroy()
    assert losses[-1] < 0.2 * losses[0]
    assert acc > 0.95


def test_autotune_sets_fastest_class():
    torch = torch_or_skip()
    d = batch_member(9, 1, n_lo=2e4, n_hi=3e4)
    A = batch_matrix(d)
    e = D.encode(A.nrows, A.ncols, A.rowptr, A.colids, A.vals, allow_rcm=False)
    M = D.Matrix.create(A.nrows, A.ncols, e["rowptr"], e["off"], e["vals"])
    x = dev(np.ones(A.ncols))
    y = torch.zeros(A.nrows, dtype=torch.float64, device="cuda")
    t = D.autotune(M, 1, x, y, reps=2)
    assert np.all(np.isfinite(t[:S0])) and np.all(np.isinf(t[S0:]))
    assert S.config_class(M.get_config(), 1) == int(np.argmin(t))
    X = dev(np.ones((A.ncols, 3)))
    Y = torch.zeros(A.nrows, 3, dtype=torch.float64, device="cuda")
    t3 = D.autotune(M, 3, X, Y, reps=2)
    assert np.all(np.isinf(t3[:S0])) and np.all(np.isfinite(t3[S0:]))
    assert S.config_class(M.get_config(), 3) == S0 + int(np.argmin(t3[S0:]))
    M.destroy()


def test_class_table_matches_tuning_candidates():
    assert len(candidates()) == S0
    for k, c in enumerate(candidates()):
        v, l, u, tile, mm = D.class_config(k)
        assert (v, l, u) == c[:3] and not mm
        if v == 1:
            assert tile == c[3]
            assert S.config_class({"variant": v, "lanes": l, "unroll": u, "tile": tile}, 1) == k
    for k in range(S0, K):
        v, l, u, tile, mm = D.class_config(k)
        assert mm and v == 1 and u == 1 and l == 2 ** (k - S0)


def test_shipped_selector_beats_the_default_on_unseen_matrices():
    """Matrices from seeds the network was not trained on: the shipped
    network's choice against the library default (no selector) and against
    the exhaustive autotuner.  The autotuner's times are averaged over three
    collections: the regret divides by the fastest of 63 timings, and with a
    single noisy collection that minimum is biased low."""
    torch_or_skip()
    assert os.path.exists(S.WEIGHTS), "trained selector weights are missing"
    runs = [S.collect(64, seed=6006, reps=5) for _ in range(3)]
    data = runs[0]
    T = np.mean([d["T"] for d in runs], axis=0)
    W = S.load_weights()
    res = S.evaluate(W, data["F"], T, data["default"])
    fb = S.evaluate_fallback(W, data["F"], T, 0.2)
    print(f"selector: {res['samples']} products, mean regret {res['mean_regret']:.4f}, "
          f"p95 {res['p95_regret']:.4f}, within 5% {res['within_5pct']:.3f}; with the "
          f"autotuner fallback (p < 0.2): mean {fb['mean_regret']:.4f}, "
          f"p95 {fb['p95_regret']:.4f}, within 5% {fb['within_5pct']:.3f}, "
          f"fallback {fb['fallback_fraction']:.2f}", flush=True)
    assert res["mean_regret"] < res["default_mean_slowdown"]
    assert res["time_ratio_default_over_selected"] > 1.0
    # the target: choices within 5% of the autotuner's time on average
    assert res["mean_regret"] <= 0.05
    assert res["within_5pct"] >= 0.75
    # with the fallback (selector.choose), the tail is held too
    assert fb["mean_regret"] <= 0.05 and fb["p95_regret"] <= 0.10
    assert fb["within_5pct"] >= 0.9


def test_select_probability_matches_oracle_softmax():
    torch_or_skip()
    p = _params(8)
    F, _ = _batch(200, 9)
    net = D.Mlp(p)
    cls, prob = net.select(F, with_prob=True)
    net.destroy()
    P = OM.unpack(p.astype(np.float64), K)
    mask = _mask(F)
    Z = np.where(mask, OM.forward(P, F.astype(np.float64), mask)["Z"], -np.inf)
    ez = np.exp(Z - Z.max(axis=1, keepdims=True))
    ref = (ez / ez.sum(axis=1, keepdims=True))[np.arange(len(F)), cls]
    assert np.all(np.abs(prob - ref) <= 1e-4 * ref + 1e-6)
    assert np.all((prob > 0) & (prob <= 1.0 + 1e-6))


def test_choose_takes_interleaved_gathers_where_paired_do_not_apply():
    """A network class with paired gathers, chosen for a handle whose format
    has none (DA-BSR), sets the same lanes and tile with the interleaved
    gathers."""
    torch = torch_or_skip()
    from workloads.matrices import block_stencil_27pt
    A = block_stencil_27pt(6, 2, 5)
    eb = D.bsr_encode(A.nrows, A.ncols, A.rowptr, A.colids, A.vals, 2, D.FORMAT_DABSR16)
    MB = D.Matrix.bsr_create(D.FORMAT_DABSR16, A.nrows // 2, A.ncols // 2, 2, eb["browptr"],
                             eb["bidx"], eb["bvals"])
    k = S.config_class({"variant": D.VAR_STREAM, "lanes": 4, "unroll": 2, "tile": 2048}, 1)
    assert D.class_config(k)[:4] == (D.VAR_STREAM, 4, 2, 2048)

    class Fixed:  # answers class k with probability 1
        def select(self, f, with_prob=False):
            return np.array([k]), np.array([1.0], dtype=np.float32)

    x = dev(np.ones(A.ncols))
    y = torch.zeros(A.nrows, dtype=torch.float64, device="cuda")
    cls, prob, tuned = S.choose(Fixed(), A, MB, 1, x, y)
    assert cls == k and not tuned
    cfg = MB.get_config()
    assert (cfg["variant"], cfg["lanes"], cfg["unroll"], cfg["tile"]) == (D.VAR_STREAM, 4, 1, 2048)
    MB.destroy()


def test_choose_falls_back_to_the_autotuner():
    """Below the probability threshold the exhaustive autotuner configures
    the handle; above it the network's class is set."""
    torch = torch_or_skip()
    d = batch_member(12, 3, n_lo=2e4, n_hi=4e4)
    A = batch_matrix(d)
    e = D.encode(A.nrows, A.ncols, A.rowptr, A.colids, A.vals, allow_rcm=False)
    M = D.Matrix.create(A.nrows, A.ncols, e["rowptr"], e["off"], e["vals"])
    x = dev(np.ones(A.ncols))
    y = torch.zeros(A.nrows, dtype=torch.float64, device="cuda")
    net = S.load_net()
    cls, prob, tuned = S.choose(net, A, M, 1, x, y, threshold=0.0)
    assert not tuned and S.config_class(M.get_config(), 1) == cls
    cls2, prob2, tuned2 = S.choose(net, A, M, 1, x, y, threshold=1.01)
    assert tuned2 and prob2 == prob and S.config_class(M.get_config(), 1) == cls2
    net.destroy()
    M.destroy()
