"""The allocation-free selection entry point, damn_select_noalloc, against
damn_select_prob through the C ABI: the same classes and probabilities, bit
for bit (the same inference kernel on the same rows), on two calls in a
row, the second with fewer rows than the first, so stale rows left in the
fixed scratch area by the first call must not leak into the second.  Row
counts beyond the scratch area are refused before anything is launched."""

import numpy as np
import pytest

import paper_2307_06305_amd as D
from gpu_util import torch_or_skip
from paper_2307_06305_amd import selector as S

pytestmark = pytest.mark.gpu


def _rows(n, seed, P):
    """Feature rows spread around the network's own normalisation (mu,
    sigma), nrhs (feature 9) in 1..8 so both class ranges occur."""
    rng = np.random.default_rng(seed)
    mu = P[D.MLP_NPARAMS - 32:D.MLP_NPARAMS - 16]
    sigma = P[D.MLP_NPARAMS - 16:]
    F = (mu + sigma * rng.standard_normal((n, 16)) * 1.5).astype(np.float32)
    F[:, 9] = rng.integers(1, 9, n)
    return F


def test_select_noalloc_matches_select_prob():
    torch_or_skip()
    P = S.load_weights()
    net = D.Mlp(P)
    mx = D.SELECT_NOALLOC_MAX_ROWS
    for n, seed in ((mx, 11), (257, 12)):
        print(f"case select_noalloc n={n}", flush=True)
        F = _rows(n, seed, P)
        want_c, want_p = net.select(F, with_prob=True)
        got_c, got_p = net.select_noalloc(F, with_prob=True)
        assert np.array_equal(got_c, want_c), f"n={n}: classes differ"
        assert np.array_equal(got_p.view(np.int32), want_p.view(np.int32)), \
            f"n={n}: probabilities differ"
        # without the probability output
        assert np.array_equal(net.select_noalloc(F), want_c)
        assert set(np.unique(want_c[F[:, 9] > 1.5])) <= set(range(D.CLASS_SPMM, D.NCLASS))
        assert set(np.unique(want_c[F[:, 9] < 1.5])) <= set(range(D.CLASS_SPMM))
    # nothing to do
    assert net.select_noalloc(np.zeros((0, 16), dtype=np.float32)).size == 0
    # beyond the scratch area: refused with its own status
    with pytest.raises(D.DamnError) as e:
        net.select_noalloc(_rows(mx + 1, 13, P))
    assert e.value.code == -9
    net.destroy()
