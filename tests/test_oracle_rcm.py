"""Pins of the oracle's reverse Cuthill-McKee ordering: hand-worked graphs,
closed-form bandwidths and invariants (the paper gives no RCM example whose
data is available; its ldoor bandwidth 9120 needs a matrix not present here)."""

import collections

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import reverse_cuthill_mckee

from conftest import golden
from oracle import rcm as R
from oracle import storage as S
from workloads import laplace_2d_5pt, random_banded, scramble_symmetric, random_csr


def _csr_from_edges(n, edges):
    rows = [[] for _ in range(n)]
    for a, b in edges:
        rows[a].append(b)
    rp = np.zeros(n + 1, dtype=np.int32)
    rp[1:] = np.cumsum([len(r) for r in rows])
    c = np.array([x for r in rows for x in sorted(r)], dtype=np.int32)
    return rp, c


def test_example1_by_hand():
    # pattern of Fig. 1: (0,0) (1,2) (2,1) (2,3) (3,3); graph edges 1-2, 2-3,
    # vertex 0 isolated.  deg = (0,1,2,1): seed 0 first (deg 0), then 1 (deg 1,
    # lower index than 3).  From 1 the levels are {1},{2},{3}; from 3 also
    # three levels, so 1 stays the start.  CM order 0,1,2,3; reversed 3,2,1,0.
    g = golden("example1.json")
    perm = R.rcm(4, np.array(g["rowptr"]), np.array(g["csr_colids"]))
    assert perm.tolist() == [3, 2, 1, 0]


def test_star_by_hand():
    # star: centre 0, leaves 1..4.  Seed is leaf 1 (deg 1).  Levels from 1:
    # {1},{0},{2,3,4}; the last level's smallest (deg,index) is 2, whose level
    # structure also has 3 levels, so start = 1.  CM: 1, 0, then 0's list in
    # (deg,index) order 2, 3, 4.  Reversed: 4, 3, 2, 0, 1.
    edges = [(0, k) for k in range(1, 5)]
    rp, c = _csr_from_edges(5, edges)
    assert R.rcm(5, rp, c).tolist() == [4, 3, 2, 0, 1]


def test_pseudo_peripheral_moves_start_by_hand():
    # path 2-0-1-3 plus pendant 4 on 1 (edges 0-2, 0-1, 1-3, 1-4).
    # deg: 0:2, 1:3, 2:1, 3:1, 4:1.  Seed = 2.  Levels from 2: {2},{0},{1},{3,4}
    # (4 levels); last level min (deg,index) = 3; levels from 3: {3},{1},{0,4},{2}
    # also 4 levels -> start stays 2.  CM from 2: 2, 0, 1, then 1's unvisited
    # neighbours in (deg,index) order: 3, 4.  Reversed: 4, 3, 1, 0, 2.
    rp, c = _csr_from_edges(5, [(0, 2), (0, 1), (1, 3), (1, 4)])
    assert R.rcm(5, rp, c).tolist() == [4, 3, 1, 0, 2]


def test_pseudo_peripheral_improves_start_by_hand():
    # "broom": path 0-1-2-3 with extra leaves 4,5 on vertex 0, and leaf 6 on 1.
    # deg: 0:3, 1:3, 2:2, 3:1, 4:1, 5:1, 6:1.  Seed = 3 (deg 1, smallest index).
    # Levels from 3: {3},{2},{1},{0,6},{4,5}: 5 levels.  Last level min = 4;
    # levels from 4: {4},{0},{1,5},{2,6},{3}: 5 levels, not more -> start 3.
    # CM from 3: 3, 2, 1, then 1's list by (deg,index): 6 (deg 1), 0 (deg 3);
    # then 6 has nothing new, 0 adds 4, 5.  Order 3,2,1,6,0,4,5; reversed.
    edges = [(0, 1), (1, 2), (2, 3), (0, 4), (0, 5), (1, 6)]
    rp, c = _csr_from_edges(7, edges)
    assert R.rcm(7, rp, c).tolist() == [5, 4, 0, 6, 1, 2, 3]


def test_george_liu_search_changes_start_by_hand():
    # a "lollipop": triangle 0-1-2 with a tail 2-3-4.  deg: 0:2, 1:2, 2:3, 3:2,
    # 4:1.  Seed is 4 (deg 1).  Levels from 4: {4},{3},{2},{0,1} (4 levels);
    # last level min (deg,index) = 0; levels from 0: {0},{1,2},{3},{4} also 4
    # -> start 4.  CM: 4, 3, 2, then 2's list (deg,index): 0, 1.  Reverse:
    # 1, 0, 2, 3, 4.
    edges = [(0, 1), (1, 2), (0, 2), (2, 3), (3, 4)]
    rp, c = _csr_from_edges(5, edges)
    assert R.rcm(5, rp, c).tolist() == [1, 0, 2, 3, 4]


def test_search_moves_to_farther_vertex_by_hand():
    # graph 0-1, 1-2, 2-3, 1-4, 4-5; deg: 0:1, 1:3, 2:2, 3:1, 4:2, 5:1.
    # Seed 0.  Levels from 0: {0},{1},{2,4},{3,5}: 4 levels; the last level's
    # smallest (deg,index) is 3; levels from 3: {3},{2},{1},{0,4},{5}: 5
    # levels -> move to 3.  From 3 the last level is {5}: levels from 5:
    # {5},{4},{1},{0,2},{3}: 5, not more -> start 3.  CM from 3: 3, 2, 1,
    # then 1's list by (deg,index): 0 (deg 1), 4 (deg 2); then 4 adds 5.
    # Order 3,2,1,0,4,5; reversed 5,4,0,1,2,3.
    edges = [(0, 1), (1, 2), (2, 3), (1, 4), (4, 5)]
    rp, c = _csr_from_edges(6, edges)
    assert R.rcm(6, rp, c).tolist() == [5, 4, 0, 1, 2, 3]


def test_components_in_discovery_order_by_hand():
    # two components: triangle {0,1,2} (deg 2 each) and edge {3,4} (deg 1).
    # First seed is 3 (deg 1): CM 3, 4.  Then seed 0: levels {0},{1,2}; last
    # level min is 1 with levels {1},{0,2} (2 levels, not more) -> start 0,
    # CM 0, 1, 2.  Order 3,4,0,1,2, reversed 2,1,0,4,3.
    edges = [(0, 1), (1, 2), (2, 0), (3, 4)]
    rp, c = _csr_from_edges(5, edges)
    assert R.rcm(5, rp, c).tolist() == [2, 1, 0, 4, 3]


def test_one_sided_pattern_is_symmetrised():
    # only the upper triangle stored: the graph is still the path 0-1-2-3
    rp, c = _csr_from_edges(4, [(0, 1), (1, 2), (2, 3)])
    perm = R.rcm(4, rp, c)
    assert perm.tolist() == [3, 2, 1, 0]


def _bandwidth_after(n, rp, c, perm):
    rp2, c2, _ = S.permute_symmetric(n, rp, c, np.zeros(len(c)), perm)
    return S.fit(n, n, rp2, c2)[0]


@pytest.mark.parametrize("seed", range(3))
def test_scrambled_path_returns_to_bandwidth_1(seed):
    n = 500
    rp = np.zeros(n + 1, dtype=np.int32)
    rows = []
    for i in range(n):
        rows.append([j for j in (i - 1, i, i + 1) if 0 <= j < n])
    rp[1:] = np.cumsum([len(r) for r in rows])
    c = np.array([x for r in rows for x in r], dtype=np.int32)
    from workloads.matrices import CSR
    A = scramble_symmetric(CSR(n, n, rp, c, np.ones(len(c))), seed)
    assert S.fit(n, n, A.rowptr, A.colids)[0] > 100
    perm = R.rcm(n, A.rowptr, A.colids)
    assert np.array_equal(np.sort(perm), np.arange(n))
    assert _bandwidth_after(n, A.rowptr, A.colids, perm) == 1


@pytest.mark.parametrize("N", [8, 20, 33])
def test_scrambled_grid_bandwidth(N):
    A = scramble_symmetric(laplace_2d_5pt(N), 11)
    perm = R.rcm(A.nrows, A.rowptr, A.colids)
    # a corner start gives anti-diagonal levels of at most N vertices
    assert _bandwidth_after(A.nrows, A.rowptr, A.colids, perm) <= N + 1


def test_scrambled_banded_rcm_bandwidth_and_scipy_start():
    A = random_banded(60000, 9, half_band=2000)
    Q = scramble_symmetric(A, 3)
    n = Q.nrows
    assert S.fit(n, n, Q.rowptr, Q.colids)[0] > 50000
    perm = R.rcm(n, Q.rowptr, Q.colids)
    w = _bandwidth_after(n, Q.rowptr, Q.colids, perm)
    # random banded graphs come back with about two band half-widths: BFS
    # levels are about one half-width wide and edges join adjacent levels
    assert w < 2.5 * 2000
    # scipy's RCM (different start rule): ours is at least as narrow here
    M = sp.csr_matrix((np.ones(Q.nnz), Q.colids, Q.rowptr), shape=(n, n))
    ps = reverse_cuthill_mckee(M, symmetric_mode=False)
    assert w <= _bandwidth_after(n, Q.rowptr, Q.colids, ps)


def _fifo_cm(n, adj_ptr, adj, start):
    """Plain queue Cuthill-McKee of one component (for the vectorised BFS)."""
    seen = {start}
    q = collections.deque([start])
    out = []
    while q:
        v = q.popleft()
        out.append(v)
        for u in adj[adj_ptr[v]:adj_ptr[v + 1]]:
            if u not in seen:
                seen.add(u)
                q.append(u)
    return out


@pytest.mark.parametrize("seed", range(8))
def test_level_bfs_equals_fifo_queue(seed):
    A = random_csr(80, 80, seed, mean_len=2.5, empty_frac=0.05)
    adj_ptr, adj, deg = R.symmetric_graph(80, A.rowptr, A.colids)
    marks = R._Marks(80)
    for start in range(0, 80, 7):
        levels = R.level_structure(start, adj_ptr, adj, marks)
        assert np.concatenate(levels).tolist() == _fifo_cm(80, adj_ptr, adj, start)


def test_symmetric_graph_degrees_brute_force():
    A = random_csr(50, 50, 4, mean_len=3, dup_frac=0.3)
    adj_ptr, adj, deg = R.symmetric_graph(50, A.rowptr, A.colids)
    nb = [set() for _ in range(50)]
    rows = S.entry_rows(50, A.rowptr)
    for r, c in zip(rows, A.colids):
        if r != c:
            nb[r].add(int(c))
            nb[c].add(int(r))
    assert deg.tolist() == [len(s) for s in nb]
    for v in range(50):
        lst = adj[adj_ptr[v]:adj_ptr[v + 1]].tolist()
        assert sorted(lst) == sorted(nb[v])
        assert lst == sorted(lst, key=lambda u: (len(nb[u]), u))


def test_perm_is_permutation_with_isolated_and_empty():
    A = random_csr(300, 300, 2, mean_len=1.0, empty_frac=0.5)
    perm = R.rcm(300, A.rowptr, A.colids)
    assert np.array_equal(np.sort(perm), np.arange(300))


def test_midpoint_refine_by_hand():
    # path 0-1-2-3 ordered [1, 0, 3, 2]: positions 1:0 0:1 3:2 2:3, edge 1-2
    # spans 3.  Keys (min + max neighbour position): v0: 0+0 = 0, v1: 1+3 = 4,
    # v2: 0+2 = 2, v3: 3+3 = 6 -> order [0, 2, 1, 3] with bandwidth 2 < 3.
    rp, c = _csr_from_edges(4, [(0, 1), (1, 2), (2, 3)])
    perm, w, sweeps = R.midpoint_refine(4, rp, c, [1, 0, 3, 2], limit=3)
    assert perm.tolist() == [0, 2, 1, 3] and w == 2 and sweeps == 1


def test_midpoint_refine_keeps_narrowest_when_nothing_fits():
    # path 0-1-2-3-4 ordered [0, 2, 4, 1, 3] (bandwidth 3): one sweep gives
    # [1, 3, 0, 2, 4] (bandwidth 3), the next returns to the start; with
    # limit 3 nothing fits and the earliest narrowest order is the input.
    rp, c = _csr_from_edges(5, [(0, 1), (1, 2), (2, 3), (3, 4)])
    perm, w, sweeps = R.midpoint_refine(5, rp, c, [0, 2, 4, 1, 3], limit=3, max_sweeps=4)
    assert perm.tolist() == [0, 2, 4, 1, 3] and w == 3 and sweeps == 4


def test_midpoint_refine_brings_scrambled_band_into_range():
    # RCM leaves a random band at about twice its half-width; refinement
    # brings it below 1.5 half-widths
    A = random_banded(60000, 9, half_band=2000)
    Q = scramble_symmetric(A, 3)
    n = Q.nrows
    perm = R.rcm(n, Q.rowptr, Q.colids)
    assert _bandwidth_after(n, Q.rowptr, Q.colids, perm) > 3000
    p2, w, sweeps = R.midpoint_refine(n, Q.rowptr, Q.colids, perm, limit=3000)
    assert w < 3000 and 1 <= sweeps <= 32
    assert w == _bandwidth_after(n, Q.rowptr, Q.colids, p2)
    assert np.array_equal(np.sort(p2), np.arange(n))
