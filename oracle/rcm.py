"""Reverse Cuthill-McKee bandwidth reduction (cited in Sec. 2, Example 2 and
Sec. 3; the paper fixes no details).

Reading used here (every choice the paper leaves open):

1. The graph is the pattern of A + A^T, repeated edges merged, self loops
   dropped.  Explicitly stored zeros are edges.
2. deg(v) is the number of distinct neighbours of v.  Each adjacency list is
   ordered by (deg, index), ascending.
3. Components are taken one at a time: the next component is the one holding
   the unvisited vertex with the smallest (deg, index).
4. Its start vertex comes from the George-Liu pseudo-peripheral search:
   r = that vertex; form r's BFS level structure; among the last level take
   the vertex x with the smallest (deg, index) and form x's level structure;
   if x has more levels than r, set r = x and repeat, else keep r.
5. Cuthill-McKee: breadth-first from r, a first-in-first-out queue, each
   dequeued vertex appending its not yet visited neighbours in adjacency-list
   order.  Components are concatenated in the order they were found.
6. The whole concatenated order is reversed; the result perm maps new
   position -> old vertex.

The BFS below works level by level: the vertices of level k+1 are, in order,
the first occurrences of not-yet-visited vertices in the concatenation of
the adjacency lists of level k (taken in level-k order).  That is exactly
the order a FIFO queue produces.
"""

from __future__ import annotations

import numpy as np


def symmetric_graph(n, rowptr, colids):
    """Adjacency of pattern(A + A^T) without self loops.

    Returns (adj_ptr[n+1], adj[m], deg[n]); each list sorted by (deg, index).
    """
    rowptr = np.asarray(rowptr, dtype=np.int64)
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(rowptr))
    cols = np.asarray(colids, dtype=np.int64)
    keep = rows != cols
    src = np.concatenate([rows[keep], cols[keep]])
    dst = np.concatenate([cols[keep], rows[keep]])
    del rows, cols, keep
    key = np.unique(src * n + dst)  # merges repeats, sorted by (src, dst)
    del src, dst
    src = key // n
    dst = key - src * n
    del key
    deg = np.bincount(src, minlength=n).astype(np.int64)
    adj_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(deg, out=adj_ptr[1:])
    # order each list by (deg[dst], dst); src stays the major key
    order = np.lexsort((dst, deg[dst], src))
    adj = dst[order]
    return adj_ptr, adj, deg


def _gather_lists(frontier, adj_ptr, adj):
    """Concatenation of the adjacency lists of `frontier`, in frontier order."""
    starts = adj_ptr[frontier]
    lens = adj_ptr[frontier + 1] - starts
    total = int(lens.sum())
    if total == 0:
        return np.empty(0, dtype=np.int64)
    base = np.repeat(starts - np.concatenate([[0], np.cumsum(lens)[:-1]]), lens)
    return adj[base + np.arange(total, dtype=np.int64)]


def _next_level(frontier, adj_ptr, adj, mark, stamp):
    """Neighbours of `frontier` not yet marked with `stamp`, in FIFO
    discovery order; marks them."""
    cand = _gather_lists(frontier, adj_ptr, adj)
    cand = cand[mark[cand] != stamp]
    if cand.size == 0:
        return cand
    _, first = np.unique(cand, return_index=True)
    nxt = cand[np.sort(first)]
    mark[nxt] = stamp
    return nxt


class _Marks:
    """Visit marks for repeated searches: each search uses a fresh stamp, so
    a search costs time proportional to its component, not to n."""

    def __init__(self, n):
        self.mark = np.zeros(n, dtype=np.int64)
        self.stamp = 1

    def fresh(self):
        self.stamp += 1
        return self.stamp


def level_structure(root, adj_ptr, adj, marks):
    """BFS level sets rooted at `root` (list of arrays, discovery order)."""
    stamp = marks.fresh()
    marks.mark[root] = stamp
    levels = [np.array([root], dtype=np.int64)]
    while True:
        nxt = _next_level(levels[-1], adj_ptr, adj, marks.mark, stamp)
        if nxt.size == 0:
            return levels
        levels.append(nxt)


def _min_deg_index(vertices, deg):
    """Vertex with the smallest (deg, index) among `vertices`."""
    d = deg[vertices]
    cands = vertices[d == d.min()]
    return int(cands.min())


def pseudo_peripheral(s0, adj_ptr, adj, deg, marks):
    """George-Liu pseudo-peripheral vertex search from s0 (reading item 4)."""
    r = s0
    levels = level_structure(r, adj_ptr, adj, marks)
    while True:
        x = _min_deg_index(levels[-1], deg)
        lx = level_structure(x, adj_ptr, adj, marks)
        if len(lx) > len(levels):
            r, levels = x, lx
        else:
            return r


def rcm(n, rowptr, colids):
    """RCM permutation (new -> old), int64 array of length n."""
    if n == 0:
        return np.empty(0, dtype=np.int64)
    adj_ptr, adj, deg = symmetric_graph(n, rowptr, colids)
    marks = _Marks(n)
    placed_mark = np.zeros(n, dtype=np.int64)  # stamp 1 = placed in the order
    # unvisited vertices in (deg, index) order: the next component's seed is
    # the first of them still unvisited (reading item 3)
    by_deg = np.lexsort((np.arange(n), deg))
    cursor = 0
    order = []
    placed = 0
    while placed < n:
        while placed_mark[by_deg[cursor]]:
            cursor += 1
        s0 = int(by_deg[cursor])
        r = s0 if deg[s0] == 0 else pseudo_peripheral(s0, adj_ptr, adj, deg, marks)
        placed_mark[r] = 1
        frontier = np.array([r], dtype=np.int64)
        while frontier.size:
            order.append(frontier)
            placed += frontier.size
            frontier = _next_level(frontier, adj_ptr, adj, placed_mark, 1)
    cm = np.concatenate(order)
    return cm[::-1].copy()


def graph_bandwidth(n, adj_ptr, adj, perm):
    """max |pos[u] - pos[v]| over graph edges for the order perm (new -> old);
    0 without edges.  Equals the bandwidth of P A P^T (Eq. 2)."""
    if adj.size == 0:
        return 0
    pos = np.empty(n, dtype=np.int64)
    pos[np.asarray(perm, dtype=np.int64)] = np.arange(n, dtype=np.int64)
    src = np.repeat(np.arange(n, dtype=np.int64), np.diff(adj_ptr))
    return int(np.abs(pos[src] - pos[adj]).max())


def midpoint_refine(n, rowptr, colids, perm, limit=2**15, max_sweeps=32):
    """Bandwidth refinement of an ordering, used when the RCM order does not
    reach bandwidth < limit (the paper reports RCM falling short on two
    matrices, Sec. 3, and gives no remedy; this is the reading used here).

    One sweep: with pos the current position of every vertex, a vertex with
    neighbours gets key = min pos + max pos over its neighbours (twice the
    midpoint of the span it must cover), an isolated vertex key = 2 pos; the
    new order sorts vertices by (key, pos).  Sweeps repeat until an order has
    bandwidth < limit.  Returns (perm, w, sweeps): the first fitting order,
    or after max_sweeps the narrowest order seen (earliest on ties).
    """
    adj_ptr, adj, deg = symmetric_graph(n, rowptr, colids)
    perm = np.asarray(perm, dtype=np.int64)
    best_perm, best_w = perm, graph_bandwidth(n, adj_ptr, adj, perm)
    if best_w < limit:
        return perm, best_w, 0
    has = deg > 0
    starts = adj_ptr[:-1][has]
    for sweep in range(1, max_sweeps + 1):
        pos = np.empty(n, dtype=np.int64)
        pos[perm] = np.arange(n, dtype=np.int64)
        p = pos[adj]
        key = 2 * pos
        if starts.size:
            key[has] = np.minimum.reduceat(p, starts) + np.maximum.reduceat(p, starts)
        perm = np.lexsort((pos, key))
        w = graph_bandwidth(n, adj_ptr, adj, perm)
        if w < best_w:
            best_perm, best_w = perm, w
        if w < limit:
            return perm, w, sweep
    return best_perm, best_w, max_sweeps
