// Reverse Cuthill-McKee on the host (the bandwidth reduction the paper applies
// before DA storage, Sec. 2 Example 2 and Sec. 3).  The paper fixes no details;
// this implementation uses:
//   graph      pattern of A + A^T, repeated edges merged, no self loops
//   adjacency  each list ordered by (degree, index)
//   components seeded by the unvisited vertex of smallest (degree, index)
//   start      George-Liu pseudo-peripheral search from that seed: move to the
//              smallest-(degree, index) vertex of the last BFS level while its
//              level structure is deeper
//   order      FIFO breadth-first Cuthill-McKee, components concatenated,
//              the whole order reversed (perm[new] = old)
#include <algorithm>
#include <cstdint>
#include <mutex>
#include <new>
#include <vector>

#include "damn.h"
#include "damn_internal.h"

namespace damn {
namespace {

struct Graph {
  int32_t n = 0;
  std::vector<int64_t> ptr;  // n + 1
  std::vector<int32_t> adj;  // merged, ordered by (deg, index)
  std::vector<int32_t> deg;
};

void build_graph(int32_t n, const int32_t* rowptr, const int32_t* colids, Graph& g) {
  g.n = n;
  // raw lists with repeats: entry (r, c), r != c, adds c to r and r to c
  std::vector<int64_t> cnt(size_t(n) + 1, 0);
  for (int32_t r = 0; r < n; ++r)
    for (int32_t i = rowptr[r]; i < rowptr[r + 1]; ++i) {
      const int32_t c = colids[i];
      if (c != r) {
        ++cnt[r + 1];
        ++cnt[c + 1];
      }
    }
  for (int32_t v = 0; v < n; ++v) cnt[v + 1] += cnt[v];
  std::vector<int32_t> raw(cnt[n]);
  {
    std::vector<int64_t> fill(cnt.begin(), cnt.end() - 1);
    for (int32_t r = 0; r < n; ++r)
      for (int32_t i = rowptr[r]; i < rowptr[r + 1]; ++i) {
        const int32_t c = colids[i];
        if (c != r) {
          raw[fill[r]++] = c;
          raw[fill[c]++] = r;
        }
      }
  }
  // merge repeats per list
  g.deg.assign(n, 0);
  parallel_for(n, [&](int64_t b, int64_t e) {
    for (int64_t v = b; v < e; ++v) {
      int32_t* s = raw.data() + cnt[v];
      int32_t* t = raw.data() + cnt[v + 1];
      std::sort(s, t);
      g.deg[v] = int32_t(std::unique(s, t) - s);
    }
  }, 4096);
  g.ptr.assign(size_t(n) + 1, 0);
  for (int32_t v = 0; v < n; ++v) g.ptr[v + 1] = g.ptr[v] + g.deg[v];
  g.adj.resize(g.ptr[n]);
  const int32_t* deg = g.deg.data();
  parallel_for(n, [&](int64_t b, int64_t e) {
    for (int64_t v = b; v < e; ++v) {
      int32_t* d = g.adj.data() + g.ptr[v];
      std::copy(raw.data() + cnt[v], raw.data() + cnt[v] + deg[v], d);
      std::sort(d, d + deg[v], [deg](int32_t a, int32_t c) {
        return deg[a] != deg[c] ? deg[a] < deg[c] : a < c;
      });
    }
  }, 4096);
}

inline bool less_deg_index(const Graph& g, int32_t a, int32_t b) {
  return g.deg[a] != g.deg[b] ? g.deg[a] < g.deg[b] : a < b;
}

// BFS level structure from root using stamp marks.  Returns the number of
// levels and the smallest-(deg, index) vertex of the last level.
struct LevelInfo {
  int32_t depth;
  int32_t last_min;
};

LevelInfo levels_from(const Graph& g, int32_t root, std::vector<int32_t>& mark,
                      int32_t stamp, std::vector<int32_t>& queue) {
  queue.clear();
  queue.push_back(root);
  mark[root] = stamp;
  size_t level_begin = 0, level_end = 1;
  int32_t depth = 1;
  while (true) {
    for (size_t q = level_begin; q < level_end; ++q) {
      const int32_t v = queue[q];
      for (int64_t k = g.ptr[v]; k < g.ptr[v + 1]; ++k) {
        const int32_t u = g.adj[k];
        if (mark[u] != stamp) {
          mark[u] = stamp;
          queue.push_back(u);
        }
      }
    }
    if (queue.size() == level_end) break;
    level_begin = level_end;
    level_end = queue.size();
    ++depth;
  }
  int32_t best = queue[level_begin];
  for (size_t q = level_begin + 1; q < level_end; ++q)
    if (less_deg_index(g, queue[q], best)) best = queue[q];
  return {depth, best};
}

// max |pos[u] - pos[v]| over graph edges
int64_t graph_bandwidth(const Graph& g, const std::vector<int32_t>& pos) {
  std::mutex m;
  int64_t w = 0;
  parallel_for(g.n, [&](int64_t b, int64_t e) {
    int64_t local = 0;
    for (int64_t v = b; v < e; ++v)
      for (int64_t k = g.ptr[v]; k < g.ptr[v + 1]; ++k) {
        const int64_t d = int64_t(pos[g.adj[k]]) - pos[v];
        local = std::max(local, d < 0 ? -d : d);
      }
    std::lock_guard<std::mutex> l(m);
    w = std::max(w, local);
  }, 4096);
  return w;
}

}  // namespace

// Midpoint refinement sweeps (see damn_refine_bandwidth).  perm is replaced
// by the first order with bandwidth < limit, or by the narrowest order seen.
int refine_bandwidth(int32_t n, const int32_t* rowptr, const int32_t* colids, int32_t* perm,
                     int32_t max_sweeps, int64_t limit, int64_t* w_out) {
  Graph g;
  build_graph(n, rowptr, colids, g);
  std::vector<int32_t> pos(n), cur(perm, perm + n), best(perm, perm + n);
  for (int32_t i = 0; i < n; ++i) pos[cur[i]] = i;
  int64_t best_w = graph_bandwidth(g, pos);
  if (best_w >= limit) {
    std::vector<std::pair<int64_t, int32_t>> keyed(n);
    for (int32_t sweep = 1; sweep <= max_sweeps; ++sweep) {
      parallel_for(n, [&](int64_t b, int64_t e) {
        for (int64_t v = b; v < e; ++v) {
          int64_t key = 2 * int64_t(pos[v]);
          if (g.ptr[v + 1] > g.ptr[v]) {
            int32_t mn = pos[g.adj[g.ptr[v]]], mx = mn;
            for (int64_t k = g.ptr[v] + 1; k < g.ptr[v + 1]; ++k) {
              mn = std::min(mn, pos[g.adj[k]]);
              mx = std::max(mx, pos[g.adj[k]]);
            }
            key = int64_t(mn) + mx;
          }
          // (key, current position) is unique per vertex
          keyed[pos[v]] = {key, int32_t(v)};
        }
      }, 4096);
      // keyed is indexed by current position, so sorting by key and then by
      // index orders ties by current position
      std::vector<int32_t> order(n);
      for (int32_t i = 0; i < n; ++i) order[i] = i;
      std::sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
        return keyed[a].first != keyed[b].first ? keyed[a].first < keyed[b].first : a < b;
      });
      for (int32_t i = 0; i < n; ++i) cur[i] = keyed[order[i]].second;
      for (int32_t i = 0; i < n; ++i) pos[cur[i]] = i;
      const int64_t w = graph_bandwidth(g, pos);
      if (w < best_w) {
        best_w = w;
        best = cur;
      }
      if (w < limit) break;
    }
  }
  std::copy(best.begin(), best.end(), perm);
  *w_out = best_w;
  return best_w < limit ? DAMN_OK : DAMN_ERR_NO_FIT;
}

}  // namespace damn

using namespace damn;

extern "C" int damn_refine_bandwidth(int32_t n, const int32_t* rowptr, const int32_t* colids,
                                     int32_t* perm, int32_t max_sweeps, int32_t limit,
                                     int32_t* w_out) {
  if ((perm == nullptr && n > 0) || w_out == nullptr || max_sweeps < 0 || limit < 1)
    return DAMN_ERR_INVALID_ARG;
  int st = check_csr(n, n, rowptr, colids);
  if (st != DAMN_OK) return st;
  // perm must be a permutation of 0..n-1
  std::vector<char> seen(n, 0);
  for (int32_t i = 0; i < n; ++i) {
    if (perm[i] < 0 || perm[i] >= n || seen[perm[i]]) return DAMN_ERR_INVALID_ARG;
    seen[perm[i]] = 1;
  }
  int64_t w = 0;
  try {
    st = refine_bandwidth(n, rowptr, colids, perm, max_sweeps, limit, &w);
  } catch (const std::bad_alloc&) {
    return DAMN_ERR_ALLOC;
  }
  *w_out = int32_t(w);
  return st;
}

extern "C" int damn_rcm(int32_t n, const int32_t* rowptr, const int32_t* colids,
                        int32_t* perm) {
  if (perm == nullptr && n > 0) return DAMN_ERR_INVALID_ARG;
  int st = check_csr(n, n, rowptr, colids);
  if (st != DAMN_OK) return st;
  if (n == 0) return DAMN_OK;
  try {
    Graph g;
    build_graph(n, rowptr, colids, g);
    // vertices by (deg, index): the next unplaced one seeds a component
    std::vector<int32_t> by_deg(n);
    for (int32_t v = 0; v < n; ++v) by_deg[v] = v;
    std::stable_sort(by_deg.begin(), by_deg.end(),
                     [&](int32_t a, int32_t b) { return g.deg[a] < g.deg[b]; });
    std::vector<int32_t> mark(n, 0), queue;
    queue.reserve(n);
    std::vector<char> placed(n, 0);
    std::vector<int32_t> order;
    order.reserve(n);
    int32_t stamp = 0;
    size_t cursor = 0;
    while (order.size() < size_t(n)) {
      while (placed[by_deg[cursor]]) ++cursor;
      const int32_t s0 = by_deg[cursor];
      int32_t r = s0;
      if (g.deg[s0] > 0) {
        LevelInfo cur = levels_from(g, r, mark, ++stamp, queue);
        while (true) {
          const int32_t x = cur.last_min;
          LevelInfo nx = levels_from(g, x, mark, ++stamp, queue);
          if (nx.depth > cur.depth) {
            r = x;
            cur = nx;
          } else {
            break;
          }
        }
      }
      // Cuthill-McKee breadth-first from r
      size_t head = order.size();
      order.push_back(r);
      placed[r] = 1;
      while (head < order.size()) {
        const int32_t v = order[head++];
        for (int64_t k = g.ptr[v]; k < g.ptr[v + 1]; ++k) {
          const int32_t u = g.adj[k];
          if (!placed[u]) {
            placed[u] = 1;
            order.push_back(u);
          }
        }
      }
    }
    for (int32_t i = 0; i < n; ++i) perm[i] = order[size_t(n) - 1 - i];
  } catch (const std::bad_alloc&) {
    return DAMN_ERR_ALLOC;
  }
  return DAMN_OK;
}
