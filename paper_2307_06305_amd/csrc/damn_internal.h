// Internal declarations shared by the library's translation units.
#pragma once

#include <algorithm>
#include <cstdint>
#include <functional>
#include <mutex>
#include <thread>
#include <vector>

namespace damn {

// 16-bit DA offsets are used when the bandwidth is below 2^15.
constexpr int64_t kInt16BandwidthLimit = 32768;

// Number of host worker threads (DAMN_THREADS overrides; capped at 64).
int host_threads();

// Run fn(begin, end) over [0, n) split into contiguous chunks on worker
// threads; small ranges run on the calling thread.
inline void parallel_for(int64_t n, const std::function<void(int64_t, int64_t)>& fn,
                         int64_t grain = 1 << 16) {
  const int nt = int(std::min<int64_t>(host_threads(), (n + grain - 1) / grain));
  if (nt <= 1) {
    if (n > 0) fn(0, n);
    return;
  }
  std::vector<std::thread> th;
  th.reserve(nt);
  const int64_t chunk = (n + nt - 1) / nt;
  for (int t = 0; t < nt; ++t) {
    const int64_t b = t * chunk, e = std::min(n, b + chunk);
    if (b >= e) break;
    th.emplace_back(fn, b, e);
  }
  for (auto& x : th) x.join();
}

int check_csr(int32_t nrows, int32_t ncols, const int32_t* rowptr,
              const int32_t* colids);
void bandwidth(int32_t nrows, const int32_t* rowptr, const int32_t* colids,
               int64_t* lo, int64_t* hi);
int refine_bandwidth(int32_t n, const int32_t* rowptr, const int32_t* colids, int32_t* perm,
                     int32_t max_sweeps, int64_t limit, int64_t* w_out);
constexpr int32_t kRefineSweeps = 32;

// The storage grid of Fig. 3 (host_grid.cpp): bytes of a format's index and
// of a scalar type (0 for an unknown enum value), and whether a format holds
// DA offsets.
int index_bytes(int32_t format);
bool format_is_da(int32_t format);
bool format_is_block(int32_t format);
bool format_is_coo(int32_t format);
int value_bytes(int32_t dtype);

}  // namespace damn
