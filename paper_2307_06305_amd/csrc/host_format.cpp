// Host-side preprocessing: CSR validation, bandwidth fit (Eq. 2), the DA
// transform col - row (Sec. 2, Example 1), symmetric permutation and the
// encode entry point.  Pure C++; no GPU calls.
#include <algorithm>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "damn.h"
#include "damn_internal.h"

namespace damn {

int check_csr(int32_t nrows, int32_t ncols, const int32_t* rowptr,
              const int32_t* colids) {
  if (nrows < 0 || ncols < 0 || rowptr == nullptr) return DAMN_ERR_INVALID_ARG;
  if (rowptr[0] != 0) return DAMN_ERR_BAD_CSR;
  for (int32_t r = 0; r < nrows; ++r)
    if (rowptr[r + 1] < rowptr[r]) return DAMN_ERR_BAD_CSR;
  const int64_t nnz = rowptr[nrows];
  if (nnz > 0 && colids == nullptr) return DAMN_ERR_INVALID_ARG;
  int32_t bad = 0;
  parallel_for(nnz, [&](int64_t b, int64_t e) {
    int32_t local = 0;
    for (int64_t i = b; i < e; ++i)
      local |= (colids[i] < 0) | (colids[i] >= ncols);
    if (local) __atomic_store_n(&bad, 1, __ATOMIC_RELAXED);
  });
  return bad ? DAMN_ERR_BAD_CSR : DAMN_OK;
}

// Bandwidth split into its two sides: lo = max(r - c), hi = max(c - r).
void bandwidth(int32_t nrows, const int32_t* rowptr, const int32_t* colids,
               int64_t* lo, int64_t* hi) {
  std::mutex m;
  int64_t glo = 0, ghi = 0;
  parallel_for(nrows, [&](int64_t b, int64_t e) {
    int64_t l = 0, h = 0;
    for (int64_t r = b; r < e; ++r)
      for (int64_t i = rowptr[r]; i < rowptr[r + 1]; ++i) {
        const int64_t d = int64_t(colids[i]) - r;
        if (d > h) h = d;
        if (-d > l) l = -d;
      }
    std::lock_guard<std::mutex> g(m);
    glo = std::max(glo, l);
    ghi = std::max(ghi, h);
  });
  *lo = glo;
  *hi = ghi;
}

// Permuted copy P A P^T (square): new row i is old row perm[i], columns
// relabelled by the inverse permutation, each row ordered by new column with
// ties in old order.
int permute_symmetric(int32_t n, const int32_t* rowptr, const int32_t* colids,
                      const double* vals, const int32_t* perm,
                      std::vector<int32_t>& rp_out, std::vector<int32_t>& cols_out,
                      std::vector<double>& vals_out) {
  try {
    std::vector<int32_t> inv(n);
    for (int32_t i = 0; i < n; ++i) inv[perm[i]] = i;
    rp_out.assign(size_t(n) + 1, 0);
    for (int32_t i = 0; i < n; ++i)
      rp_out[i + 1] = rp_out[i] + (rowptr[perm[i] + 1] - rowptr[perm[i]]);
    const int64_t nnz = rp_out[n];
    cols_out.resize(nnz);
    vals_out.resize(nnz);
    parallel_for(n, [&](int64_t b, int64_t e) {
      std::vector<std::pair<int32_t, int32_t>> row;  // (new col, old position)
      for (int64_t i = b; i < e; ++i) {
        const int32_t src = perm[i];
        const int32_t s = rowptr[src], len = rowptr[src + 1] - s;
        row.resize(len);
        for (int32_t k = 0; k < len; ++k) row[k] = {inv[colids[s + k]], k};
        // (new col, old position) is unique, so sort == stable sort by col
        std::sort(row.begin(), row.end());
        const int32_t d = rp_out[i];
        for (int32_t k = 0; k < len; ++k) {
          cols_out[d + k] = row[k].first;
          vals_out[d + k] = vals[s + row[k].second];
        }
      }
    });
  } catch (const std::bad_alloc&) {
    return DAMN_ERR_ALLOC;
  }
  return DAMN_OK;
}

}  // namespace damn

using namespace damn;

extern "C" int damn_fit_check(int32_t nrows, int32_t ncols, const int32_t* rowptr,
                              const int32_t* colids, int32_t* w, int32_t* lo,
                              int32_t* hi, int32_t* fits) {
  int st = check_csr(nrows, ncols, rowptr, colids);
  if (st != DAMN_OK) return st;
  int64_t l, h;
  bandwidth(nrows, rowptr, colids, &l, &h);
  const int64_t ww = std::max(l, h);
  if (w) *w = int32_t(ww);
  if (lo) *lo = int32_t(l);
  if (hi) *hi = int32_t(h);
  if (fits) *fits = ww < kInt16BandwidthLimit;
  return DAMN_OK;
}

extern "C" int damn_encode(int32_t nrows, int32_t ncols, const int32_t* rowptr,
                           const int32_t* colids, const double* vals,
                           int32_t allow_rcm, int32_t* rowptr_out, int16_t* off_out,
                           double* vals_out, int32_t* perm_out, int32_t* permuted,
                           int32_t* w_out) {
  int st = check_csr(nrows, ncols, rowptr, colids);
  if (st != DAMN_OK) return st;
  const int64_t nnz = rowptr[nrows];
  if (rowptr_out == nullptr || permuted == nullptr || w_out == nullptr ||
      (nnz > 0 && (vals == nullptr || off_out == nullptr || vals_out == nullptr)))
    return DAMN_ERR_INVALID_ARG;
  int64_t l, h;
  bandwidth(nrows, rowptr, colids, &l, &h);
  int64_t ww = std::max(l, h);
  if (ww < kInt16BandwidthLimit) {
    std::memcpy(rowptr_out, rowptr, sizeof(int32_t) * (size_t(nrows) + 1));
    parallel_for(nrows, [&](int64_t b, int64_t e) {
      for (int64_t r = b; r < e; ++r)
        for (int64_t i = rowptr[r]; i < rowptr[r + 1]; ++i) {
          off_out[i] = int16_t(int64_t(colids[i]) - r);
          vals_out[i] = vals[i];
        }
    });
    if (perm_out)
      for (int32_t i = 0; i < nrows; ++i) perm_out[i] = i;
    *permuted = 0;
    *w_out = int32_t(ww);
    return DAMN_OK;
  }
  if (!allow_rcm || nrows != ncols) {
    *w_out = int32_t(ww);
    return DAMN_ERR_NO_FIT;
  }
  std::vector<int32_t> perm, rp2, c2;
  std::vector<double> v2;
  try {
    perm.resize(nrows);
  } catch (const std::bad_alloc&) {
    return DAMN_ERR_ALLOC;
  }
  st = damn_rcm(nrows, rowptr, colids, perm.data());
  if (st != DAMN_OK) return st;
  // the RCM order alone may stay too wide: refine it
  int64_t wr = 0;
  try {
    st = refine_bandwidth(nrows, rowptr, colids, perm.data(), kRefineSweeps,
                          kInt16BandwidthLimit, &wr);
  } catch (const std::bad_alloc&) {
    return DAMN_ERR_ALLOC;
  }
  if (st != DAMN_OK) {
    *w_out = int32_t(wr);
    return st;
  }
  st = permute_symmetric(nrows, rowptr, colids, vals, perm.data(), rp2, c2, v2);
  if (st != DAMN_OK) return st;
  bandwidth(nrows, rp2.data(), c2.data(), &l, &h);
  ww = std::max(l, h);
  *w_out = int32_t(ww);
  if (ww >= kInt16BandwidthLimit) return DAMN_ERR_NO_FIT;
  std::memcpy(rowptr_out, rp2.data(), sizeof(int32_t) * (size_t(nrows) + 1));
  parallel_for(nrows, [&](int64_t b, int64_t e) {
    for (int64_t r = b; r < e; ++r)
      for (int64_t i = rp2[r]; i < rp2[r + 1]; ++i) {
        off_out[i] = int16_t(int64_t(c2[i]) - r);
        vals_out[i] = v2[i];
      }
  });
  if (perm_out) std::memcpy(perm_out, perm.data(), sizeof(int32_t) * size_t(nrows));
  *permuted = 1;
  return DAMN_OK;
}
