// Host-side sparsity features for the kernel-variant selector.  Each feature
// is a plain statistic of the int32 CSR arrays, computed in double and
// returned as float:
//   0 log2(nrows + 1)        6 log2(w + 1)            12 std / mean row length
//   1 log2(nnz + 1)          7 w / max(ncols, 1)      13 fraction of rows >= 64
//   2 mean row length        8 w >= 2^15 ? 1 : 0      14 log2(ncols + 1)
//   3 std of row lengths     9 nrhs                   15 fraction of adjacent
//   4 log2(max row len + 1) 10 log2(mean |c-r| + 1)      entry pairs in a row
//   5 fraction of empty rows 11 fraction |c-r| <= 64      with column step 1
// (w is the bandwidth of Eq. 2; std is the population standard deviation.)
#include <cmath>
#include <cstdint>

#include "damn.h"
#include "damn_internal.h"

extern "C" int damn_features(int32_t nrows, int32_t ncols, const int32_t* rowptr,
                             const int32_t* colids, int32_t nrhs, float* feat) {
  if (feat == nullptr || nrhs < 1) return DAMN_ERR_INVALID_ARG;
  const int st = damn::check_csr(nrows, ncols, rowptr, colids);
  if (st != DAMN_OK) return st;
  const int64_t nnz = rowptr[nrows];
  const double n = nrows > 0 ? double(nrows) : 1.0;
  double sum_sq = 0, sum_d = 0;
  int64_t max_len = 0, empty = 0, long_rows = 0, near = 0, pairs = 0, unit = 0, w = 0;
  for (int32_t r = 0; r < nrows; ++r) {
    const int64_t len = rowptr[r + 1] - rowptr[r];
    sum_sq += double(len) * double(len);
    if (len > max_len) max_len = len;
    empty += len == 0;
    long_rows += len >= 64;
    for (int64_t i = rowptr[r]; i < rowptr[r + 1]; ++i) {
      const int64_t d = std::llabs(int64_t(colids[i]) - r);
      sum_d += double(d);
      if (d > w) w = d;
      near += d <= 64;
      if (i > rowptr[r]) {
        ++pairs;
        unit += int64_t(colids[i]) - colids[i - 1] == 1;
      }
    }
  }
  const double mean = double(nnz) / n;
  const double var = sum_sq / n - mean * mean;
  const double sd = nrows > 0 && var > 0 ? std::sqrt(var) : 0.0;
  double f[16];
  f[0] = std::log2(double(nrows) + 1);
  f[1] = std::log2(double(nnz) + 1);
  f[2] = mean;
  f[3] = sd;
  f[4] = std::log2(double(max_len) + 1);
  f[5] = double(empty) / n;
  f[6] = std::log2(double(w) + 1);
  f[7] = double(w) / (ncols > 0 ? double(ncols) : 1.0);
  f[8] = w >= damn::kInt16BandwidthLimit ? 1.0 : 0.0;
  f[9] = double(nrhs);
  f[10] = nnz > 0 ? std::log2(sum_d / double(nnz) + 1) : 0.0;
  f[11] = nnz > 0 ? double(near) / double(nnz) : 0.0;
  f[12] = mean > 0 ? sd / mean : 0.0;
  f[13] = double(long_rows) / n;
  f[14] = std::log2(double(ncols) + 1);
  f[15] = pairs > 0 ? double(unit) / double(pairs) : 0.0;
  for (int k = 0; k < 16; ++k) feat[k] = float(f[k]);
  return DAMN_OK;
}
