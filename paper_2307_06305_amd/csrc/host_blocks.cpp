// Host-side BSR and DA-BSR encoding (diagonal addressing applied to block
// storage, Sec. 1).  Pure C++; no GPU calls.
//
// A matrix cut into b x b blocks stores, per block row, the nonzero blocks in
// ascending block column with their b*b values row-major.  A block is stored
// when a pattern entry (stored zeros included) falls into it; repeated
// entries add up, in storage order.  DA-BSR keeps the block offset bc - br in
// int16 (block bandwidth below 2^15); BSR keeps bc in int32.
#include <algorithm>
#include <cstdint>
#include <new>
#include <vector>

#include "damn.h"
#include "damn_internal.h"

namespace damn {
namespace {

// Sorted distinct block columns of block row br.
void block_columns(int32_t br, int32_t b, const int32_t* rowptr, const int32_t* colids,
                   std::vector<int32_t>& out) {
  out.clear();
  for (int32_t i = 0; i < b; ++i) {
    const int32_t r = br * b + i;
    for (int32_t k = rowptr[r]; k < rowptr[r + 1]; ++k) out.push_back(colids[k] / b);
  }
  std::sort(out.begin(), out.end());
  out.erase(std::unique(out.begin(), out.end()), out.end());
}

int check_blocks(int32_t nrows, int32_t ncols, const int32_t* rowptr, const int32_t* colids,
                 int32_t b) {
  if (b < 1 || nrows < 0 || ncols < 0 || nrows % b != 0 || ncols % b != 0)
    return DAMN_ERR_INVALID_ARG;
  return check_csr(nrows, ncols, rowptr, colids);
}

}  // namespace
}  // namespace damn

using namespace damn;

extern "C" {

int damn_bsr_count(int32_t nrows, int32_t ncols, const int32_t* rowptr, const int32_t* colids,
                   int32_t b, int64_t* nnzb, int32_t* wb) {
  if (nnzb == nullptr || wb == nullptr) return DAMN_ERR_INVALID_ARG;
  const int st = check_blocks(nrows, ncols, rowptr, colids, b);
  if (st != DAMN_OK) return st;
  const int32_t nbr = nrows / b;
  std::mutex m;
  int64_t total = 0, wmax = 0;
  try {
    parallel_for(nbr, [&](int64_t lo, int64_t hi) {
      std::vector<int32_t> cols;
      int64_t cnt = 0, w = 0;
      for (int64_t br = lo; br < hi; ++br) {
        block_columns(int32_t(br), b, rowptr, colids, cols);
        cnt += int64_t(cols.size());
        for (int32_t bc : cols) w = std::max<int64_t>(w, bc > br ? bc - br : br - bc);
      }
      std::lock_guard<std::mutex> g(m);
      total += cnt;
      wmax = std::max(wmax, w);
    }, 1024);
  } catch (const std::bad_alloc&) {
    return DAMN_ERR_ALLOC;
  }
  *nnzb = total;
  *wb = int32_t(wmax);
  return DAMN_OK;
}

int damn_bsr_encode(int32_t nrows, int32_t ncols, const int32_t* rowptr, const int32_t* colids,
                    const double* vals, int32_t b, int32_t format, int32_t* browptr_out,
                    void* bidx_out, double* bvals_out) {
  if (format != DAMN_FORMAT_DABSR16 && format != DAMN_FORMAT_BSR32) return DAMN_ERR_INVALID_ARG;
  int64_t nnzb = 0;
  int32_t wb = 0;
  int st = damn_bsr_count(nrows, ncols, rowptr, colids, b, &nnzb, &wb);
  if (st != DAMN_OK) return st;
  if (browptr_out == nullptr || (nnzb > 0 && (bidx_out == nullptr || bvals_out == nullptr)) ||
      (rowptr[nrows] > 0 && vals == nullptr))
    return DAMN_ERR_INVALID_ARG;
  if (nnzb >= (int64_t(1) << 31)) return DAMN_ERR_UNSUPPORTED;
  if (format == DAMN_FORMAT_DABSR16 && wb >= kInt16BandwidthLimit) return DAMN_ERR_NO_FIT;
  const int32_t nbr = nrows / b;
  try {
    // block row lengths, then the prefix sum
    std::vector<int32_t> len(size_t(nbr) + 1, 0);
    parallel_for(nbr, [&](int64_t lo, int64_t hi) {
      std::vector<int32_t> cols;
      for (int64_t br = lo; br < hi; ++br) {
        block_columns(int32_t(br), b, rowptr, colids, cols);
        len[br] = int32_t(cols.size());
      }
    }, 1024);
    browptr_out[0] = 0;
    for (int32_t br = 0; br < nbr; ++br) browptr_out[br + 1] = browptr_out[br] + len[br];
    const int64_t bb = int64_t(b) * b;
    parallel_for(nbr, [&](int64_t lo, int64_t hi) {
      std::vector<int32_t> cols;
      for (int64_t br = lo; br < hi; ++br) {
        block_columns(int32_t(br), b, rowptr, colids, cols);
        const int64_t base = browptr_out[br];
        for (size_t q = 0; q < cols.size(); ++q) {
          if (format == DAMN_FORMAT_DABSR16)
            static_cast<int16_t*>(bidx_out)[base + int64_t(q)] = int16_t(cols[q] - br);
          else
            static_cast<int32_t*>(bidx_out)[base + int64_t(q)] = cols[q];
        }
        double* bv = bvals_out + base * bb;
        std::fill(bv, bv + int64_t(cols.size()) * bb, 0.0);
        // entries in storage order, so repeated entries add up in that order
        for (int32_t i = 0; i < b; ++i) {
          const int32_t r = int32_t(br) * b + i;
          for (int32_t k = rowptr[r]; k < rowptr[r + 1]; ++k) {
            const int32_t c = colids[k];
            const int64_t q = std::lower_bound(cols.begin(), cols.end(), c / b) - cols.begin();
            bv[q * bb + int64_t(i) * b + (c % b)] += vals[k];
          }
        }
      }
    }, 1024);
  } catch (const std::bad_alloc&) {
    return DAMN_ERR_ALLOC;
  }
  return DAMN_OK;
}

}  // extern "C"
