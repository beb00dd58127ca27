// SpMM Y <- alpha*A*X + beta*Y, stream variant: the tiles of the SpMV stream
// kernel (indices, float64 values and row pointers copied into LDS with
// 16-byte direct-to-LDS loads, the entries non-temporal), then G lanes per
// row, split over the right-hand sides and the entries, accumulate all NRHS
// right-hand sides at once.  X is ncols x NRHS and Y nrows x NRHS, row-major
// (the NRHS values of a row adjacent); with PAIRS (NRHS even, X and Y 16-byte
// aligned) they move as 16-byte pairs.  Each index and value is read once
// for all right-hand sides (Sec. 4's product repeated over nrhs vectors).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "damn_device.h"
#include "damn_kernels.h"
#include "spmm_rows.h"
#include "spmv_templates.h"

namespace damn {
namespace kern {

template <typename I, bool DA, int G, int NRHS, bool PAIRS>
__global__ __launch_bounds__(256) void spmm_stream(
    const TileStart* __restrict__ tile_row, const int32_t* __restrict__ rowptr,
    const I* __restrict__ idx, const double* __restrict__ val, const double* __restrict__ X,
    double* __restrict__ Y, double alpha, double beta, int32_t read_y, int32_t cap) {
  using L = TileLds<I, double>;
  extern __shared__ __align__(16) unsigned char lds[];
  const int32_t slots = L::slots(cap);
  double* val_s = reinterpret_cast<double*>(lds);
  I* idx_s = reinterpret_cast<I*>(lds + sizeof(double) * slots);
  int32_t* rp_s = reinterpret_cast<int32_t*>(lds + (sizeof(double) + sizeof(I)) * slots);

  const uint32_t t = xcd_contiguous(blockIdx.x, gridDim.x);
  const TileStart ta = tile_row[t], tb = tile_row[t + 1];
  const int32_t r0 = ta.row, r1 = tb.row, p0 = ta.entry, p1 = tb.entry;

  if (p1 - p0 > cap) {
    // one long row: the whole workgroup strides over it
    __shared__ double part[4][NRHS];
    const double* Xs = DA ? X + int64_t(r0) * NRHS : X;
    double acc[NRHS];
#pragma unroll
    for (int j = 0; j < NRHS; ++j) acc[j] = 0.0;
    for (int32_t q = p0 + threadIdx.x; q < p1; q += 256) {
      const double v = val[q];
      const double* xr = Xs + int64_t(idx[q]) * NRHS;
#pragma unroll
      for (int j = 0; j < NRHS; ++j) acc[j] += v * xr[j];
    }
#pragma unroll
    for (int j = 0; j < NRHS; ++j) {
      const double s = group_sum(acc[j], 64);
      if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6][j] = s;
    }
    __syncthreads();
    if (threadIdx.x < NRHS) {
      const int j = threadIdx.x;
      const double s = (part[0][j] + part[1][j]) + (part[2][j] + part[3][j]);
      double* yr = Y + int64_t(r0) * NRHS + j;
      *yr = finish(s, alpha, beta, read_y != 0, yr);
    }
    return;
  }

  // 1. the tile into LDS, as in spmv_stream
  const int32_t a0 = p0 & ~(L::kAlign - 1);
  copy_to_lds(val_s, val, a0, p1 - a0);
  copy_to_lds(idx_s, idx, a0, p1 - a0);
  const int32_t ar = r0 & ~3;
  copy_to_lds(rp_s, rowptr, ar, r1 + 1 - ar);
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();

  // 2. G lanes per row, split over the right-hand sides and the entries
  if constexpr (SpmmDeep<G, NRHS, PAIRS>::kUse)
    spmm_tile_rows_deep<I, DA, G, NRHS, PAIRS>(r0, r1, a0, ar, val_s, idx_s, rp_s, X, Y, alpha,
                                               beta, read_y != 0);
  else
    spmm_tile_rows<I, DA, NRHS, PAIRS>(G, r0, r1, a0, ar, val_s, idx_s, rp_s, X, Y, alpha, beta,
                                       read_y != 0);
}

}  // namespace kern

namespace {

template <typename I, bool DA, int G, int NRHS, bool PAIRS>
hipError_t go(const SpmvArgs& a) {
  hipLaunchKernelGGL((kern::spmm_stream<I, DA, G, NRHS, PAIRS>), dim3(uint32_t(a.ntiles)),
                     dim3(256), (kern::TileLds<I, double>::bytes(a.cap, a.tile_rows)), a.stream, a.tile_row,
                     a.rowptr, static_cast<const I*>(a.idx), static_cast<const double*>(a.val),
                     static_cast<const double*>(a.x), static_cast<double*>(a.y), a.alpha, a.beta,
                     a.read_y, a.cap);
  return hipGetLastError();
}

template <typename I, bool DA, int G>
hipError_t by_nrhs(const SpmvArgs& a, int nrhs, bool pairs) {
  switch (nrhs) {
    case 1: return go<I, DA, G, 1, false>(a);
    case 2: return pairs ? go<I, DA, G, 2, true>(a) : go<I, DA, G, 2, false>(a);
    case 3: return go<I, DA, G, 3, false>(a);
    case 4: return pairs ? go<I, DA, G, 4, true>(a) : go<I, DA, G, 4, false>(a);
    case 5: return go<I, DA, G, 5, false>(a);
    case 6: return pairs ? go<I, DA, G, 6, true>(a) : go<I, DA, G, 6, false>(a);
    case 7: return go<I, DA, G, 7, false>(a);
    default: return pairs ? go<I, DA, G, 8, true>(a) : go<I, DA, G, 8, false>(a);
  }
}

template <typename I, bool DA>
hipError_t by_lanes(const SpmvArgs& a, int lanes, int nrhs, bool pairs) {
  switch (lanes) {
    case 1: return by_nrhs<I, DA, 1>(a, nrhs, pairs);
    case 2: return by_nrhs<I, DA, 2>(a, nrhs, pairs);
    case 4: return by_nrhs<I, DA, 4>(a, nrhs, pairs);
    case 8: return by_nrhs<I, DA, 8>(a, nrhs, pairs);
    case 16: return by_nrhs<I, DA, 16>(a, nrhs, pairs);
    case 32: return by_nrhs<I, DA, 32>(a, nrhs, pairs);
    default: return by_nrhs<I, DA, 64>(a, nrhs, pairs);
  }
}

}  // namespace

hipError_t launch_spmm_stream(const SpmvArgs& a, int lanes, int nrhs) {
  if (a.ntiles == 0) return hipSuccess;
  const bool pairs = nrhs % 2 == 0 &&
                     ((reinterpret_cast<uintptr_t>(a.x) | reinterpret_cast<uintptr_t>(a.y)) & 15) == 0;
  return a.format == DAMN_FORMAT_DA16 ? by_lanes<int16_t, true>(a, lanes, nrhs, pairs)
                                      : by_lanes<int32_t, false>(a, lanes, nrhs, pairs);
}

}  // namespace damn
