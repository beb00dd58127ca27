// Block-sparse products y <- alpha*A*x + beta*y for DA-BSR (int16 block
// offsets bc - br) and BSR (int32 block columns), with b x b blocks of
// float64 or float32 values (diagonal addressing applied to BSR, Sec. 1).
//
// Stream variant over tiles of consecutive block rows holding at most `cap`
// blocks.  A workgroup copies the tile's block values, block indices and
// block-row pointers into LDS with 16-byte direct-to-LDS loads, then reduces
// each scalar row br*b + i with G lanes, every lane taking every G-th block
// of the block row.  Consecutive threads hold consecutive scalar rows of a
// block row, so they read consecutive rows of each block from LDS and the
// same b entries of x.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "damn_device.h"
#include "damn_kernels.h"

namespace damn {
namespace kern {

template <typename I, typename S, int B>
struct BsrLds {
  // the copied block range starts at the tile's first block rounded down to
  // kAlign blocks: 16-byte pieces of the index array are then aligned, and so
  // are those of the value array (kAlign * B * B * sizeof(S) is a multiple
  // of 16 for every instantiated type)
  static constexpr int32_t kAlign = int32_t(16 / sizeof(I));
  static_assert((kAlign * B * B * sizeof(S)) % 16 == 0, "value pieces must be aligned");
  __host__ __device__ static constexpr int32_t idx_slots(int32_t cap) {
    return (cap + kAlign + 16 + 15) & ~15;
  }
  __host__ __device__ static constexpr int32_t val_slots(int32_t cap) {
    return ((cap + kAlign) * B * B + 16 + 15) & ~15;
  }
  static constexpr size_t bytes(int32_t cap, int32_t rows) {
    return size_t(val_slots(cap)) * sizeof(S) + size_t(idx_slots(cap)) * sizeof(I) +
           sizeof(int32_t) * (size_t(rows) + 16);
  }
};

template <typename I, typename S, typename V, bool DA, int B, int G>
__global__ __launch_bounds__(256) void spmv_bsr_stream(
    const TileStart* __restrict__ tile_row, const int32_t* __restrict__ browptr,
    const I* __restrict__ bidx, const S* __restrict__ bval, const V* __restrict__ x,
    V* __restrict__ y, V alpha, V beta, int32_t read_y, int32_t cap) {
  using L = BsrLds<I, S, B>;
  extern __shared__ __align__(16) unsigned char lds[];
  S* val_s = reinterpret_cast<S*>(lds);
  I* idx_s = reinterpret_cast<I*>(lds + sizeof(S) * L::val_slots(cap));
  int32_t* rp_s = reinterpret_cast<int32_t*>(lds + sizeof(S) * L::val_slots(cap) +
                                             sizeof(I) * L::idx_slots(cap));
  const uint32_t t = xcd_contiguous(blockIdx.x, gridDim.x);
  const TileStart ta = tile_row[t], tb = tile_row[t + 1];
  const int32_t r0 = ta.row, r1 = tb.row, p0 = ta.entry, p1 = tb.entry;

  if (p1 - p0 > cap) {
    // one long block row: the whole workgroup strides over its blocks
    __shared__ V part[4][B];
    const V* xs = DA ? x + int64_t(r0) * B : x;
    V acc[B];
#pragma unroll
    for (int i = 0; i < B; ++i) acc[i] = V(0);
    for (int32_t q = p0 + threadIdx.x; q < p1; q += 256) {
      const V* xb = xs + int64_t(bidx[q]) * B;
      const S* v = bval + int64_t(q) * B * B;
#pragma unroll
      for (int i = 0; i < B; ++i)
#pragma unroll
        for (int j = 0; j < B; ++j) acc[i] += V(v[i * B + j]) * xb[j];
    }
#pragma unroll
    for (int i = 0; i < B; ++i) {
      const V s = group_sum(acc[i], 64);
      if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6][i] = s;
    }
    __syncthreads();
    if (threadIdx.x < B) {
      const int i = threadIdx.x;
      const V s = (part[0][i] + part[1][i]) + (part[2][i] + part[3][i]);
      V* yr = y + int64_t(r0) * B + i;
      *yr = finish(s, alpha, beta, read_y != 0, yr);
    }
    return;
  }

  // 1. blocks [a0, p1) and block-row pointers [ar, r1] into LDS
  const int32_t a0 = p0 & ~(L::kAlign - 1);
  copy_to_lds(val_s, bval, a0 * B * B, (p1 - a0) * B * B);
  copy_to_lds(idx_s, bidx, a0, p1 - a0);
  const int32_t ar = r0 & ~3;
  copy_to_lds(rp_s, browptr, ar, r1 + 1 - ar);
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();

  // 2. scalar row br*B + i with G lanes, spread over the wave as in the
  //    scalar stream kernel (lane l takes scalar row l mod (64/G) of the
  //    wave's rows and part l / (64/G))
  constexpr int RPW = 64 / G;
  const int wl = int(threadIdx.x & 63);
  const int lane = wl / RPW;
  const int32_t nsr = (r1 - r0) * B;
  for (int32_t sr = int32_t(threadIdx.x >> 6) * RPW + wl % RPW; sr < nsr; sr += 256 / G) {
    const int32_t bro = sr / B, i = sr - bro * B;
    const int32_t br = r0 + bro;
    const int32_t s = rp_s[br - ar] - a0, e = rp_s[br + 1 - ar] - a0;
    const V* xs = DA ? x + int64_t(br) * B : x;
    // UB blocks' x values in flight per lane before the first is used (up
    // to 16 values for b <= 3, 12 for larger blocks, within 64 VGPRs):
    // 3 x 3 blocks on the 27-point pattern, float64 86.4 -> 81.6 us and
    // float32 45.3 -> 42.0 us against two blocks
    constexpr int UB0 = (B <= 3 ? 16 : 12) / B;
    constexpr int UB = UB0 < 2 ? 2 : (UB0 > 8 ? 8 : UB0);
    V a2[2] = {V(0), V(0)};
    for (int32_t k0 = s + lane; k0 < e; k0 += UB * G) {
      V xv[UB][B];
#pragma unroll
      for (int u = 0; u < UB; ++u) {
        const int32_t k = k0 + u * G;
        if (k < e) {
          const V* xa = xs + int64_t(idx_s[k]) * B;
#pragma unroll
          for (int j = 0; j < B; ++j) xv[u][j] = xa[j];
        } else {
#pragma unroll
          for (int j = 0; j < B; ++j) xv[u][j] = V(0);
        }
      }
#pragma unroll
      for (int u = 0; u < UB; ++u) {
        const int32_t k = k0 + u * G;
        if (k < e) {
          const S* va = val_s + (k * B + i) * B;
#pragma unroll
          for (int j = 0; j < B; ++j) a2[u & 1] += V(va[j]) * xv[u][j];
        }
      }
    }
    V sum = a2[0] + a2[1];
    if (G > 1) sum = strided_group_sum<G>(sum);
    if (lane == 0) {
      V* yr = y + int64_t(br) * B + i;
      *yr = finish(sum, alpha, beta, read_y != 0, yr);
    }
  }
}

}  // namespace kern

namespace {

template <typename I, typename S, typename V, bool DA, int B, int G>
hipError_t bsr_g(const SpmvArgs& a) {
  if (a.ntiles == 0) return hipSuccess;
  hipLaunchKernelGGL((kern::spmv_bsr_stream<I, S, V, DA, B, G>), dim3(uint32_t(a.ntiles)),
                     dim3(256), (kern::BsrLds<I, S, B>::bytes(a.cap, a.tile_rows)), a.stream, a.tile_row,
                     a.rowptr, static_cast<const I*>(a.idx), static_cast<const S*>(a.val),
                     static_cast<const V*>(a.x), static_cast<V*>(a.y), V(a.alpha), V(a.beta),
                     a.read_y, a.cap);
  return hipGetLastError();
}

template <typename I, typename S, typename V, bool DA, int B>
hipError_t bsr_lanes(const SpmvArgs& a, int lanes) {
  switch (lanes) {
    case 1: return bsr_g<I, S, V, DA, B, 1>(a);
    case 2: return bsr_g<I, S, V, DA, B, 2>(a);
    case 4: return bsr_g<I, S, V, DA, B, 4>(a);
    case 8: return bsr_g<I, S, V, DA, B, 8>(a);
    default: return bsr_g<I, S, V, DA, B, 16>(a);
  }
}

template <typename I, typename S, typename V, bool DA>
hipError_t bsr_block(const SpmvArgs& a, int lanes) {
  switch (a.block) {
    case 2: return bsr_lanes<I, S, V, DA, 2>(a, lanes);
    case 3: return bsr_lanes<I, S, V, DA, 3>(a, lanes);
    case 4: return bsr_lanes<I, S, V, DA, 4>(a, lanes);
    case 6: return bsr_lanes<I, S, V, DA, 6>(a, lanes);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_spmv_bsr(const SpmvArgs& a, int lanes) {
  const bool da = a.format == DAMN_FORMAT_DABSR16;
  if (a.store == DAMN_F64)
    return da ? bsr_block<int16_t, double, double, true>(a, lanes)
              : bsr_block<int32_t, double, double, false>(a, lanes);
  return da ? bsr_block<int16_t, float, float, true>(a, lanes)
            : bsr_block<int32_t, float, float, false>(a, lanes);
}

}  // namespace damn
