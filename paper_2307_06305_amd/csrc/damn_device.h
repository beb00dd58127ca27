// Device helpers shared by the library's kernels (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace damn {
namespace kern {

// Workgroups are dispatched round-robin over the 8 XCDs (workgroup b runs on
// XCD b % 8).  Renumber them so each XCD walks one contiguous range of rows:
// the x window a range touches then stays in that XCD's L2 instead of being
// fetched by all eight.
__device__ __forceinline__ uint32_t xcd_contiguous(uint32_t b, uint32_t nb) {
  const uint32_t q = nb >> 3, r = nb & 7u;
  const uint32_t xcd = b & 7u, pos = b >> 3;
  return (xcd < r ? xcd * (q + 1) : r * (q + 1) + (xcd - r) * q) + pos;
}

template <typename V>
__device__ __forceinline__ V group_sum(V v, int width) {
  for (int o = width >> 1; o > 0; o >>= 1) v += __shfl_xor(v, o, width);
  return v;
}

// Sum over the G lanes of a wave whose lane numbers agree modulo 64 / G
// (lane l and lanes l + 64/G, l + 2*64/G, ...); every lane gets the sum.
template <int G, typename V>
__device__ __forceinline__ V strided_group_sum(V v) {
  for (int o = 32; o >= 64 / G; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

template <typename V>
__device__ __forceinline__ V finish(V acc, V alpha, V beta, bool read_y, const V* y) {
  return read_y ? alpha * acc + beta * (*y) : alpha * acc;
}

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int kNonTemporal = 2;  // cache-policy bit "nt" of gfx950 loads

// Issue direct-to-LDS copies of elements [a0, a0 + n) of src (src + a0
// 16-byte aligned) into dst[0, ...), 16 bytes per lane; the last piece may
// run up to 16 bytes past the range.  Lane l of wave w copies piece
// 64*(w + 4*j) + l; every wave writes 1 KiB contiguous blocks of LDS.
// AUX is the instruction's cache-policy field (kNonTemporal, or 0 for a
// plain load that may be kept in every cache level).
template <typename T, int AUX = kNonTemporal>
__device__ __forceinline__ void copy_to_lds(T* __restrict__ dst, const T* __restrict__ src,
                                            int32_t a0, int32_t n) {
#if defined(__HIP_DEVICE_COMPILE__)  // the builtin exists only in the device pass
  constexpr int32_t kPer = 16 / int32_t(sizeof(T));  // elements per piece
  const int32_t pieces = (n + kPer - 1) / kPer;
  const int32_t wave = int32_t(threadIdx.x >> 6), lane = int32_t(threadIdx.x & 63);
  for (int32_t base = wave * 64; base < pieces; base += 256) {
    const int32_t q = base + lane;
    if (q < pieces)
      __builtin_amdgcn_global_load_lds(src + a0 + kPer * q, dst + kPer * base, 16, 0, AUX);
  }
#endif
}

}  // namespace kern
}  // namespace damn
