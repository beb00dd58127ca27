// SpMV / SpMM kernels for 16-bit DA offsets and 32-bit CSR columns with
// float64 and float32 values on gfx950, y <- alpha*A*x + beta*y (Sec. 4);
// the dispatch over the whole storage grid of Fig. 3; the SpMM kernels and
// the streaming probes.  The product templates are in spmv_templates.h.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "damn_device.h"
#include "damn_kernels.h"
#include "spmv_templates.h"

namespace damn {
namespace kern {

// ---------------------------------------------------------------------------
// SpMM, vector variant: X is ncols x NRHS and Y nrows x NRHS, row-major.
// Each entry's index and value are read once for all NRHS right-hand sides.
// ---------------------------------------------------------------------------
template <typename I, bool DA, int LANES, int NRHS>
__global__ __launch_bounds__(256) void spmm_vector(
    int32_t nrows, const int32_t* __restrict__ rowptr, const I* __restrict__ idx,
    const double* __restrict__ val, const double* __restrict__ X, double* __restrict__ Y,
    double alpha, double beta, int32_t read_y) {
  constexpr int RPB = 256 / LANES;
  const uint32_t b = xcd_contiguous(blockIdx.x, gridDim.x);
  const int64_t row = int64_t(b) * RPB + threadIdx.x / LANES;
  const int lane = threadIdx.x % LANES;
  if (row >= nrows) return;
  const int32_t p0 = rowptr[row], p1 = rowptr[row + 1];
  const double* Xs = DA ? X + row * NRHS : X;
  double acc[NRHS];
#pragma unroll
  for (int j = 0; j < NRHS; ++j) acc[j] = 0.0;
  for (int32_t p = p0 + lane; p < p1; p += LANES) {
    const double v = val[p];
    const double* xr = Xs + int64_t(idx[p]) * NRHS;
#pragma unroll
    for (int j = 0; j < NRHS; ++j) acc[j] += v * xr[j];
  }
#pragma unroll
  for (int j = 0; j < NRHS; ++j) {
    double s = acc[j];
    if (LANES > 1) s = group_sum(s, LANES);
    acc[j] = s;
  }
  if (lane == 0) {
    double* yr = Y + row * NRHS;
#pragma unroll
    for (int j = 0; j < NRHS; ++j) yr[j] = finish(acc[j], alpha, beta, read_y != 0, yr + j);
  }
}

// y <- beta*y (alpha == 0): A and x are not read.  beta == 0 writes zeros.
template <typename V>
__global__ __launch_bounds__(256) void scale_vector(int64_t n, V* __restrict__ y, V beta) {
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (i < n) y[i] = beta == V(0) ? V(0) : beta * y[i];
}

// Streaming read probe: each workgroup reads a contiguous slice with 16-byte
// loads into registers (non-temporal or plain) and writes one checksum, so
// the compiler cannot drop the loads.  The grid is `slices` workgroups per
// pass; workgroup t (after the XCD renumbering) reads slice t mod slices, so
// a launch of several passes reads the buffer that many times over.
template <bool NT>
__global__ __launch_bounds__(256) void stream_read(const u32x4* __restrict__ src, int64_t n16,
                                                   uint32_t slices, double* __restrict__ sink) {
  const uint32_t b = xcd_contiguous(blockIdx.x, gridDim.x) % slices;
  const int64_t per = (n16 + slices - 1) / slices;
  const int64_t s = int64_t(b) * per;
  const int64_t e = s + per < n16 ? s + per : n16;
  uint32_t acc = 0;
  for (int64_t i = s + threadIdx.x; i < e; i += 256) {
    const u32x4 v = NT ? __builtin_nontemporal_load(src + i) : src[i];
    acc ^= v.x ^ v.y ^ v.z ^ v.w;
  }
  __shared__ uint32_t red[256];
  red[threadIdx.x] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t t = 0;
    for (int k = 0; k < 256; ++k) t ^= red[k];
    sink[blockIdx.x & 65535u] = double(t);
  }
}

// Streaming read probe on the product kernels' own path: one workgroup per
// tile of `tile16` 16-byte pieces, copied from HBM straight into LDS with
// the direct-to-LDS loads of copy_to_lds (non-temporal or plain), then one
// word per thread folded into a checksum.  sink[b mod 65536] receives it.
// The grid is `tiles` workgroups per pass; workgroup t (after the XCD
// renumbering) reads tile t mod tiles.
template <int AUX>
__global__ __launch_bounds__(256) void stream_lds(const u32x4* __restrict__ src, int64_t n16,
                                                  int32_t tile16, uint32_t tiles,
                                                  double* __restrict__ sink) {
  extern __shared__ __align__(16) unsigned char lds[];
  u32x4* buf = reinterpret_cast<u32x4*>(lds);
  const uint32_t b = xcd_contiguous(blockIdx.x, gridDim.x) % tiles;
  const int64_t s = int64_t(b) * tile16;
  const int64_t left = n16 - s;
  const int32_t m = int32_t(left < tile16 ? left : tile16);
  copy_to_lds<u32x4, AUX>(buf, src + s, 0, m);
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();
  uint32_t acc = 0;
  for (int32_t i = int32_t(threadIdx.x); i < m; i += 256) acc ^= buf[i].x;
  acc = __shfl_xor(acc, 1, 64) ^ acc;
  __shared__ uint32_t red[4];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) sink[blockIdx.x & 65535u] = double(red[0] ^ red[1] ^ red[2] ^ red[3]);
}

// Gather probe: the x accesses of a product without its matrix.  Thread r
// reads per_row values x[c]: with offs, c = r + offs[k] (a stencil's DA
// offsets, the same for every row); without, c is drawn from [r - hw,
// r + hw] by an integer hash of (r, k), scattered over a band as a random
// banded matrix's columns are.  Columns are clipped to [0, n).  No matrix
// is streamed.  One checksum per workgroup into sink[b mod 65536].
__global__ __launch_bounds__(256) void gather_read(const double* __restrict__ x, int64_t n,
                                                   int64_t rows, int32_t per_row, int32_t hw,
                                                   const int32_t* __restrict__ offs,
                                                   double* __restrict__ sink) {
  const uint32_t b = xcd_contiguous(blockIdx.x, gridDim.x);
  const int64_t r = int64_t(b) * 256 + threadIdx.x;
  double acc = 0.0;
  if (r < rows) {
    const uint32_t span = 2u * uint32_t(hw) + 1u;
#pragma unroll 4
    for (int32_t k = 0; k < per_row; ++k) {
      int64_t c;
      if (offs) {
        c = r + offs[k];
      } else {
        // a 32-bit mixing function (multiply, xor-shift) of the row and k
        uint32_t h = uint32_t(r) * 0x9E3779B1u ^ (uint32_t(k) + 1u) * 0x85EBCA77u;
        h ^= h >> 16;
        h *= 0x7FEB352Du;
        h ^= h >> 15;
        h *= 0x846CA68Bu;
        h ^= h >> 16;
        c = r - hw + int64_t(h % span);
      }
      c = c < 0 ? 0 : (c >= n ? n - 1 : c);
      acc += x[c];
    }
  }
  acc = group_sum(acc, 64);
  __shared__ double red[4];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) sink[blockIdx.x & 65535u] = (red[0] + red[1]) + (red[2] + red[3]);
}

// Copy probe: dst = src in 16-byte pieces, one contiguous slice per
// workgroup (known bytes read and written, to calibrate traffic counters).
__global__ __launch_bounds__(256) void stream_copy(const u32x4* __restrict__ src,
                                                   u32x4* __restrict__ dst, int64_t n16) {
  const uint32_t b = xcd_contiguous(blockIdx.x, gridDim.x);
  const int64_t per = (n16 + gridDim.x - 1) / gridDim.x;
  const int64_t s = int64_t(b) * per;
  const int64_t e = s + per < n16 ? s + per : n16;
  for (int64_t i = s + threadIdx.x; i < e; i += 256) dst[i] = __builtin_nontemporal_load(src + i);
}

}  // namespace kern

// ---------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------
namespace {

template <typename I, bool DA, int LANES>
hipError_t launch_spmm_l(const SpmvArgs& a, int nrhs) {
  const int rpb = 256 / LANES;
  const uint32_t blocks = uint32_t((int64_t(a.nrows) + rpb - 1) / rpb);
  if (blocks == 0) return hipSuccess;
  const I* idx = static_cast<const I*>(a.idx);
  const double* val = static_cast<const double*>(a.val);
  const double* X = static_cast<const double*>(a.x);
  double* Y = static_cast<double*>(a.y);
#define DAMN_SPMM_CASE(K)                                                                   \
  case K:                                                                                   \
    hipLaunchKernelGGL((kern::spmm_vector<I, DA, LANES, K>), dim3(blocks), dim3(256), 0,   \
                       a.stream, a.nrows, a.rowptr, idx, val, X, Y, a.alpha, a.beta,       \
                       a.read_y);                                                          \
    break;
  switch (nrhs) {
    DAMN_SPMM_CASE(1)
    DAMN_SPMM_CASE(2)
    DAMN_SPMM_CASE(3)
    DAMN_SPMM_CASE(4)
    DAMN_SPMM_CASE(5)
    DAMN_SPMM_CASE(6)
    DAMN_SPMM_CASE(7)
    DAMN_SPMM_CASE(8)
    default: return hipErrorInvalidValue;
  }
#undef DAMN_SPMM_CASE
  return hipGetLastError();
}

template <typename I, bool DA>
hipError_t launch_spmm(const SpmvArgs& a, int lanes, int nrhs) {
  switch (lanes) {
    case 1: return launch_spmm_l<I, DA, 1>(a, nrhs);
    case 2: return launch_spmm_l<I, DA, 2>(a, nrhs);
    case 4: return launch_spmm_l<I, DA, 4>(a, nrhs);
    case 8: return launch_spmm_l<I, DA, 8>(a, nrhs);
    case 16: return launch_spmm_l<I, DA, 16>(a, nrhs);
    case 32: return launch_spmm_l<I, DA, 32>(a, nrhs);
    default: return launch_spmm_l<I, DA, 64>(a, nrhs);
  }
}

}  // namespace

hipError_t launch_spmv(const SpmvArgs& a, int variant, int lanes, int unroll) {
  if (a.alpha == 0.0) {
    const int64_t n = a.nrows;
    if (n == 0) return hipSuccess;
    const uint32_t blocks = uint32_t((n + 255) / 256);
    if (a.store != DAMN_F64)
      hipLaunchKernelGGL(kern::scale_vector<float>, dim3(blocks), dim3(256), 0, a.stream, n,
                         static_cast<float*>(a.y), float(a.read_y ? a.beta : 0.0));
    else
      hipLaunchKernelGGL(kern::scale_vector<double>, dim3(blocks), dim3(256), 0, a.stream, n,
                         static_cast<double*>(a.y), a.read_y ? a.beta : 0.0);
    return hipGetLastError();
  }
  if (a.store == DAMN_F16 || a.format == DAMN_FORMAT_DA8 || a.format == DAMN_FORMAT_CSR16)
    return launch_spmv_grid(a, variant, lanes, unroll);
  const bool f64 = a.store == DAMN_F64;
  if (a.format == DAMN_FORMAT_DA16)
    return f64 ? launch::product<int16_t, true, double, double>(a, variant, lanes, unroll)
               : launch::product<int16_t, true, float, float>(a, variant, lanes, unroll);
  return f64 ? launch::product<int32_t, false, double, double>(a, variant, lanes, unroll)
             : launch::product<int32_t, false, float, float>(a, variant, lanes, unroll);
}

hipError_t launch_spmv_dot(const SpmvArgs& a, int lanes, const void* w, double* partial,
                           const int32_t* done) {
  const bool f64 = a.store == DAMN_F64;
  if (a.format == DAMN_FORMAT_DA16)
    return f64 ? launch::stream_dot<int16_t, double, true>(a, lanes, w, partial, done)
               : launch::stream_dot<int16_t, float, true>(a, lanes, w, partial, done);
  return f64 ? launch::stream_dot<int32_t, double, false>(a, lanes, w, partial, done)
             : launch::stream_dot<int32_t, float, false>(a, lanes, w, partial, done);
}

hipError_t launch_spmm(const SpmvArgs& a, int lanes, int nrhs) {
  return a.format == DAMN_FORMAT_DA16 ? launch_spmm<int16_t, true>(a, lanes, nrhs)
                                      : launch_spmm<int32_t, false>(a, lanes, nrhs);
}

hipError_t launch_stream_read(const void* src, int64_t bytes, int32_t passes, double* sink,
                              int mode, int32_t tile_bytes, hipStream_t s) {
  const int64_t n16 = bytes / 16;
  if (n16 == 0 || passes == 0) return hipSuccess;
  const kern::u32x4* p = static_cast<const kern::u32x4*>(src);
  if (mode == DAMN_READ_LDS_NT || mode == DAMN_READ_LDS_PLAIN) {
    const int32_t t16 = tile_bytes / 16;
    const int64_t tiles = (n16 + t16 - 1) / t16;
    const int64_t blocks = tiles * passes;
    if (blocks > INT32_MAX) return hipErrorInvalidValue;
    const size_t lds = size_t(t16) * 16;
    if (mode == DAMN_READ_LDS_NT)
      hipLaunchKernelGGL(kern::stream_lds<kern::kNonTemporal>, dim3(uint32_t(blocks)), dim3(256),
                         lds, s, p, n16, t16, uint32_t(tiles), sink);
    else
      hipLaunchKernelGGL(kern::stream_lds<0>, dim3(uint32_t(blocks)), dim3(256), lds, s, p, n16,
                         t16, uint32_t(tiles), sink);
    return hipGetLastError();
  }
  int64_t slices = n16 / 4096;  // about 64 KiB per workgroup
  if (slices < 256) slices = 256;
  if (slices > 65536) slices = 65536;
  const int64_t blocks = slices * passes;
  if (blocks > INT32_MAX) return hipErrorInvalidValue;
  if (mode == DAMN_READ_NT)
    hipLaunchKernelGGL(kern::stream_read<true>, dim3(uint32_t(blocks)), dim3(256), 0, s, p, n16,
                       uint32_t(slices), sink);
  else
    hipLaunchKernelGGL(kern::stream_read<false>, dim3(uint32_t(blocks)), dim3(256), 0, s, p, n16,
                       uint32_t(slices), sink);
  return hipGetLastError();
}

hipError_t launch_gather_read(const double* x, int64_t n, int64_t rows, int32_t per_row,
                              int32_t hw, const int32_t* offs, double* sink, hipStream_t s) {
  if (rows == 0 || per_row == 0) return hipSuccess;
  const int64_t blocks = (rows + 255) / 256;
  if (blocks > INT32_MAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL(kern::gather_read, dim3(uint32_t(blocks)), dim3(256), 0, s, x, n, rows,
                     per_row, hw, offs, sink);
  return hipGetLastError();
}

hipError_t launch_stream_copy(const void* src, void* dst, int64_t bytes, hipStream_t s) {
  const int64_t n16 = bytes / 16;
  if (n16 == 0) return hipSuccess;
  int64_t blocks = n16 / 4096;
  if (blocks < 256) blocks = 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(kern::stream_copy, dim3(uint32_t(blocks)), dim3(256), 0, s,
                     static_cast<const kern::u32x4*>(src), static_cast<kern::u32x4*>(dst), n16);
  return hipGetLastError();
}

}  // namespace damn
