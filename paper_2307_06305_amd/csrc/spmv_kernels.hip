// SpMV / SpMM kernels for CSR (int32 columns) and DA-CSR (int16 offsets) on
// gfx950.  y <- alpha*A*x + beta*y (Sec. 4).
//
// DA-CSR rows use the shifted vector xs = x + row, so entry i of row r reads
// xs[off[i]] = x[r + off[i]] (the per-row pointer shift of Sec. 4; one add
// per row instead of one per entry).  For a tall matrix xs may point outside
// x, but every dereference lands inside it (Sec. 4, remark on non-square
// matrices); the host checks r + off[i] in [0, ncols) when a matrix is
// uploaded, so no kernel reads outside x.
//
// SpMV is bound by HBM bandwidth (Eq. 1, Eq. 3): 2 flops per 10 bytes of
// DA-CSR float64 matrix data.  The kernels therefore care about coalesced
// streaming of offsets and values, about keeping x in L2, and about filling
// all 256 CUs; no matrix cores are involved.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "damn_device.h"
#include "damn_kernels.h"

namespace damn {
namespace kern {

// ---------------------------------------------------------------------------
// Vector variant: LANES lanes of a wavefront per row (LANES = 1: one row per
// lane), UNROLL independent partial sums per lane.  One workgroup of 256
// threads covers 256/LANES consecutive rows.
// ---------------------------------------------------------------------------
template <typename I, typename V, bool DA, int LANES, int UNROLL>
__global__ __launch_bounds__(256) void spmv_vector(
    int32_t nrows, const int32_t* __restrict__ rowptr, const I* __restrict__ idx,
    const V* __restrict__ val, const V* __restrict__ x, V* __restrict__ y, V alpha,
    V beta, int32_t read_y) {
  constexpr int RPB = 256 / LANES;
  const uint32_t b = xcd_contiguous(blockIdx.x, gridDim.x);
  const int64_t row = int64_t(b) * RPB + threadIdx.x / LANES;
  const int lane = threadIdx.x % LANES;
  if (row >= nrows) return;  // a row's LANES lanes leave together
  const int32_t p0 = rowptr[row], p1 = rowptr[row + 1];
  const V* xs = DA ? x + row : x;
  V acc[UNROLL];
#pragma unroll
  for (int u = 0; u < UNROLL; ++u) acc[u] = V(0);
  int32_t p = p0 + lane;
  for (; p + (UNROLL - 1) * LANES < p1; p += UNROLL * LANES) {
#pragma unroll
    for (int u = 0; u < UNROLL; ++u) {
      const int32_t q = p + u * LANES;
      acc[u] += val[q] * xs[idx[q]];
    }
  }
#pragma unroll
  for (int u = 0; u < UNROLL - 1; ++u) {
    const int32_t q = p + u * LANES;
    if (q < p1) acc[u] += val[q] * xs[idx[q]];
  }
  V s = acc[0];
#pragma unroll
  for (int u = 1; u < UNROLL; ++u) s += acc[u];
  if (LANES > 1) s = group_sum(s, LANES);
  if (lane == 0) y[row] = finish(s, alpha, beta, read_y != 0, y + row);
}

// ---------------------------------------------------------------------------
// Stream variant.  The host cuts the rows into tiles of consecutive rows
// holding at most `cap` entries (and at most kMaxTileRows rows); a row longer
// than `cap` is a tile of its own.  A workgroup:
//   1. copies the tile's indices and values from HBM straight into LDS with
//      16-byte direct-to-LDS loads (global_load_lds_dwordx4), starting at the
//      tile's first entry rounded down to a multiple of 8.  The loads carry
//      the non-temporal hint: the matrix is read once, and keeping it from
//      displacing x in L2 means each x line is fetched from HBM once;
//   2. reduces each row from LDS with G lanes per row, gathering x.
// Step 1 streams at full load width whatever the row lengths; step 2 puts
// neighbouring rows on neighbouring lanes, so for banded matrices the x
// gathers of one instruction hit few cache lines.
// ---------------------------------------------------------------------------
// Workgroup sum of one double per thread, in a fixed order (wave sums, then
// the four wave results left to right); the result is valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double* scratch4) {
  v = group_sum(v, 64);
  if ((threadIdx.x & 63) == 0) scratch4[threadIdx.x >> 6] = v;
  __syncthreads();
  return (scratch4[0] + scratch4[1]) + (scratch4[2] + scratch4[3]);
}

// Optional epilogue for conjugate gradients (DOT): each workgroup also writes
// partial[t] = sum over its rows of y_r * w_r in float64 (w = nullptr means
// w = y), and every workgroup returns at once when *done is nonzero.
template <typename I, typename V, bool DA, int G, bool DOT = false>
__global__ __launch_bounds__(256) void spmv_stream(
    const int32_t* __restrict__ tile_row, const int32_t* __restrict__ rowptr,
    const I* __restrict__ idx, const V* __restrict__ val, const V* __restrict__ x,
    V* __restrict__ y, V alpha, V beta, int32_t read_y, int32_t cap,
    const V* __restrict__ w = nullptr, double* __restrict__ partial = nullptr,
    const int32_t* __restrict__ done = nullptr) {
  extern __shared__ __align__(16) unsigned char lds[];
  __shared__ double red[4];
  if (DOT && *done) return;
  V* val_s = reinterpret_cast<V*>(lds);
  I* idx_s = reinterpret_cast<I*>(lds + sizeof(V) * (cap + 16));
  int32_t* rp_s = reinterpret_cast<int32_t*>(lds + (sizeof(V) + sizeof(I)) * (cap + 16));

  const uint32_t t = xcd_contiguous(blockIdx.x, gridDim.x);
  const int32_t r0 = tile_row[t], r1 = tile_row[t + 1];
  const int32_t p0 = rowptr[r0], p1 = rowptr[r1];

  if (p1 - p0 > cap) {
    // one long row: the whole workgroup strides over it
    __shared__ V part[4];
    const V* xs = DA ? x + r0 : x;
    V acc = V(0);
    for (int32_t q = p0 + threadIdx.x; q < p1; q += 256) acc += val[q] * xs[idx[q]];
    acc = group_sum(acc, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
      const V s = (part[0] + part[1]) + (part[2] + part[3]);
      const V yr = finish(s, alpha, beta, read_y != 0, y + r0);
      y[r0] = yr;
      if (DOT) partial[t] = double(yr) * double(w ? w[r0] : yr);
    }
    return;
  }

  // 1. [a0, p1) into LDS (a0 = p0 rounded down to 8 entries; at most
  //    cap + 7 entries plus the rounding of the last piece, within cap + 16)
  const int32_t a0 = p0 & ~7;
  copy_to_lds(val_s, val, a0, p1 - a0);
  copy_to_lds(idx_s, idx, a0, p1 - a0);
  // the tile's row pointers rowptr[ar .. r1] (ar = r0 rounded down to 4;
  // at most kMaxTileRows + 4 entries, padded allocation)
  const int32_t ar = r0 & ~3;
  copy_to_lds(rp_s, rowptr, ar, r1 + 1 - ar);
  // the direct-to-LDS writes are tracked by vmcnt; the memory clobber keeps
  // the compiler from moving LDS reads above the wait
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();

  // 2. G lanes per row
  const int lane = threadIdx.x % G;
  double dot = 0.0;
  for (int32_t r = r0 + int32_t(threadIdx.x / G); r < r1; r += 256 / G) {
    const int32_t s = rp_s[r - ar] - a0, e = rp_s[r + 1 - ar] - a0;
    const V* xs = DA ? x + r : x;
    V acc[4] = {V(0), V(0), V(0), V(0)};
    int32_t k = s + lane;
    for (; k + 3 * G < e; k += 4 * G) {
#pragma unroll
      for (int u = 0; u < 4; ++u) acc[u] += val_s[k + u * G] * xs[idx_s[k + u * G]];
    }
#pragma unroll
    for (int u = 0; u < 3; ++u)
      if (k + u * G < e) acc[u] += val_s[k + u * G] * xs[idx_s[k + u * G]];
    V sum = (acc[0] + acc[1]) + (acc[2] + acc[3]);
    if (G > 1) sum = group_sum(sum, G);
    if (lane == 0) {
      const V yr = finish(sum, alpha, beta, read_y != 0, y + r);
      y[r] = yr;
      if (DOT) dot += double(yr) * double(w ? w[r] : yr);
    }
  }
  if (DOT) {
    dot = block_sum(dot, red);
    if (threadIdx.x == 0) partial[t] = dot;
  }
}

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
// loads and writes one checksum, so the compiler cannot drop the loads.
__global__ __launch_bounds__(256) void stream_read(const u32x4* __restrict__ src, int64_t n16,
                                                   double* __restrict__ sink) {
  const uint32_t b = xcd_contiguous(blockIdx.x, gridDim.x);
  const int64_t per = (n16 + gridDim.x - 1) / gridDim.x;
  const int64_t s = int64_t(b) * per;
  const int64_t e = s + per < n16 ? s + per : n16;
  uint32_t acc = 0;
  for (int64_t i = s + threadIdx.x; i < e; i += 256) {
    const u32x4 v = __builtin_nontemporal_load(src + i);
    acc ^= v.x ^ v.y ^ v.z ^ v.w;
  }
  __shared__ uint32_t red[256];
  red[threadIdx.x] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t t = 0;
    for (int k = 0; k < 256; ++k) t ^= red[k];
    sink[blockIdx.x] = double(t);
  }
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

template <typename I, typename V, bool DA, int LANES>
hipError_t launch_vector_u(const SpmvArgs& a, int unroll) {
  const int rpb = 256 / LANES;
  const uint32_t blocks = uint32_t((int64_t(a.nrows) + rpb - 1) / rpb);
  if (blocks == 0) return hipSuccess;
  const I* idx = static_cast<const I*>(a.idx);
  const V* val = static_cast<const V*>(a.val);
  const V* x = static_cast<const V*>(a.x);
  V* y = static_cast<V*>(a.y);
  switch (unroll) {
    case 1:
      hipLaunchKernelGGL((kern::spmv_vector<I, V, DA, LANES, 1>), dim3(blocks), dim3(256), 0,
                         a.stream, a.nrows, a.rowptr, idx, val, x, y, V(a.alpha), V(a.beta),
                         a.read_y);
      break;
    case 2:
      hipLaunchKernelGGL((kern::spmv_vector<I, V, DA, LANES, 2>), dim3(blocks), dim3(256), 0,
                         a.stream, a.nrows, a.rowptr, idx, val, x, y, V(a.alpha), V(a.beta),
                         a.read_y);
      break;
    default:
      hipLaunchKernelGGL((kern::spmv_vector<I, V, DA, LANES, 4>), dim3(blocks), dim3(256), 0,
                         a.stream, a.nrows, a.rowptr, idx, val, x, y, V(a.alpha), V(a.beta),
                         a.read_y);
      break;
  }
  return hipGetLastError();
}

template <typename I, typename V, bool DA>
hipError_t launch_vector(const SpmvArgs& a, int lanes, int unroll) {
  switch (lanes) {
    case 1: return launch_vector_u<I, V, DA, 1>(a, unroll);
    case 2: return launch_vector_u<I, V, DA, 2>(a, unroll);
    case 4: return launch_vector_u<I, V, DA, 4>(a, unroll);
    case 8: return launch_vector_u<I, V, DA, 8>(a, unroll);
    case 16: return launch_vector_u<I, V, DA, 16>(a, unroll);
    case 32: return launch_vector_u<I, V, DA, 32>(a, unroll);
    default: return launch_vector_u<I, V, DA, 64>(a, unroll);
  }
}

template <typename I, typename V, bool DA, int G>
hipError_t launch_stream_g(const SpmvArgs& a) {
  if (a.ntiles == 0) return hipSuccess;
  const size_t shmem = size_t(a.cap + 16) * (sizeof(I) + sizeof(V)) +
                       sizeof(int32_t) * (kMaxTileRows + 16);
  hipLaunchKernelGGL((kern::spmv_stream<I, V, DA, G>), dim3(uint32_t(a.ntiles)), dim3(256),
                     shmem, a.stream, a.tile_row, a.rowptr, static_cast<const I*>(a.idx),
                     static_cast<const V*>(a.val), static_cast<const V*>(a.x),
                     static_cast<V*>(a.y), V(a.alpha), V(a.beta), a.read_y, a.cap);
  return hipGetLastError();
}

template <typename I, typename V, bool DA, int G>
hipError_t launch_stream_dot_g(const SpmvArgs& a, const void* w, double* partial,
                               const int32_t* done) {
  if (a.ntiles == 0) return hipSuccess;
  const size_t shmem = size_t(a.cap + 16) * (sizeof(I) + sizeof(V)) +
                       sizeof(int32_t) * (kMaxTileRows + 16);
  hipLaunchKernelGGL((kern::spmv_stream<I, V, DA, G, true>), dim3(uint32_t(a.ntiles)), dim3(256),
                     shmem, a.stream, a.tile_row, a.rowptr, static_cast<const I*>(a.idx),
                     static_cast<const V*>(a.val), static_cast<const V*>(a.x),
                     static_cast<V*>(a.y), V(a.alpha), V(a.beta), a.read_y, a.cap,
                     static_cast<const V*>(w), partial, done);
  return hipGetLastError();
}

template <typename I, typename V, bool DA>
hipError_t launch_stream_dot(const SpmvArgs& a, int lanes, const void* w, double* partial,
                             const int32_t* done) {
  switch (lanes) {
    case 1: return launch_stream_dot_g<I, V, DA, 1>(a, w, partial, done);
    case 2: return launch_stream_dot_g<I, V, DA, 2>(a, w, partial, done);
    case 4: return launch_stream_dot_g<I, V, DA, 4>(a, w, partial, done);
    case 8: return launch_stream_dot_g<I, V, DA, 8>(a, w, partial, done);
    default: return launch_stream_dot_g<I, V, DA, 16>(a, w, partial, done);
  }
}

template <typename I, typename V, bool DA>
hipError_t launch_stream(const SpmvArgs& a, int lanes) {
  switch (lanes) {
    case 1: return launch_stream_g<I, V, DA, 1>(a);
    case 2: return launch_stream_g<I, V, DA, 2>(a);
    case 4: return launch_stream_g<I, V, DA, 4>(a);
    case 8: return launch_stream_g<I, V, DA, 8>(a);
    case 16: return launch_stream_g<I, V, DA, 16>(a);
    case 32: return launch_stream_g<I, V, DA, 32>(a);
    default: return launch_stream_g<I, V, DA, 64>(a);
  }
}

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
    if (a.f32)
      hipLaunchKernelGGL(kern::scale_vector<float>, dim3(blocks), dim3(256), 0, a.stream, n,
                         static_cast<float*>(a.y), float(a.read_y ? a.beta : 0.0));
    else
      hipLaunchKernelGGL(kern::scale_vector<double>, dim3(blocks), dim3(256), 0, a.stream, n,
                         static_cast<double*>(a.y), a.read_y ? a.beta : 0.0);
    return hipGetLastError();
  }
  if (variant == 1) {
    if (a.da)
      return a.f32 ? launch_stream<int16_t, float, true>(a, lanes)
                   : launch_stream<int16_t, double, true>(a, lanes);
    return a.f32 ? launch_stream<int32_t, float, false>(a, lanes)
                 : launch_stream<int32_t, double, false>(a, lanes);
  }
  if (a.da)
    return a.f32 ? launch_vector<int16_t, float, true>(a, lanes, unroll)
                 : launch_vector<int16_t, double, true>(a, lanes, unroll);
  return a.f32 ? launch_vector<int32_t, float, false>(a, lanes, unroll)
               : launch_vector<int32_t, double, false>(a, lanes, unroll);
}

hipError_t launch_spmv_dot(const SpmvArgs& a, int lanes, const void* w, double* partial,
                           const int32_t* done) {
  if (a.da)
    return a.f32 ? launch_stream_dot<int16_t, float, true>(a, lanes, w, partial, done)
                 : launch_stream_dot<int16_t, double, true>(a, lanes, w, partial, done);
  return a.f32 ? launch_stream_dot<int32_t, float, false>(a, lanes, w, partial, done)
               : launch_stream_dot<int32_t, double, false>(a, lanes, w, partial, done);
}

hipError_t launch_spmm(const SpmvArgs& a, int lanes, int nrhs) {
  if (a.alpha == 0.0) {
    const int64_t n = int64_t(a.nrows) * nrhs;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(kern::scale_vector<double>, dim3(uint32_t((n + 255) / 256)), dim3(256), 0,
                       a.stream, n, static_cast<double*>(a.y), a.read_y ? a.beta : 0.0);
    return hipGetLastError();
  }
  return a.da ? launch_spmm<int16_t, true>(a, lanes, nrhs)
              : launch_spmm<int32_t, false>(a, lanes, nrhs);
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

hipError_t launch_stream_read(const void* src, int64_t bytes, double* sink, hipStream_t s) {
  const int64_t n16 = bytes / 16;
  if (n16 == 0) return hipSuccess;
  int64_t blocks = n16 / 4096;  // about 64 KiB per workgroup
  if (blocks < 256) blocks = 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(kern::stream_read, dim3(uint32_t(blocks)), dim3(256), 0, s,
                     static_cast<const kern::u32x4*>(src), n16, sink);
  return hipGetLastError();
}

}  // namespace damn
