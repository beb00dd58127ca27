// Product kernels y <- alpha*A*x + beta*y (Sec. 4) as templates over the
// storage grid of Fig. 3, and their launchers.  Instantiated by
// spmv_kernels.hip (16-bit DA offsets and 32-bit CSR columns with float64 and
// float32 values) and spmv_grid.hip (the other cells).
//
// Template arguments: I is the stored index type (int8/int16 offsets c - r
// for DA, int16/int32 columns for CSR), S the stored value type (double,
// float or _Float16), V the arithmetic type of x, y and the sums (double for
// double values, float otherwise).
//
// DA rows use the shifted vector xs = x + row, so entry i of row r reads
// xs[off[i]] = x[r + off[i]] (the per-row pointer shift of Sec. 4; one add
// per row instead of one per entry).  For a tall matrix xs may point outside
// x, but every dereference lands inside it (Sec. 4, remark on non-square
// matrices); the host checks every column against [0, ncols) when a matrix
// is uploaded, so no kernel reads outside x.
//
// SpMV is bound by HBM bandwidth (Eq. 1, Eq. 3): 2 flops per 10 bytes of
// DA-CSR float64 matrix data.  The kernels therefore care about coalesced
// streaming of indices and values, about keeping x in L2, and about filling
// all 256 CUs; no matrix cores are involved.
#pragma once

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
template <typename I, typename V, bool DA, int LANES, int UNROLL, typename S = V>
__global__ __launch_bounds__(256) void spmv_vector(
    int32_t nrows, const int32_t* __restrict__ rowptr, const I* __restrict__ idx,
    const S* __restrict__ val, const V* __restrict__ x, V* __restrict__ y, V alpha,
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
      acc[u] += V(val[q]) * xs[idx[q]];
    }
  }
#pragma unroll
  for (int u = 0; u < UNROLL - 1; ++u) {
    const int32_t q = p + u * LANES;
    if (q < p1) acc[u] += V(val[q]) * xs[idx[q]];
  }
  V s = acc[0];
#pragma unroll
  for (int u = 1; u < UNROLL; ++u) s += acc[u];
  if (LANES > 1) s = group_sum(s, LANES);
  if (lane == 0) y[row] = finish(s, alpha, beta, read_y != 0, y + row);
}

// ---------------------------------------------------------------------------
// Stream variant.  The host cuts the rows into tiles of consecutive rows
// holding at most `cap` entries (and at most kMaxTileRows rows, cut back to
// a power-of-two count); a row longer than `cap` is a tile of its own.  Each
// tile is listed with its first row and that row's first entry, so a
// workgroup knows its rows and entries after one load.  A workgroup:
//   1. copies the tile's indices, values and row pointers from HBM straight
//      into LDS with 16-byte direct-to-LDS loads (global_load_lds_dwordx4),
//      starting at the tile's first entry rounded down so every 16-byte piece
//      is aligned.  The entry loads carry the non-temporal hint: the matrix is
//      read once, and keeping it from displacing x in L2 means each x line is
//      fetched from HBM once;
//   2. reduces each row from LDS with G lanes per row, gathering x one value
//      per load (interleaved) or two neighbouring values per load (paired).
// Step 1 streams at full load width whatever the row lengths; step 2 puts
// neighbouring rows on neighbouring lanes, so for banded matrices the x
// gathers of one instruction hit few cache lines.
// ---------------------------------------------------------------------------

// LDS layout of one tile: indices and values of up to `cap` entries plus the
// alignment slack, then the row pointers of up to `rows` rows (the host's
// largest tile), so short-row tiles leave LDS for more workgroups per CU.
template <typename I, typename S>
struct TileLds {
  // the copied range starts at the tile's first entry rounded down to kAlign
  // entries, so 16-byte pieces of both arrays start on 16-byte boundaries
  static constexpr int32_t kAlign =
      int32_t(16 / sizeof(I) > 16 / sizeof(S) ? 16 / sizeof(I) : 16 / sizeof(S));
  // entries per array: cap + (kAlign - 1) leading slack + at most
  // kAlign - 1 entries of the last partial piece, rounded to 16 so every
  // array starts 16-byte aligned
  __host__ __device__ static constexpr int32_t slots(int32_t cap) {
    return (cap + 2 * kAlign - 2 + 15) & ~15;
  }
  // the row-pointer copy covers rows + 1 entries from a start rounded down
  // to 4, in pieces of 4: at most rows + 8 entries
  static constexpr size_t bytes(int32_t cap, int32_t rows) {
    return size_t(slots(cap)) * (sizeof(I) + sizeof(S)) + sizeof(int32_t) * (size_t(rows) + 16);
  }
};

// Phase 2 of the stream kernel for one row whose entries sit at LDS
// positions [s, e): the share of lane `part` (0 <= part < G) of the row's sum.
//
// Interleaved gathers (one x value per load): the lane takes entries
// s + part, s + part + G, ... with four independent partial sums.
template <int G, typename I, typename V, typename S>
__device__ __forceinline__ V row_interleaved(const S* __restrict__ val_s,
                                             const I* __restrict__ idx_s, int32_t s, int32_t e,
                                             int part, const V* __restrict__ xs) {
  V acc[4] = {V(0), V(0), V(0), V(0)};
  int32_t k = s + part;
  for (; k + 3 * G < e; k += 4 * G) {
#pragma unroll
    for (int u = 0; u < 4; ++u) acc[u] += V(val_s[k + u * G]) * xs[idx_s[k + u * G]];
  }
#pragma unroll
  for (int u = 0; u < 3; ++u)
    if (k + u * G < e) acc[u] += V(val_s[k + u * G]) * xs[idx_s[k + u * G]];
  return (acc[0] + acc[1]) + (acc[2] + acc[3]);
}

// Paired gathers (two x values per load): the lane takes the contiguous
// chunk of h = ceil((e - s) / G) entries starting at s + part * h and walks
// it greedily.  Each step loads x[c] and x[c + 1] with one load and also
// uses the second value when the next entry's column is c + 1, so a run of
// neighbouring columns (three per stencil line) costs one load per two
// entries.  cb is the column base (the row for DA offsets, 0 for CSR
// columns); the load address is clamped to `last` = ncols - 2 (ncols >= 2),
// so no load reads past x.  U steps are in flight per lane, chosen so that
// a lane's share of a stencil row issues all its loads before the first
// wait (the kernel picks U by lanes per row).  The positions read past the
// chunk (at most e + 1) lie inside the tile's LDS slots, and what they hold
// is never used.
template <int G, int U, typename I, typename V, typename S>
__device__ __forceinline__ V row_paired(const S* __restrict__ val_s, const I* __restrict__ idx_s,
                                        int32_t s, int32_t e, int part,
                                        const V* __restrict__ x, int32_t cb, int32_t last) {
  typedef V V2 __attribute__((ext_vector_type(2), aligned(sizeof(V))));
  const int32_t h = (e - s + G - 1) / G;
  int32_t k = s + part * h;
  const int32_t kend = min(e, k + h);
  V acc0 = V(0), acc1 = V(0);
  while (k < kend) {
    int32_t kk[U], la[U];
    bool in[U], pr[U], hi[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int32_t o0 = int32_t(idx_s[k]), o1 = int32_t(idx_s[k + 1]);
      in[u] = k < kend;
      pr[u] = in[u] && k + 1 < kend && o1 == o0 + 1;
      const int32_t c = cb + o0;
      la[u] = min(c, last);
      hi[u] = c != la[u];  // only the last column: its value is the pair's second
      kk[u] = k;
      k += in[u] ? (pr[u] ? 2 : 1) : 0;
    }
    V2 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (in[u])
        __builtin_memcpy(&v[u], x + la[u], sizeof(V2));
      else
        v[u] = V2{V(0), V(0)};
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      // selects, not multiplications by zero: an unused value may be inf
      const V f0 = acc0 + V(val_s[kk[u]]) * (hi[u] ? v[u].y : v[u].x);
      const V f1 = acc1 + V(val_s[kk[u] + 1]) * v[u].y;
      acc0 = in[u] ? f0 : acc0;
      acc1 = pr[u] ? f1 : acc1;
    }
  }
  return acc0 + acc1;
}

// Optional epilogue for conjugate gradients (DOT): each workgroup also writes
// partial[t] = sum over its rows of y_r * w_r in float64 (w = nullptr means
// w = y), and every workgroup returns at once when *done is nonzero.
// AUX is the cache policy of the entry arrays' copies: non-temporal by
// default, plain (AUX = 0) for products whose whole working set fits the
// MALL, where caching the matrix lets repeated products read it from there.
// X is the number of x values per gather load: 1 for interleaved gathers,
// 2 for paired ones (then `last` = ncols - 2 >= 0).
template <typename I, typename V, bool DA, int G, bool DOT = false, typename S = V,
          int AUX = kNonTemporal, int X = 1>
__global__ __launch_bounds__(256) void spmv_stream(
    const TileStart* __restrict__ tile_row, const int32_t* __restrict__ rowptr,
    const I* __restrict__ idx, const S* __restrict__ val, const V* __restrict__ x,
    V* __restrict__ y, V alpha, V beta, int32_t read_y, int32_t cap, int32_t last,
    const V* __restrict__ w = nullptr, double* __restrict__ partial = nullptr,
    const int32_t* __restrict__ done = nullptr) {
  using L = TileLds<I, S>;
  extern __shared__ __align__(16) unsigned char lds[];
  __shared__ double red[4];
  __shared__ uint32_t arrived;  // DOT: waves that have left their sum in red
  const int32_t slots = L::slots(cap);
  S* val_s = reinterpret_cast<S*>(lds);
  I* idx_s = reinterpret_cast<I*>(lds + sizeof(S) * slots);
  int32_t* rp_s = reinterpret_cast<int32_t*>(lds + (sizeof(S) + sizeof(I)) * slots);

  const uint32_t t = xcd_contiguous(blockIdx.x, gridDim.x);
  const TileStart ta = tile_row[t], tb = tile_row[t + 1];
  // the flag is loaded after the tile records, so the three loads overlap
  if (DOT && *done) return;
  const int32_t r0 = ta.row, r1 = tb.row, p0 = ta.entry, p1 = tb.entry;

  if (p1 - p0 > cap) {
    // one long row: the whole workgroup strides over it
    __shared__ V part[4];
    const V* xs = DA ? x + r0 : x;
    V acc = V(0);
    for (int32_t q = p0 + threadIdx.x; q < p1; q += 256) acc += V(val[q]) * xs[idx[q]];
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

  // 1. entries [a0, p1) into LDS (a0 = p0 rounded down to kAlign; the copies
  //    stay within slots entries), and the row pointers rowptr[ar .. r1]
  //    (ar = r0 rounded down to 4; at most rows + 4 entries for a tile of
  //    `rows` rows, rounded up to a whole piece: within the rows + 16 the
  //    launch allocates for its largest tile)
  const int32_t a0 = p0 & ~(L::kAlign - 1);
  copy_to_lds<S, AUX>(val_s, val, a0, p1 - a0);
  copy_to_lds<I, AUX>(idx_s, idx, a0, p1 - a0);
  const int32_t ar = r0 & ~3;
  copy_to_lds(rp_s, rowptr, ar, r1 + 1 - ar);
  if (DOT && threadIdx.x == 0) arrived = 0;  // ordered before every wave's add by the barrier
  // the direct-to-LDS writes are tracked by vmcnt; the memory clobber keeps
  // the compiler from moving LDS reads above the wait
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();

  // 2. G lanes per row.  Within a wave, lane l takes row l mod (64/G) of the
  //    wave's rows and part l / (64/G) of that row, so neighbouring lanes
  //    hold neighbouring rows at the same position of their parts: for a
  //    banded matrix their x gathers are adjacent words, which the vector
  //    cache serves as one access.
  constexpr int RPW = 64 / G;  // rows per wave and pass
  const int wl = int(threadIdx.x & 63);
  const int lane = wl / RPW;
  double dot = 0.0;
  for (int32_t r = r0 + int32_t(threadIdx.x >> 6) * RPW + (wl % RPW); r < r1; r += 256 / G) {
    const int32_t s = rp_s[r - ar] - a0, e = rp_s[r + 1 - ar] - a0;
    // the dot epilogue's w_r and, for beta != 0, y_r: loaded with the row's
    // gathers rather than after its sum, where they would add a dependent
    // round trip to the end of the workgroup
    const V wr = (DOT && w && lane == 0) ? w[r] : V(0);
    const V yo = (read_y && lane == 0) ? y[r] : V(0);
    V sum;
    // paired steps in flight: six at one lane per row (a 7-point row with
    // its one pair takes six steps: 128 x 128 x 1024 box, 1024-entry tiles,
    // float64 252.9 -> 241.4 us, float32 196.1 -> 181.3 us against five),
    // five at two and four lanes (27-point rows at four lanes: 95.3 us
    // against 101.9 us with four); four at eight or more lanes, where the
    // shorter parts leave a fifth idle (27-point rows at eight lanes:
    // 117.2 us with five against 107.7 us with four), and in the
    // conjugate-gradient product at four or more lanes, where five would
    // take it past 64 VGPRs (and one wave per SIMD of occupancy)
    constexpr int kPairSteps = G == 1 ? 6 : (G >= 8 || (DOT && G >= 4)) ? 4 : 5;
    if constexpr (X == 2)
      sum = row_paired<G, kPairSteps>(val_s, idx_s, s, e, lane, x, DA ? r : 0, last);
    else
      sum = row_interleaved<G>(val_s, idx_s, s, e, lane, DA ? x + r : x);
    if (G > 1) sum = strided_group_sum<G>(sum);
    if (lane == 0) {
      const V yr = read_y ? alpha * sum + beta * yo : alpha * sum;
      // y is written once per product: where a wave's stores fill whole
      // 128-byte lines (float64, at most 4 lanes per row), a non-temporal
      // store keeps y from displacing x in L2.  The conjugate-gradient
      // product keeps plain stores: its next kernel reads y at once.
      constexpr bool kNtY = !DOT && sizeof(V) == 8 && G <= 4;
      if (kNtY) __builtin_nontemporal_store(yr, y + r); else y[r] = yr;
      if (DOT) dot += double(yr) * double(w ? wr : yr);
    }
  }
  if (DOT) {
    // Each wave leaves its sum in red[wave]; the wave that arrives last
    // combines the four in a fixed order and writes the partial.  No
    // workgroup barrier: a wave whose rows are done (or that has none)
    // leaves at once instead of waiting for the slowest wave.
    dot = group_sum(dot, 64);
    if ((threadIdx.x & 63) == 0) {
      red[threadIdx.x >> 6] = dot;
      const uint32_t before = __hip_atomic_fetch_add(&arrived, 1u, __ATOMIC_ACQ_REL,
                                                     __HIP_MEMORY_SCOPE_WORKGROUP);
      if (before == 3) partial[t] = (red[0] + red[1]) + (red[2] + red[3]);
    }
  }
}

}  // namespace kern

// ---------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------
namespace launch {

template <typename I, typename S, typename V, bool DA, int LANES>
hipError_t vector_u(const SpmvArgs& a, int unroll) {
  const int rpb = 256 / LANES;
  const uint32_t blocks = uint32_t((int64_t(a.nrows) + rpb - 1) / rpb);
  if (blocks == 0) return hipSuccess;
  const I* idx = static_cast<const I*>(a.idx);
  const S* val = static_cast<const S*>(a.val);
  const V* x = static_cast<const V*>(a.x);
  V* y = static_cast<V*>(a.y);
  switch (unroll) {
    case 1:
      hipLaunchKernelGGL((kern::spmv_vector<I, V, DA, LANES, 1, S>), dim3(blocks), dim3(256), 0,
                         a.stream, a.nrows, a.rowptr, idx, val, x, y, V(a.alpha), V(a.beta),
                         a.read_y);
      break;
    case 2:
      hipLaunchKernelGGL((kern::spmv_vector<I, V, DA, LANES, 2, S>), dim3(blocks), dim3(256), 0,
                         a.stream, a.nrows, a.rowptr, idx, val, x, y, V(a.alpha), V(a.beta),
                         a.read_y);
      break;
    default:
      hipLaunchKernelGGL((kern::spmv_vector<I, V, DA, LANES, 4, S>), dim3(blocks), dim3(256), 0,
                         a.stream, a.nrows, a.rowptr, idx, val, x, y, V(a.alpha), V(a.beta),
                         a.read_y);
      break;
  }
  return hipGetLastError();
}

template <typename I, typename S, typename V, bool DA>
hipError_t vector(const SpmvArgs& a, int lanes, int unroll) {
  switch (lanes) {
    case 1: return vector_u<I, S, V, DA, 1>(a, unroll);
    case 2: return vector_u<I, S, V, DA, 2>(a, unroll);
    case 4: return vector_u<I, S, V, DA, 4>(a, unroll);
    case 8: return vector_u<I, S, V, DA, 8>(a, unroll);
    case 16: return vector_u<I, S, V, DA, 16>(a, unroll);
    case 32: return vector_u<I, S, V, DA, 32>(a, unroll);
    default: return vector_u<I, S, V, DA, 64>(a, unroll);
  }
}

// Cells of the storage grid that have the plain-stream kernels: 16-bit DA
// offsets and 32-bit CSR columns with float64 or float32 values.
template <typename I, typename S, bool DA>
constexpr bool kHasPlainStream =
    (DA ? sizeof(I) == 2 : sizeof(I) == 4) && (sizeof(S) == 8 || sizeof(S) == 4);

// Paired gathers run in every scalar cell when the matrix has at least two
// columns (a one-column matrix takes the interleaved kernel).
inline bool use_paired(const SpmvArgs& a) { return a.gather == 2 && a.ncols >= 2; }

template <typename I, typename S, typename V, bool DA, int G>
hipError_t stream_g(const SpmvArgs& a) {
  if (a.ntiles == 0) return hipSuccess;
  const dim3 grid(uint32_t(a.ntiles)), block(256);
  const size_t lds = kern::TileLds<I, S>::bytes(a.cap, a.tile_rows);
  const I* idx = static_cast<const I*>(a.idx);
  const S* val = static_cast<const S*>(a.val);
  const V* x = static_cast<const V*>(a.x);
  V* y = static_cast<V*>(a.y);
  if constexpr (kHasPlainStream<I, S, DA>) {
    if (a.cache == DAMN_CACHE_PLAIN) {
      if (use_paired(a))
        hipLaunchKernelGGL((kern::spmv_stream<I, V, DA, G, false, S, 0, 2>), grid, block, lds,
                           a.stream, a.tile_row, a.rowptr, idx, val, x, y, V(a.alpha),
                           V(a.beta), a.read_y, a.cap, a.ncols - 2, nullptr, nullptr, nullptr);
      else
        hipLaunchKernelGGL((kern::spmv_stream<I, V, DA, G, false, S, 0>), grid, block, lds,
                           a.stream, a.tile_row, a.rowptr, idx, val, x, y, V(a.alpha),
                           V(a.beta), a.read_y, a.cap, 0, nullptr, nullptr, nullptr);
      return hipGetLastError();
    }
  }
  if (use_paired(a)) {
    hipLaunchKernelGGL((kern::spmv_stream<I, V, DA, G, false, S, kern::kNonTemporal, 2>), grid,
                       block, lds, a.stream, a.tile_row, a.rowptr, idx, val, x, y, V(a.alpha),
                       V(a.beta), a.read_y, a.cap, a.ncols - 2, nullptr, nullptr, nullptr);
    return hipGetLastError();
  }
  hipLaunchKernelGGL((kern::spmv_stream<I, V, DA, G, false, S>), grid, block, lds, a.stream,
                     a.tile_row, a.rowptr, idx, val, x, y, V(a.alpha), V(a.beta), a.read_y, a.cap,
                     0, nullptr, nullptr, nullptr);
  return hipGetLastError();
}

template <typename I, typename S, typename V, bool DA>
hipError_t stream(const SpmvArgs& a, int lanes) {
  switch (lanes) {
    case 1: return stream_g<I, S, V, DA, 1>(a);
    case 2: return stream_g<I, S, V, DA, 2>(a);
    case 4: return stream_g<I, S, V, DA, 4>(a);
    case 8: return stream_g<I, S, V, DA, 8>(a);
    case 16: return stream_g<I, S, V, DA, 16>(a);
    case 32: return stream_g<I, S, V, DA, 32>(a);
    default: return stream_g<I, S, V, DA, 64>(a);
  }
}

template <typename I, typename V, bool DA, int G>
hipError_t stream_dot_g(const SpmvArgs& a, const void* w, double* partial, const int32_t* done) {
  if (a.ntiles == 0) return hipSuccess;
  const dim3 grid(uint32_t(a.ntiles)), block(256);
  const size_t lds = kern::TileLds<I, V>::bytes(a.cap, a.tile_rows);
  const I* idx = static_cast<const I*>(a.idx);
  const V* val = static_cast<const V*>(a.val);
  const V* x = static_cast<const V*>(a.x);
  V* y = static_cast<V*>(a.y);
  if (use_paired(a)) {
    hipLaunchKernelGGL((kern::spmv_stream<I, V, DA, G, true, V, kern::kNonTemporal, 2>), grid,
                       block, lds, a.stream, a.tile_row, a.rowptr, idx, val, x, y, V(a.alpha),
                       V(a.beta), a.read_y, a.cap, a.ncols - 2, static_cast<const V*>(w), partial,
                       done);
    return hipGetLastError();
  }
  hipLaunchKernelGGL((kern::spmv_stream<I, V, DA, G, true, V>), grid, block, lds, a.stream,
                     a.tile_row, a.rowptr, idx, val, x, y, V(a.alpha), V(a.beta), a.read_y, a.cap,
                     0, static_cast<const V*>(w), partial, done);
  return hipGetLastError();
}

template <typename I, typename V, bool DA>
hipError_t stream_dot(const SpmvArgs& a, int lanes, const void* w, double* partial,
                      const int32_t* done) {
  switch (lanes) {
    case 1: return stream_dot_g<I, V, DA, 1>(a, w, partial, done);
    case 2: return stream_dot_g<I, V, DA, 2>(a, w, partial, done);
    case 4: return stream_dot_g<I, V, DA, 4>(a, w, partial, done);
    case 8: return stream_dot_g<I, V, DA, 8>(a, w, partial, done);
    default: return stream_dot_g<I, V, DA, 16>(a, w, partial, done);
  }
}

// One index format with the value types of its translation unit.
template <typename I, bool DA, typename S, typename V>
hipError_t product(const SpmvArgs& a, int variant, int lanes, int unroll) {
  return variant == DAMN_VAR_STREAM ? stream<I, S, V, DA>(a, lanes)
                                    : vector<I, S, V, DA>(a, lanes, unroll);
}

}  // namespace launch
}  // namespace damn
