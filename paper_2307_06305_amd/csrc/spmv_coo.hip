// Coordinate-format products y <- alpha*A*x + beta*y for DA-COO (row index
// plus int16 offset c - r per entry; diagonal addressing applied to one of
// COO's index vectors, Sec. 1) and COO (row plus int32 column), with float64
// or float32 values.  Entries are in row order.
//
// Three launches on the caller's stream, all deterministic (no atomics):
//   1. y <- beta*y (zeros when beta == 0): rows without entries are done;
//   2. chunks of kCooChunk consecutive entries per workgroup: indices and
//      values into LDS with 16-byte direct-to-LDS loads, the runs of equal
//      rows numbered by a workgroup prefix sum, then G lanes per run form
//      and sum its products val * x[col].  A run wholly inside the
//      chunk updates y; a run cut by the chunk's start leaves its sum in
//      head[t], one cut only by its end (its row starts in this chunk)
//      leaves it in tail[t];
//   3. one thread per chunk whose tail row continues: tail plus the heads of
//      the following chunks that row covers, in chunk order, into y.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "damn_device.h"
#include "damn_kernels.h"

namespace damn {
namespace kern {

template <typename V>
__global__ __launch_bounds__(256) void coo_scale(int64_t n, V* __restrict__ y, V beta,
                                                 int32_t read_y) {
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (i < n) y[i] = read_y ? beta * y[i] : V(0);
}

template <typename I, typename V, bool DA, int G>
__global__ __launch_bounds__(256) void coo_chunk(int64_t nnz, const int32_t* __restrict__ rows,
                                                 const I* __restrict__ idx,
                                                 const V* __restrict__ val,
                                                 const V* __restrict__ x, V* __restrict__ y,
                                                 V alpha, CooCarry* __restrict__ carry) {
  constexpr int kPerThread = kCooChunk / 256;
  __shared__ __align__(16) int32_t rows_s[kCooChunk];
  __shared__ __align__(16) I idx_s[kCooChunk];
  __shared__ __align__(16) V val_s[kCooChunk];
  __shared__ int32_t seg_s[kCooChunk + 1];  // first entry of each run of equal rows
  __shared__ int32_t wave_cnt[4];
  __shared__ int32_t edge[2];
  __shared__ double head_s, tail_s;
  __shared__ int32_t tail_row_s, through_s;
  const uint32_t t = xcd_contiguous(blockIdx.x, gridDim.x);
  const int64_t c0 = int64_t(t) * kCooChunk;
  const int32_t len = int32_t(nnz - c0 < kCooChunk ? nnz - c0 : kCooChunk);

  // 1. the chunk into LDS (c0 is a multiple of kCooChunk: 16-byte aligned)
  copy_to_lds(rows_s, rows + c0, 0, len);
  copy_to_lds(idx_s, idx + c0, 0, len);
  copy_to_lds(val_s, val + c0, 0, len);
  if (threadIdx.x == 0) {
    edge[0] = c0 > 0 ? rows[c0 - 1] : -1;           // row before the chunk
    edge[1] = c0 + len < nnz ? rows[c0 + len] : -1;  // row after it
    head_s = 0.0;
    tail_s = 0.0;
    tail_row_s = -1;
    through_s = 0;
  }
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();

  // 2. each thread counts the runs starting among its kPerThread
  //    consecutive entries
  const int32_t first = int32_t(threadIdx.x) * kPerThread;
  int32_t cnt = 0;
#pragma unroll
  for (int u = 0; u < kPerThread; ++u) {
    const int32_t k = first + u;
    cnt += k < len && (k == 0 || rows_s[k] != rows_s[k - 1]);
  }
  // 3. exclusive scan of the counts over the workgroup: the run numbers
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int32_t inc = cnt;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int32_t v = __shfl_up(inc, d, 64);
    if (lane >= d) inc += v;
  }
  if (lane == 63) wave_cnt[wave] = inc;
  __syncthreads();
  int32_t pos = inc - cnt;
  for (int w = 0; w < wave; ++w) pos += wave_cnt[w];
  const int32_t nseg = wave_cnt[0] + wave_cnt[1] + wave_cnt[2] + wave_cnt[3];
#pragma unroll
  for (int u = 0; u < kPerThread; ++u) {
    const int32_t k = first + u;
    if (k < len && (k == 0 || rows_s[k] != rows_s[k - 1])) seg_s[pos++] = k;
  }
  if (threadIdx.x == 0) seg_s[nseg] = len;
  __syncthreads();

  // 4. G lanes per run form and sum its products; lane l of a wave takes
  //    run l mod (64/G) of the wave's runs and part l / (64/G) of it, so
  //    neighbouring runs, that is neighbouring rows, sit on neighbouring
  //    lanes and the x gathers of one instruction stay close; a run wholly
  //    inside the chunk updates y, a run cut by an edge leaves its sum for
  //    the join
  constexpr int RPW = 64 / G;
  const int wl = int(threadIdx.x & 63);
  const int gl = wl / RPW;
  for (int32_t q = int32_t(threadIdx.x >> 6) * RPW + wl % RPW; q < nseg; q += 256 / G) {
    const int32_t sk = seg_s[q], ek = seg_s[q + 1];
    const int32_t r = rows_s[sk];
    const V* xs = DA ? x + r : x;
    V acc = V(0), acc2 = V(0);
    int32_t k = sk + gl;
    for (; k + G < ek; k += 2 * G) {
      acc += val_s[k] * xs[idx_s[k]];
      acc2 += val_s[k + G] * xs[idx_s[k + G]];
    }
    if (k < ek) acc += val_s[k] * xs[idx_s[k]];
    acc += acc2;
    if (G > 1) acc = strided_group_sum<G>(acc);
    if (gl == 0) {
      const bool cont_prev = sk == 0 && edge[0] == r;
      const bool cont_next = ek == len && edge[1] == r;
      if (cont_prev) {  // only the first run
        head_s = double(acc);
        through_s = cont_next ? 1 : 0;
      } else if (cont_next) {  // only the last run
        tail_s = double(acc);
        tail_row_s = r;
      } else {
        y[r] = alpha * acc + y[r];
      }
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) carry[t] = CooCarry{head_s, tail_s, tail_row_s, through_s};
}

template <typename V>
__global__ __launch_bounds__(256) void coo_join(int64_t nchunks, const CooCarry* __restrict__ carry,
                                                V* __restrict__ y, V alpha) {
  const int64_t t = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (t >= nchunks) return;
  const int32_t r = carry[t].tail_row;
  if (r < 0) return;
  // the row continues into chunk t+1; it runs through every chunk flagged
  // `through`, and ends in the first chunk that is not
  V s = V(carry[t].tail);
  for (int64_t u = t + 1; u < nchunks; ++u) {
    s += V(carry[u].head);
    if (!carry[u].through) break;
  }
  y[r] = alpha * s + y[r];
}

}  // namespace kern

namespace {

template <typename I, typename V, bool DA>
hipError_t coo(const SpmvArgs& a) {
  V* y = static_cast<V*>(a.y);
  if (a.nrows > 0) {
    hipLaunchKernelGGL(kern::coo_scale<V>, dim3(uint32_t((int64_t(a.nrows) + 255) / 256)),
                       dim3(256), 0, a.stream, int64_t(a.nrows), y, V(a.beta), a.read_y);
  }
  if (a.alpha == 0.0 || a.nchunks == 0) return hipGetLastError();
  // lanes per run from the mean run length (entries per nonempty row)
  const double mean = a.nrows > 0 ? double(a.nnz) / a.nrows : 0.0;
  const dim3 grid(uint32_t(a.nchunks)), block(256);
  const I* idx = static_cast<const I*>(a.idx);
  const V* val = static_cast<const V*>(a.val);
  const V* x = static_cast<const V*>(a.x);
  if (mean < 6.0)
    hipLaunchKernelGGL((kern::coo_chunk<I, V, DA, 1>), grid, block, 0, a.stream, a.nnz,
                       a.coo_rows, idx, val, x, y, V(a.alpha), a.coo_carry);
  else if (mean < 48.0)
    hipLaunchKernelGGL((kern::coo_chunk<I, V, DA, 4>), grid, block, 0, a.stream, a.nnz,
                       a.coo_rows, idx, val, x, y, V(a.alpha), a.coo_carry);
  else
    hipLaunchKernelGGL((kern::coo_chunk<I, V, DA, 16>), grid, block, 0, a.stream, a.nnz,
                       a.coo_rows, idx, val, x, y, V(a.alpha), a.coo_carry);
  hipLaunchKernelGGL(kern::coo_join<V>, dim3(uint32_t((a.nchunks + 255) / 256)), dim3(256), 0,
                     a.stream, a.nchunks, a.coo_carry, y, V(a.alpha));
  return hipGetLastError();
}

}  // namespace

hipError_t launch_spmv_coo(const SpmvArgs& a) {
  const bool da = a.format == DAMN_FORMAT_DACOO16;
  if (a.store == DAMN_F64)
    return da ? coo<int16_t, double, true>(a) : coo<int32_t, double, false>(a);
  return da ? coo<int16_t, float, true>(a) : coo<int32_t, float, false>(a);
}

}  // namespace damn
