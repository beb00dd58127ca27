// Coordinate-format products y <- alpha*A*x + beta*y for DA-COO (row index
// plus int16 offset c - r per entry; diagonal addressing applied to one of
// COO's index vectors, Sec. 1) and COO (row plus int32 column), with float64
// or float32 values.  Entries are in row order.
//
// One launch, deterministic (no atomics): each workgroup takes a chunk of
// kCooChunk consecutive entries, copies its rows, indices and values into
// LDS with 16-byte direct-to-LDS loads, numbers the runs of equal rows with
// a workgroup prefix sum, and then
//   - gives each run G lanes that form and sum its products val * x[col];
//   - skips a first run whose row began in an earlier chunk: the chunk where
//     a row begins sums all of it, so the last run, when its row continues
//     past the chunk, also takes the row's remaining entries [chunk end,
//     cross): up to kCooExtra of them are copied into LDS with the chunk
//     (the stencil rows' remainders), the rest of a longer row is summed by
//     the whole workgroup from global memory;
//   - writes every row it sums once, y[r] = alpha*s + beta*y[r];
//   - writes beta*y (zeros when beta == 0) to the rows without entries: a
//     run's lanes take those between the previous run's row (the row before
//     the chunk for the first run) and its own, the last chunk also those
//     after the matrix's last row.
// cross[t] (built at upload) is the end of the row holding the chunk's last
// entry.  A matrix without entries takes coo_scale only.
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

constexpr int32_t kCooExtra = 64;  // entries past the chunk copied for its crossing row

template <typename I, typename V, bool DA, int G>
__global__ __launch_bounds__(256) void coo_chunk(int64_t nnz, int32_t nrows,
                                                 const int32_t* __restrict__ rows,
                                                 const I* __restrict__ idx,
                                                 const V* __restrict__ val,
                                                 const V* __restrict__ x, V* __restrict__ y,
                                                 V alpha, V beta, int32_t read_y,
                                                 const int32_t* __restrict__ cross) {
  constexpr int kPerThread = kCooChunk / 256;
  __shared__ __align__(16) int32_t rows_s[kCooChunk];
  __shared__ __align__(16) I idx_s[kCooChunk + kCooExtra];
  __shared__ __align__(16) V val_s[kCooChunk + kCooExtra];
  __shared__ int32_t seg_s[kCooChunk + 1];  // first entry of each run of equal rows
  __shared__ int32_t wave_cnt[4];
  __shared__ int32_t edge_s;
  __shared__ V part_s[5];  // the crossing row: its LDS part, then the wave sums
  const uint32_t t = xcd_contiguous(blockIdx.x, gridDim.x);
  const int64_t c0 = int64_t(t) * kCooChunk;
  const int32_t len = int32_t(nnz - c0 < kCooChunk ? nnz - c0 : kCooChunk);
  const int32_t xend = cross[t];  // end of the row of the chunk's last entry
  const int64_t rem = int64_t(xend) - (c0 + len);  // > 0: that row continues
  const int32_t ext = int32_t(rem < kCooExtra ? rem : kCooExtra);

  // 1. the chunk into LDS (c0 is a multiple of kCooChunk: 16-byte aligned),
  //    with the first ext entries past it (the pieces may run up to 16
  //    bytes further: the entry arrays are padded)
  copy_to_lds(rows_s, rows + c0, 0, len);
  copy_to_lds(idx_s, idx + c0, 0, len + ext);
  copy_to_lds(val_s, val + c0, 0, len + ext);
  if (threadIdx.x == 0) {
    edge_s = c0 > 0 ? rows[c0 - 1] : -1;  // row before the chunk
    part_s[0] = V(0);
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
  if (threadIdx.x == 0) seg_s[nseg] = len + ext;  // the last run takes the copied extra
  __syncthreads();
  const int32_t edge = edge_s;

  // 4. G lanes per run form and sum its products; lane l of a wave takes
  //    run l mod (64/G) of the wave's runs and part l / (64/G) of it, so
  //    neighbouring runs, that is neighbouring rows, sit on neighbouring
  //    lanes and the x gathers of one instruction stay close
  constexpr int RPW = 64 / G;
  const int wl = int(threadIdx.x & 63);
  const int gl = wl / RPW;
  for (int32_t q = int32_t(threadIdx.x >> 6) * RPW + wl % RPW; q < nseg; q += 256 / G) {
    const int32_t sk = seg_s[q], ek = seg_s[q + 1];
    const int32_t r = rows_s[sk];
    if (sk == 0 && r == edge) continue;  // begun in an earlier chunk, summed there
    const int32_t prev = sk == 0 ? edge : rows_s[sk - 1];
    for (int32_t g = prev + 1 + gl; g < r; g += G) y[g] = read_y ? beta * y[g] : V(0);
    const V* xs = DA ? x + r : x;
    // eight x gathers in flight per lane before the first is used: a
    // 27-point row's share (about seven entries at four lanes) waits once
    // (27-point 128^3: DA-COO 164.5 -> 154.4 us, COO 186.2 -> 175.0 us
    // against two in flight; the random band unchanged)
    V a4[4] = {V(0), V(0), V(0), V(0)};
    for (int32_t k0 = sk + gl; k0 < ek; k0 += 8 * G) {
      V v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        if (k0 + u * G < ek)
          v[u] = xs[idx_s[k0 + u * G]];
        else
          v[u] = V(0);
      }
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (k0 + u * G < ek) a4[u & 3] += val_s[k0 + u * G] * v[u];
    }
    V acc = (a4[0] + a4[1]) + (a4[2] + a4[3]);
    if (G > 1) acc = strided_group_sum<G>(acc);
    if (gl == 0) {
      if (ek == len + ext && rem > ext)
        part_s[0] = acc;  // finished below with the rest of the row
      else
        y[r] = read_y ? alpha * acc + beta * y[r] : alpha * acc;
    }
  }

  // 5. the rows without entries after the matrix's last row
  if (c0 + len == nnz) {
    for (int32_t g = rows_s[len - 1] + 1 + int32_t(threadIdx.x); g < nrows; g += 256)
      y[g] = read_y ? beta * y[g] : V(0);
  }

  // 6. a last run whose row continues past the copied extra (and began in
  //    this chunk): the workgroup sums the rest of the row from global memory
  const int32_t rl = rows_s[len - 1];
  const bool owner = rem > ext && !(seg_s[nseg - 1] == 0 && rl == edge);
  if (!owner) return;  // uniform over the workgroup
  const V* xs = DA ? x + rl : x;
  V acc = V(0);
  for (int64_t k = c0 + len + ext + threadIdx.x; k < int64_t(xend); k += 256)
    acc += val[k] * xs[idx[k]];
  acc = group_sum(acc, 64);
  __syncthreads();  // part_s[0] is written
  if (lane == 0) part_s[1 + wave] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    const V s = part_s[0] + ((part_s[1] + part_s[2]) + (part_s[3] + part_s[4]));
    y[rl] = read_y ? alpha * s + beta * y[rl] : alpha * s;
  }
}

}  // namespace kern

namespace {

template <typename I, typename V, bool DA>
hipError_t coo(const SpmvArgs& a) {
  V* y = static_cast<V*>(a.y);
  if (a.alpha == 0.0 || a.nchunks == 0) {  // y <- beta*y only
    if (a.nrows > 0)
      hipLaunchKernelGGL(kern::coo_scale<V>, dim3(uint32_t((int64_t(a.nrows) + 255) / 256)),
                         dim3(256), 0, a.stream, int64_t(a.nrows), y, V(a.beta), a.read_y);
    return hipGetLastError();
  }
  // lanes per run from the mean run length (entries per nonempty row)
  const double mean = a.nrows > 0 ? double(a.nnz) / a.nrows : 0.0;
  const dim3 grid(uint32_t(a.nchunks)), block(256);
  const I* idx = static_cast<const I*>(a.idx);
  const V* val = static_cast<const V*>(a.val);
  const V* x = static_cast<const V*>(a.x);
  if (mean < 6.0)
    hipLaunchKernelGGL((kern::coo_chunk<I, V, DA, 1>), grid, block, 0, a.stream, a.nnz, a.nrows,
                       a.coo_rows, idx, val, x, y, V(a.alpha), V(a.beta), a.read_y, a.coo_cross);
  else if (mean < 48.0)
    hipLaunchKernelGGL((kern::coo_chunk<I, V, DA, 4>), grid, block, 0, a.stream, a.nnz, a.nrows,
                       a.coo_rows, idx, val, x, y, V(a.alpha), V(a.beta), a.read_y, a.coo_cross);
  else
    hipLaunchKernelGGL((kern::coo_chunk<I, V, DA, 16>), grid, block, 0, a.stream, a.nnz, a.nrows,
                       a.coo_rows, idx, val, x, y, V(a.alpha), V(a.beta), a.read_y, a.coo_cross);
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
