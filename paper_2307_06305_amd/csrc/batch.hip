// Batched DA-CSR SpMM: many matrices of uneven size, each with 1-8
// right-hand sides, in one launch captured in a HIP graph.
//
// At creation the host cuts every matrix into stream tiles (consecutive rows
// holding at most `cap` entries) and lists the tiles of all matrices in
// order.  By default the launch has one workgroup per tile and the hardware
// dispatcher keeps every CU full; on request the list is instead split into
// contiguous ranges of about equal modelled bytes, one per workgroup of a
// persistent grid that walks its range.  Each tile is copied from HBM into
// LDS with non-temporal 16-byte direct-to-LDS loads, then every row is
// reduced by G lanes for all right-hand sides of its matrix at once (X and Y
// row-major, the nrhs values of a row adjacent).  Neither mode needs an
// atomic work queue or a reset between launches, which keeps the launch
// replayable from a graph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <new>
#include <vector>

#include "damn.h"
#include "damn_device.h"
#include "damn_mat.h"

namespace damn {
namespace bk {

struct BatchMat {
  const int32_t* rowptr;
  const int16_t* off;
  const double* val;
  const double* X;
  double* Y;
  int32_t nrows;
  int32_t nrhs;
  int32_t lanes;
  int32_t pairs;  // X and Y 16-byte aligned and nrhs even: move values in pairs
};

constexpr int32_t kBatchTileRows = 256;

// One tile: the entry range and the pointers its copy needs, so a
// workgroup starts its copies after a single load; the matrix record
// (vectors, right-hand sides, lanes) loads meanwhile.
struct BatchTile {
  const double* val;
  const int16_t* off;
  const int32_t* rowptr;
  int32_t mat, r0, r1, p0, p1, pad;
};

typedef double d2 __attribute__((ext_vector_type(2)));

// PAIRS: X and Y rows are read and written as 16-byte pairs (NRHS even,
// both 16-byte aligned).
template <int NRHS, bool PAIRS>
__device__ __forceinline__ void tile_rows(const BatchMat& m, int32_t r0, int32_t r1, int32_t a0,
                                          int32_t ar, const double* __restrict__ val_s,
                                          const int16_t* __restrict__ idx_s,
                                          const int32_t* __restrict__ rp_s, double alpha,
                                          double beta, bool read_y) {
  // G lanes per row, spread over the wave as in the SpMV stream kernel:
  // lane l takes row l mod (64/G) of the wave's rows and part l / (64/G)
  const int G = m.lanes;
  const int rpw = 64 / G;
  const int wl = int(threadIdx.x & 63);
  const int lane = wl / rpw;
  for (int32_t r = r0 + int32_t(threadIdx.x >> 6) * rpw + wl % rpw; r < r1; r += 256 / G) {
    const int32_t s = rp_s[r - ar] - a0, e = rp_s[r + 1 - ar] - a0;
    const double* Xs = m.X + int64_t(r) * NRHS;
    // up to 4 right-hand sides, two entries in flight per lane
    double acc[NRHS], acc2[NRHS];
#pragma unroll
    for (int j = 0; j < NRHS; ++j) acc[j] = acc2[j] = 0.0;
    auto add = [&](double* a, int32_t k) {
      const double v = val_s[k];
      const double* xr = Xs + int64_t(idx_s[k]) * NRHS;
      if (PAIRS) {
#pragma unroll
        for (int j = 0; j < NRHS / 2; ++j) {
          const d2 xv = reinterpret_cast<const d2*>(xr)[j];
          a[2 * j] += v * xv.x;
          a[2 * j + 1] += v * xv.y;
        }
      } else {
#pragma unroll
        for (int j = 0; j < NRHS; ++j) a[j] += v * xr[j];
      }
    };
    int32_t k = s + lane;
    if (NRHS <= 4) {
      for (; k + G < e; k += 2 * G) {
        add(acc, k);
        add(acc2, k + G);
      }
    }
    for (; k < e; k += G) add(acc, k);
#pragma unroll
    for (int j = 0; j < NRHS; ++j) acc[j] += acc2[j];
#pragma unroll
    for (int j = 0; j < NRHS; ++j)
      for (int o = 32; o >= rpw; o >>= 1) acc[j] += __shfl_xor(acc[j], o, 64);
    if (lane == 0) {
      double* yr = m.Y + int64_t(r) * NRHS;
      if (PAIRS) {
#pragma unroll
        for (int j = 0; j < NRHS / 2; ++j) {
          d2 out;
          out.x = kern::finish(acc[2 * j], alpha, beta, read_y, yr + 2 * j);
          out.y = kern::finish(acc[2 * j + 1], alpha, beta, read_y, yr + 2 * j + 1);
          reinterpret_cast<d2*>(yr)[j] = out;
        }
      } else {
#pragma unroll
        for (int j = 0; j < NRHS; ++j) yr[j] = kern::finish(acc[j], alpha, beta, read_y, yr + j);
      }
    }
  }
}

__global__ __launch_bounds__(256) void batch_spmm(const BatchMat* __restrict__ mats,
                                                  const BatchTile* __restrict__ tiles,
                                                  const int32_t* __restrict__ range, int32_t cap,
                                                  double alpha, double beta, int32_t read_y) {
  extern __shared__ __align__(16) unsigned char lds[];
  double* val_s = reinterpret_cast<double*>(lds);
  int16_t* idx_s = reinterpret_cast<int16_t*>(lds + sizeof(double) * (cap + 16));
  int32_t* rp_s = reinterpret_cast<int32_t*>(lds + (sizeof(double) + sizeof(int16_t)) * (cap + 16));
  const uint32_t w = kern::xcd_contiguous(blockIdx.x, gridDim.x);
  // range == nullptr: one tile per workgroup; else the workgroup's range
  const int32_t t_begin = range ? range[w] : int32_t(w);
  const int32_t t_end = range ? range[w + 1] : int32_t(w) + 1;
  for (int32_t t = t_begin; t < t_end; ++t) {
    const BatchTile tile = tiles[t];
    const int32_t a0 = tile.p0 & ~7;
    __syncthreads();  // the previous tile's readers are done with LDS
    kern::copy_to_lds(val_s, tile.val, a0, tile.p1 - a0);
    kern::copy_to_lds(idx_s, tile.off, a0, tile.p1 - a0);
    // the tile's row pointers rowptr[ar .. r1] (at most kBatchTileRows + 4;
    // the allocation is padded for the last piece)
    const int32_t ar = tile.r0 & ~3;
    kern::copy_to_lds(rp_s, tile.rowptr, ar, tile.r1 + 1 - ar);
    const BatchMat m = mats[tile.mat];
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
#define DAMN_ROWS(K, P) \
  tile_rows<K, P>(m, tile.r0, tile.r1, a0, ar, val_s, idx_s, rp_s, alpha, beta, read_y)
    const bool pairs = m.pairs != 0;
    switch (m.nrhs) {
      case 1: DAMN_ROWS(1, false); break;
      case 2: if (pairs) DAMN_ROWS(2, true); else DAMN_ROWS(2, false); break;
      case 3: DAMN_ROWS(3, false); break;
      case 4: if (pairs) DAMN_ROWS(4, true); else DAMN_ROWS(4, false); break;
      case 5: DAMN_ROWS(5, false); break;
      case 6: if (pairs) DAMN_ROWS(6, true); else DAMN_ROWS(6, false); break;
      case 7: DAMN_ROWS(7, false); break;
      default: if (pairs) DAMN_ROWS(8, true); else DAMN_ROWS(8, false); break;
    }
#undef DAMN_ROWS
  }
}

}  // namespace bk
}  // namespace damn

struct damn_batch_s {
  int device = 0;
  int32_t count = 0;
  int32_t workgroups = 0;
  int32_t cap = 0;
  int64_t ntiles = 0;
  double model_bytes = 0;
  double alpha = 1.0, beta = 0.0;
  damn::bk::BatchMat* d_mats = nullptr;
  damn::bk::BatchTile* d_tiles = nullptr;
  int32_t* d_range = nullptr;  // null: one workgroup per tile
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace damn {
namespace {

void free_batch(damn_batch B) {
  if (!B) return;
  int cur = 0;
  hipGetDevice(&cur);
  hipSetDevice(B->device);
  if (B->exec) hipGraphExecDestroy(B->exec);
  if (B->graph) hipGraphDestroy(B->graph);
  if (B->d_mats) hipFree(B->d_mats);
  if (B->d_tiles) hipFree(B->d_tiles);
  if (B->d_range) hipFree(B->d_range);
  hipSetDevice(cur);
  delete B;
}

hipError_t launch_batch(damn_batch B, hipStream_t s) {
  if (B->ntiles == 0) return hipSuccess;
  const size_t shmem = size_t(B->cap + 16) * (sizeof(double) + sizeof(int16_t)) +
                       sizeof(int32_t) * (bk::kBatchTileRows + 16);
  const uint32_t grid = B->d_range ? uint32_t(B->workgroups) : uint32_t(B->ntiles);
  hipLaunchKernelGGL(bk::batch_spmm, dim3(grid), dim3(256), shmem, s,
                     B->d_mats, B->d_tiles, B->d_range, B->cap, B->alpha, B->beta,
                     int32_t(B->beta != 0.0));
  return hipGetLastError();
}

}  // namespace
}  // namespace damn

using namespace damn;

extern "C" int damn_batch_create(damn_batch* out, int32_t count, const damn_mat* mats,
                                 const int32_t* nrhs, const double* const* X,
                                 double* const* Y, double alpha, double beta,
                                 int32_t workgroups, void* stream) {
  if (out == nullptr || count < 0 || (count > 0 && (mats == nullptr || nrhs == nullptr ||
                                                    X == nullptr || Y == nullptr)))
    return DAMN_ERR_INVALID_ARG;
  if (workgroups < 0) return DAMN_ERR_INVALID_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  // tile cap: at least the longest row, rounded to 8 entries, 2048..4096
  int32_t longest = 0;
  for (int32_t i = 0; i < count; ++i) {
    const damn_mat A = mats[i];
    if (A == nullptr || A->format != DAMN_FORMAT_DA16 || A->dtype != DAMN_F64)
      return DAMN_ERR_INVALID_ARG;
    if (nrhs[i] < 1 || nrhs[i] > 8) return DAMN_ERR_UNSUPPORTED;
    if ((A->nrows > 0 && Y[i] == nullptr) || (A->ncols > 0 && X[i] == nullptr))
      return DAMN_ERR_INVALID_ARG;
    const int32_t* rp = A->h_rowptr.data();
    for (int32_t r = 0; r < A->nrows; ++r) longest = std::max(longest, rp[r + 1] - rp[r]);
  }
  int32_t cap = std::max<int32_t>(2048, (longest + 7) / 8 * 8);
  if (cap > 4096) return DAMN_ERR_UNSUPPORTED;

  std::vector<bk::BatchMat> hm(count);
  std::vector<bk::BatchTile> ht;
  std::vector<double> work;  // modelled bytes per tile
  double total = 0;
  try {
    for (int32_t i = 0; i < count; ++i) {
      const damn_mat A = mats[i];
      const int32_t k = nrhs[i];
      const int32_t lanes = A->cfg.variant == DAMN_VAR_STREAM ? std::min(A->cfg.lanes, 16) : 2;
      const bool aligned = ((reinterpret_cast<uintptr_t>(X[i]) |
                             reinterpret_cast<uintptr_t>(Y[i])) & 15) == 0;
      hm[i] = {A->d_rowptr, static_cast<const int16_t*>(A->d_idx),
               static_cast<const double*>(A->d_val), X[i], Y[i], A->nrows, k, lanes,
               int32_t(aligned && k % 2 == 0)};
      const int32_t* rp = A->h_rowptr.data();
      int32_t r = 0;
      while (r < A->nrows) {
        const int32_t first = r;
        while (r < A->nrows && r - first < bk::kBatchTileRows && rp[r + 1] - rp[first] <= cap) ++r;
        ht.push_back({static_cast<const double*>(A->d_val), static_cast<const int16_t*>(A->d_idx),
                      A->d_rowptr, i, first, r, rp[first], rp[r], 0});
        const double bytes = double(rp[r] - rp[first]) * (2 + 8) +
                             double(r - first) * (4 + 8.0 * k * (beta != 0.0 ? 2 : 1)) +
                             double(rp[r] - rp[first]) * 8.0 * k / 4;  // gathers, mostly cached
        work.push_back(bytes);
        total += bytes;
      }
      total += double(A->ncols) * 8 * k;
    }
  } catch (const std::bad_alloc&) {
    return DAMN_ERR_ALLOC;
  }
  const int64_t nt = int64_t(ht.size());
  if (nt > INT32_MAX) return DAMN_ERR_UNSUPPORTED;
  // persistent grid: contiguous ranges of about equal work
  std::vector<int32_t> range(size_t(workgroups) + 1, int32_t(nt));
  if (workgroups > 0) {
    double tw = 0;
    for (double v : work) tw += v;
    const double per = tw / workgroups;
    double acc = 0;
    int32_t w = 0;
    range[0] = 0;
    for (int64_t t = 0; t < nt; ++t) {
      acc += work[t];
      while (w + 1 < workgroups && acc >= per * (w + 1)) range[++w] = int32_t(t + 1);
    }
    for (int32_t k = w + 1; k <= workgroups; ++k) range[k] = int32_t(nt);
  }

  damn_batch B = new (std::nothrow) damn_batch_s();
  if (!B) return DAMN_ERR_ALLOC;
  hipGetDevice(&B->device);
  B->count = count;
  B->workgroups = workgroups > 0 ? workgroups : int32_t(nt);
  B->cap = cap;
  B->ntiles = nt;
  B->alpha = alpha;
  B->beta = beta;
  // modelled bytes of one launch: matrices, row pointers, X read once, Y
  for (int32_t i = 0; i < count; ++i) {
    const damn_mat A = mats[i];
    B->model_bytes += double(A->nnz) * 10 + 4.0 * (A->nrows + 1) +
                      8.0 * nrhs[i] * (A->ncols + A->nrows * (beta != 0.0 ? 2 : 1));
  }
  if (hipMalloc(&B->d_mats, sizeof(bk::BatchMat) * std::max<size_t>(hm.size(), 1)) != hipSuccess ||
      hipMalloc(&B->d_tiles, sizeof(bk::BatchTile) * std::max<size_t>(ht.size(), 1)) != hipSuccess ||
      (workgroups > 0 &&
       hipMalloc(&B->d_range, sizeof(int32_t) * range.size()) != hipSuccess)) {
    free_batch(B);
    return DAMN_ERR_ALLOC;
  }
  bool ok = (hm.empty() || hipMemcpyAsync(B->d_mats, hm.data(), sizeof(bk::BatchMat) * hm.size(),
                                          hipMemcpyHostToDevice, s) == hipSuccess) &&
            (ht.empty() || hipMemcpyAsync(B->d_tiles, ht.data(), sizeof(bk::BatchTile) * ht.size(),
                                          hipMemcpyHostToDevice, s) == hipSuccess) &&
            (workgroups == 0 ||
             hipMemcpyAsync(B->d_range, range.data(), sizeof(int32_t) * range.size(),
                            hipMemcpyHostToDevice, s) == hipSuccess) &&
            hipStreamSynchronize(s) == hipSuccess;
  // capture the launch once into a graph, on a stream of our own
  hipStream_t cs = nullptr;
  if (ok) ok = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) == hipSuccess;
  if (ok) ok = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess;
  if (ok) {
    const bool launched = launch_batch(B, cs) == hipSuccess;
    ok = hipStreamEndCapture(cs, &B->graph) == hipSuccess && launched;
  }
  if (ok) ok = hipGraphInstantiate(&B->exec, B->graph, nullptr, nullptr, 0) == hipSuccess;
  if (cs) hipStreamDestroy(cs);
  if (!ok) {
    free_batch(B);
    return DAMN_ERR_HIP;
  }
  *out = B;
  return DAMN_OK;
}

extern "C" int damn_batch_run(damn_batch B, int32_t use_graph, void* stream) {
  if (B == nullptr) return DAMN_ERR_INVALID_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (use_graph) {
    if (B->ntiles == 0) return DAMN_OK;
    return hipGraphLaunch(B->exec, s) == hipSuccess ? DAMN_OK : DAMN_ERR_HIP;
  }
  return launch_batch(B, s) == hipSuccess ? DAMN_OK : DAMN_ERR_HIP;
}

extern "C" int damn_batch_info(damn_batch B, int64_t* ntiles, int32_t* workgroups,
                               double* model_bytes) {
  if (B == nullptr) return DAMN_ERR_INVALID_ARG;
  if (ntiles) *ntiles = B->ntiles;
  if (workgroups) *workgroups = B->workgroups;
  if (model_bytes) *model_bytes = B->model_bytes;
  return DAMN_OK;
}

extern "C" int damn_batch_destroy(damn_batch B) {
  if (B == nullptr) return DAMN_ERR_INVALID_ARG;
  int cur = 0;
  hipGetDevice(&cur);
  hipSetDevice(B->device);
  hipDeviceSynchronize();
  hipSetDevice(cur);
  free_batch(B);
  return DAMN_OK;
}
