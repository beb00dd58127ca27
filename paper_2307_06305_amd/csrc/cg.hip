// Conjugate gradients on the device: float64 CG and mixed-precision
// iterative refinement with a float32 DA-CSR inner solve.
//
// Every scalar of the iteration (rho, alpha, beta, the stop test) lives in
// device memory; each iteration is five launches:
//   q = A p  with the p.q partial sums        (stream SpMV, dot epilogue)
//   alpha = rho / p.q                         (one workgroup)
//   r -= alpha q, r.r partials                (one pass over r and q)
//   beta, stop test                           (one workgroup)
//   x += alpha p, p = r + beta p              (one pass over x, p and r)
// The x update waits for the pass that reads p anyway, which saves a read
// and a write of p per iteration against updating x beside r.  Once the stop
// test fires, a device flag makes every later launch return at once (the
// iteration's own x update still runs), so the host only reads the flag
// every `check_every` iterations.
// Dot products are summed in float64 in a fixed order (per-workgroup
// partials, then one workgroup), so results do not depend on scheduling.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>

#include "damn.h"
#include "damn_kernels.h"
#include "damn_mat.h"

namespace damn {
namespace cgk {

struct Scal {
  double rho;     // r.r of the current residual
  double alpha;
  double beta;
  double stop2;   // stop when rho <= stop2
  double b2;      // squared norm of the right-hand side of this solve
  int32_t done, converged, breakdown, iters, max_iter, zero;
  int32_t last;  // the stop test fired this iteration: its x update is still due
  int32_t pad;
};

constexpr int kVecBlocks = 4096;  // workgroups of the vector kernels (16 per CU)
constexpr int kFinThreads = 1024;

enum Op { kStart = 0, kAlpha = 1, kBeta = 2, kNorm = 3 };

// Contiguous slice [s, e) of [0, n) for this workgroup; slice starts are
// multiples of `align` elements.
__device__ __forceinline__ void slice(int64_t n, int64_t align, int64_t* s, int64_t* e) {
  const int64_t per = (((n + gridDim.x - 1) / gridDim.x) + align - 1) / align * align;
  *s = int64_t(blockIdx.x) * per;
  *e = *s + per < n ? *s + per : n;
}

// 16 bytes of V: 2 doubles or 4 floats, loaded and stored as one access.
template <typename V>
struct Pack {
  static constexpr int kN = 16 / int(sizeof(V));
  typedef V vec __attribute__((ext_vector_type(kN)));
  static __device__ __forceinline__ vec load(const V* p) {
    return *reinterpret_cast<const vec*>(p);
  }
  static __device__ __forceinline__ void store(V* p, vec v) { *reinterpret_cast<vec*>(p) = v; }
  // non-temporal: for a vector no later kernel of the iteration reads, so it
  // does not displace those that are (p for the next product, r)
  static __device__ __forceinline__ vec load_nt(const V* p) {
    return __builtin_nontemporal_load(reinterpret_cast<const vec*>(p));
  }
  static __device__ __forceinline__ void store_nt(V* p, vec v) {
    __builtin_nontemporal_store(v, reinterpret_cast<vec*>(p));
  }
};

// Visit [s, e) of a slice in 16-byte packs: pack(base) for a whole pack
// starting at element base, tail(i) for the elements after the last whole
// pack (only in the last slice).
template <typename V, typename FP, typename FT>
__device__ __forceinline__ void for_packs(int64_t s, int64_t e, FP pack, FT tail) {
  constexpr int kP = Pack<V>::kN;
  int64_t base = s + int64_t(threadIdx.x) * kP;
  // two packs per step while both are whole (same visiting order as one
  // pack per step, so partial sums keep their order)
  for (; base + 256 * kP + kP <= e; base += 512 * kP) {
    pack(base);
    pack(base + 256 * kP);
  }
  for (; base < e; base += 256 * kP) {
    if (base + kP <= e) {
      pack(base);
    } else {
      for (int64_t i = base; i < e; ++i) tail(i);
    }
  }
}

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Workgroup (256 threads) sum in a fixed order; valid in thread 0.
__device__ __forceinline__ double sum256(double v) {
  __shared__ double w[4];
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) w[threadIdx.x >> 6] = v;
  __syncthreads();
  return (w[0] + w[1]) + (w[2] + w[3]);
}

// Fresh scalar records sc[0, count): zeros, with the iteration limit set.
// Written by a kernel so no host memory has to outlive the call.
__global__ void reset_scal(Scal* __restrict__ sc, int32_t count, int32_t max_iter) {
  const int32_t i = int32_t(threadIdx.x);
  if (i >= count) return;
  Scal z{};
  z.max_iter = max_iter;
  sc[i] = z;
}

// x = 0, r = b, p = b; partial[block] = sum b^2
__global__ __launch_bounds__(256) void init64(int64_t n, const double* __restrict__ b,
                                              double* __restrict__ x, double* __restrict__ r,
                                              double* __restrict__ p,
                                              double* __restrict__ partial) {
  int64_t s, e;
  slice(n, 512, &s, &e);
  double acc = 0.0;
  typedef Pack<double> P;
  for_packs<double>(s, e, [&](int64_t base) {
      const P::vec v = P::load(b + base);
      P::store(x + base, P::vec(0.0));
      P::store(r + base, v);
      if (p) P::store(p + base, v);
      acc += v.x * v.x + v.y * v.y;
    }, [&](int64_t i) {
      const double v = b[i];
      x[i] = 0.0;
      r[i] = v;
      if (p) p[i] = v;
      acc += v * v;
    });
  acc = sum256(acc);
  if (threadIdx.x == 0) partial[blockIdx.x] = acc;
}

// One workgroup: s = sum of partial[0..np) in a fixed order, then the step op.
__global__ __launch_bounds__(kFinThreads) void finalize(const double* __restrict__ partial,
                                                        int32_t np, Scal* __restrict__ sc,
                                                        int32_t op, double tol2) {
  __shared__ double w[kFinThreads / 64];
  if ((op == kAlpha || op == kBeta) && sc->done) {
    // the first skipped alpha step follows the final x update
    if (op == kAlpha && threadIdx.x == 0) sc->last = 0;
    return;
  }
  // eight independent sums per thread, each fed by 16-byte loads of two
  // partials, keep eight loads in flight; they are combined in a fixed
  // order, so the result does not depend on timing
  typedef double d2 __attribute__((ext_vector_type(2)));
  const d2* pp = reinterpret_cast<const d2*>(partial);  // partial is 16-byte aligned
  const int32_t npairs = np >> 1;
  d2 a[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) a[u] = d2(0.0);
  int32_t i = threadIdx.x;
  for (; i + 7 * kFinThreads < npairs; i += 8 * kFinThreads) {
#pragma unroll
    for (int u = 0; u < 8; ++u) a[u] += pp[i + u * kFinThreads];
  }
#pragma unroll
  for (int u = 0; u < 7; ++u)
    if (i + u * kFinThreads < npairs) a[u] += pp[i + u * kFinThreads];
  if ((np & 1) && threadIdx.x == 0) a[7].y += partial[np - 1];
  double acc = 0.0;
#pragma unroll
  for (int u = 0; u < 8; ++u) acc += a[u].x + a[u].y;
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) w[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x != 0) return;
  double s = 0.0;
  for (int k = 0; k < kFinThreads / 64; ++k) s += w[k];
  switch (op) {
    case kStart:
      sc->rho = s;
      sc->b2 = s;
      sc->stop2 = tol2 * s;
      sc->iters = 0;
      sc->breakdown = 0;
      sc->converged = s <= sc->stop2 ? 1 : 0;  // b = 0
      sc->done = sc->converged;
      break;
    case kAlpha:
      if (!(s > 0.0)) {
        sc->breakdown = 1;
        sc->done = 1;
      } else {
        sc->alpha = sc->rho / s;
      }
      break;
    case kBeta:
      sc->iters += 1;
      if (s <= sc->stop2) {
        sc->rho = s;
        sc->converged = 1;
        sc->done = 1;
        sc->last = 1;
      } else if (sc->iters >= sc->max_iter) {
        sc->rho = s;
        sc->done = 1;
        sc->last = 1;
      } else {
        sc->beta = s / sc->rho;
        sc->rho = s;
      }
      break;
    default:  // kNorm: squared norm of a freshly formed residual
      sc->rho = s;
      break;
  }
}

// r -= alpha q; partial[block] = sum r^2.  V = double or float (float: the
// update is formed in float64 and rounded once).
template <typename V>
__global__ __launch_bounds__(256) void update_r(int64_t n, V* __restrict__ r,
                                                const V* __restrict__ q,
                                                const Scal* __restrict__ sc,
                                                double* __restrict__ partial) {
  if (sc->done) return;
  const double a = sc->alpha;
  int64_t s, e;
  slice(n, 1024, &s, &e);
  double acc = 0.0;
  typedef Pack<V> P;
  for_packs<V>(s, e, [&](int64_t base) {
      typename P::vec rv = P::load(r + base);
      const typename P::vec qv = P::load_nt(q + base);
#pragma unroll
      for (int k = 0; k < P::kN; ++k) {
        rv[k] = V(double(rv[k]) - a * double(qv[k]));
        acc += double(rv[k]) * double(rv[k]);
      }
      P::store(r + base, rv);
    }, [&](int64_t i) {
      const V rn = V(double(r[i]) - a * double(q[i]));
      r[i] = rn;
      acc += double(rn) * double(rn);
    });
  acc = sum256(acc);
  if (threadIdx.x == 0) partial[blockIdx.x] = acc;
}

// x += alpha p, then p = r + beta p (p only while the iteration goes on)
template <typename V>
__global__ __launch_bounds__(256) void update_xp(int64_t n, V* __restrict__ x, V* __restrict__ p,
                                                 const V* __restrict__ r,
                                                 const Scal* __restrict__ sc) {
  if (sc->done && !sc->last) return;
  const bool more = !sc->done;
  const double a = sc->alpha, bt = sc->beta;
  int64_t s, e;
  slice(n, 1024, &s, &e);
  typedef Pack<V> P;
  for_packs<V>(s, e, [&](int64_t base) {
      // all three loads before the first store, so they are in flight together
      typename P::vec xv = P::load_nt(x + base), pv = P::load(p + base);
      const typename P::vec rv = more ? P::load(r + base) : typename P::vec(V(0));
#pragma unroll
      for (int k = 0; k < P::kN; ++k) xv[k] = V(double(xv[k]) + a * double(pv[k]));
      P::store_nt(x + base, xv);
      if (more) {
#pragma unroll
        for (int k = 0; k < P::kN; ++k) pv[k] = V(double(rv[k]) + bt * double(pv[k]));
        P::store(p + base, pv);
      }
    }, [&](int64_t i) {
      x[i] = V(double(x[i]) + a * double(p[i]));
      if (more) p[i] = V(double(r[i]) + bt * double(p[i]));
    });
}

// Inner solve start: rh = float(r / ||r||), d = 0, p = rh; partial = sum rh^2
__global__ __launch_bounds__(256) void mixed_start(int64_t n, const double* __restrict__ r,
                                                   const Scal* __restrict__ outer,
                                                   float* __restrict__ rh, float* __restrict__ d,
                                                   float* __restrict__ p,
                                                   double* __restrict__ partial) {
  const double inv = 1.0 / sqrt(outer->rho);
  int64_t s, e;
  slice(n, 256, &s, &e);
  double acc = 0.0;
  for (int64_t i = s + threadIdx.x; i < e; i += 256) {
    const float v = float(r[i] * inv);
    rh[i] = v;
    d[i] = 0.0f;
    p[i] = v;
    acc += double(v) * double(v);
  }
  acc = sum256(acc);
  if (threadIdx.x == 0) partial[blockIdx.x] = acc;
}

// x += ||r|| d
__global__ __launch_bounds__(256) void mixed_correct(int64_t n, double* __restrict__ x,
                                                     const float* __restrict__ d,
                                                     const Scal* __restrict__ outer) {
  const double scale = sqrt(outer->rho);
  int64_t s, e;
  slice(n, 256, &s, &e);
  for (int64_t i = s + threadIdx.x; i < e; i += 256) x[i] += scale * double(d[i]);
}

}  // namespace cgk
}  // namespace damn

// Workspace kept with the float64 handle.
struct damn_cg_work {
  int64_t n = 0;
  int64_t npartial = 0;
  bool mixed = false;
  double *r = nullptr, *p = nullptr, *q = nullptr;
  float *rh = nullptr, *d = nullptr, *p32 = nullptr, *q32 = nullptr;
  double* partial = nullptr;
  damn::cgk::Scal* sc = nullptr;   // [0] iteration, [1] outer residual
  damn::cgk::Scal* host = nullptr; // pinned copies
};

namespace damn {

void release_cg_work(damn_mat A) {
  damn_cg_work* w = A->cg;
  if (!w) return;
  for (void* ptr : {(void*)w->r, (void*)w->p, (void*)w->q, (void*)w->rh, (void*)w->d,
                    (void*)w->p32, (void*)w->q32, (void*)w->partial, (void*)w->sc})
    if (ptr) hipFree(ptr);
  if (w->host) hipHostFree(w->host);
  delete w;
  A->cg = nullptr;
}

namespace {

using cgk::Scal;

int get_work(damn_mat A, int64_t npartial, bool mixed, damn_cg_work** out) {
  damn_cg_work* w = A->cg;
  const int64_t n = A->nrows;
  if (w && w->n == n && w->npartial >= npartial && (w->mixed || !mixed)) {
    *out = w;
    return DAMN_OK;
  }
  release_cg_work(A);
  w = new (std::nothrow) damn_cg_work();
  if (!w) return DAMN_ERR_ALLOC;
  A->cg = w;
  w->n = n;
  w->npartial = npartial;
  w->mixed = mixed;
  const size_t n8 = sizeof(double) * size_t(n > 0 ? n : 1);
  const size_t n4 = sizeof(float) * size_t(n > 0 ? n : 1);
  bool ok = hipMalloc(&w->r, n8) == hipSuccess && hipMalloc(&w->p, n8) == hipSuccess &&
            hipMalloc(&w->q, n8) == hipSuccess &&
            hipMalloc(&w->partial, sizeof(double) * size_t(npartial)) == hipSuccess &&
            hipMalloc(&w->sc, 2 * sizeof(Scal)) == hipSuccess &&
            hipHostMalloc(&w->host, 2 * sizeof(Scal), hipHostMallocDefault) == hipSuccess;
  if (ok && mixed)
    ok = hipMalloc(&w->rh, n4) == hipSuccess && hipMalloc(&w->d, n4) == hipSuccess &&
         hipMalloc(&w->p32, n4) == hipSuccess && hipMalloc(&w->q32, n4) == hipSuccess;
  if (!ok) {
    release_cg_work(A);
    return DAMN_ERR_ALLOC;
  }
  *out = w;
  return DAMN_OK;
}

SpmvArgs stream_args(damn_mat A, const void* x, void* y, double alpha, double beta,
                     hipStream_t s) {
  SpmvArgs a;
  a.nrows = A->nrows;
  a.ncols = A->ncols;
  a.rowptr = A->d_rowptr;
  a.idx = A->d_idx;
  a.val = A->d_val;
  a.x = x;
  a.y = y;
  a.alpha = alpha;
  a.beta = beta;
  a.read_y = beta != 0.0;
  a.format = A->format;
  a.store = A->dtype;
  a.tile_row = A->d_tiles;
  a.ntiles = A->ntiles;
  a.cap = A->tiles_cap;
  a.tile_rows = A->tiles_rows;
  a.gather = gather_of(A->cfg);
  a.stream = s;
  return a;
}

int cg_lanes(damn_mat A) {
  int l = A->cfg.variant == DAMN_VAR_STREAM ? A->cfg.lanes : 2;
  return l > 16 ? 16 : l;
}

#define DAMN_HIP_TRY(expr)                          \
  do {                                              \
    if ((expr) != hipSuccess) return DAMN_ERR_HIP;  \
  } while (0)

// Fetch both scalar records to the host (synchronises the stream).
int read_scal(damn_cg_work* w, hipStream_t s) {
  DAMN_HIP_TRY(hipMemcpyAsync(w->host, w->sc, 2 * sizeof(Scal), hipMemcpyDeviceToHost, s));
  DAMN_HIP_TRY(hipStreamSynchronize(s));
  return DAMN_OK;
}

// Run CG iterations on the iteration record sc[0] until its done flag is set.
// Vectors: solution xs, residual rs, direction ps, product qs (all of the
// matrix's value type).
template <typename V>
int iterate(damn_mat M, damn_cg_work* w, V* xs, V* rs, V* ps, V* qs, int check_every,
            hipStream_t s) {
  const int64_t n = M->nrows;
  const int lanes = cg_lanes(M);
  while (true) {
    for (int k = 0; k < check_every; ++k) {
      SpmvArgs a = stream_args(M, ps, qs, 1.0, 0.0, s);
      DAMN_HIP_TRY(launch_spmv_dot(a, lanes, ps, w->partial, &w->sc[0].done));
      hipLaunchKernelGGL(cgk::finalize, dim3(1), dim3(cgk::kFinThreads), 0, s, w->partial,
                         int32_t(M->ntiles), w->sc, int32_t(cgk::kAlpha), 0.0);
      hipLaunchKernelGGL(cgk::update_r<V>, dim3(cgk::kVecBlocks), dim3(256), 0, s, n, rs, qs,
                         w->sc, w->partial);
      hipLaunchKernelGGL(cgk::finalize, dim3(1), dim3(cgk::kFinThreads), 0, s, w->partial,
                         int32_t(cgk::kVecBlocks), w->sc, int32_t(cgk::kBeta), 0.0);
      hipLaunchKernelGGL(cgk::update_xp<V>, dim3(cgk::kVecBlocks), dim3(256), 0, s, n, xs, ps,
                         rs, w->sc);
    }
    DAMN_HIP_TRY(hipGetLastError());
    const int st = read_scal(w, s);
    if (st != DAMN_OK) return st;
    if (w->host[0].done) return DAMN_OK;
  }
}

// r = b - A x (float64) and its squared norm into sc[1].rho
int residual(damn_mat A64, damn_cg_work* w, const double* b, const double* x, hipStream_t s) {
  DAMN_HIP_TRY(hipMemcpyAsync(w->r, b, sizeof(double) * size_t(A64->nrows),
                              hipMemcpyDeviceToDevice, s));
  SpmvArgs a = stream_args(A64, x, w->r, -1.0, 1.0, s);
  DAMN_HIP_TRY(launch_spmv_dot(a, cg_lanes(A64), nullptr, w->partial, &w->sc[1].zero));
  hipLaunchKernelGGL(cgk::finalize, dim3(1), dim3(cgk::kFinThreads), 0, s, w->partial,
                     int32_t(A64->ntiles), w->sc + 1, int32_t(cgk::kNorm), 0.0);
  DAMN_HIP_TRY(hipGetLastError());
  return DAMN_OK;
}

// Arguments of a solve, checked before any work is queued.
int check_args(damn_mat A64, damn_mat A32, const double* b, double* x, const damn_cg_opts* opts,
               damn_cg_info* info) {
  if (A64 == nullptr || opts == nullptr || info == nullptr) return DAMN_ERR_INVALID_ARG;
  if (A64->nrows != A64->ncols || A64->dtype != DAMN_F64) return DAMN_ERR_INVALID_ARG;
  if (A64->nrows > 0 && (b == nullptr || x == nullptr)) return DAMN_ERR_INVALID_ARG;
  if (A64->format != DAMN_FORMAT_DA16 && A64->format != DAMN_FORMAT_CSR32)
    return DAMN_ERR_UNSUPPORTED;
  // the vector kernels move 16-byte packs
  if ((reinterpret_cast<uintptr_t>(b) | reinterpret_cast<uintptr_t>(x)) & 15)
    return DAMN_ERR_INVALID_ARG;
  if (A32 && (A32->nrows != A64->nrows || A32->ncols != A64->ncols ||
              A32->dtype != DAMN_F32 || A32->format != A64->format))
    return DAMN_ERR_INVALID_ARG;
  if (!(opts->tol > 0.0) || opts->max_iter < 1 || opts->check_every < 1 ||
      (A32 && (!(opts->inner_tol > 0.0) || opts->max_outer < 1)))
    return DAMN_ERR_INVALID_ARG;
  // every tiled handle carries the stream tiles of its last stream
  // configuration (built at create)
  if (A64->d_tiles == nullptr || (A32 && A32->d_tiles == nullptr)) return DAMN_ERR_INVALID_ARG;
  return DAMN_OK;
}

// Partial sums a solve needs: one per tile of either matrix, one per
// workgroup of the vector kernels.
int64_t partial_count(damn_mat A64, damn_mat A32) {
  int64_t np = cgk::kVecBlocks;
  if (A64->ntiles > np) np = A64->ntiles;
  if (A32 && A32->ntiles > np) np = A32->ntiles;
  return np;
}

// The solve proper, on a workspace w whose vectors hold n entries (the float32
// ones only for a mixed solve) and whose partial array holds partial_count.
int solve(damn_mat A64, damn_mat A32, const double* b, double* x, const damn_cg_opts* opts,
          damn_cg_info* info, damn_cg_work* w, hipStream_t s) {
  const int64_t n = A64->nrows;
  hipLaunchKernelGGL(cgk::reset_scal, dim3(1), dim3(64), 0, s, w->sc, 2, opts->max_iter);
  DAMN_HIP_TRY(hipGetLastError());
  const double tol2 = opts->tol * opts->tol;
  damn_cg_info out{};
  int st = DAMN_OK;

  if (n == 0) {
    out.converged = 1;
    *info = out;
    return DAMN_OK;
  }
  if (A32 == nullptr) {
    // float64 CG from x = 0: r = p = b
    hipLaunchKernelGGL(cgk::init64, dim3(cgk::kVecBlocks), dim3(256), 0, s, n, b, x, w->r, w->p,
                       w->partial);
    hipLaunchKernelGGL(cgk::finalize, dim3(1), dim3(cgk::kFinThreads), 0, s, w->partial,
                       int32_t(cgk::kVecBlocks), w->sc, int32_t(cgk::kStart), tol2);
    DAMN_HIP_TRY(hipGetLastError());
    st = iterate<double>(A64, w, x, w->r, w->p, w->q, opts->check_every, s);
    if (st != DAMN_OK) return st;
    const Scal it = w->host[0];
    st = residual(A64, w, b, x, s);
    if (st == DAMN_OK) st = read_scal(w, s);
    if (st != DAMN_OK) return st;
    out.iters = it.iters;
    out.outer = 0;
    out.converged = it.converged;
    out.rel_res = it.b2 > 0 ? std::sqrt(w->host[1].rho / it.b2) : 0.0;
    *info = out;
    if (it.breakdown) return DAMN_ERR_BREAKDOWN;
    return it.converged ? DAMN_OK : DAMN_ERR_NOT_CONVERGED;
  }

  // mixed precision: outer record sc[1] holds ||b||^2 (b2) and ||r||^2 (rho)
  hipLaunchKernelGGL(cgk::init64, dim3(cgk::kVecBlocks), dim3(256), 0, s, n, b, x, w->r,
                     (double*)nullptr, w->partial);
  hipLaunchKernelGGL(cgk::finalize, dim3(1), dim3(cgk::kFinThreads), 0, s, w->partial,
                     int32_t(cgk::kVecBlocks), w->sc + 1, int32_t(cgk::kStart), tol2);
  DAMN_HIP_TRY(hipGetLastError());
  int32_t total_inner = 0;
  int32_t outer = 0;
  bool breakdown = false;
  while (true) {
    st = read_scal(w, s);
    if (st != DAMN_OK) return st;
    const Scal o = w->host[1];
    if (o.rho <= o.stop2) {
      out.converged = 1;
      break;
    }
    if (outer >= opts->max_outer) break;
    // inner CG on A32 d = r / ||r||, to the relative residual the outer
    // target still needs (never below inner_tol, never above 1/2)
    double target = 0.5 * opts->tol * std::sqrt(o.b2 / o.rho);
    if (target < opts->inner_tol) target = opts->inner_tol;
    if (target > 0.5) target = 0.5;
    hipLaunchKernelGGL(cgk::reset_scal, dim3(1), dim3(64), 0, s, w->sc, 1, opts->max_iter);
    hipLaunchKernelGGL(cgk::mixed_start, dim3(cgk::kVecBlocks), dim3(256), 0, s, n, w->r,
                       w->sc + 1, w->rh, w->d, w->p32, w->partial);
    hipLaunchKernelGGL(cgk::finalize, dim3(1), dim3(cgk::kFinThreads), 0, s, w->partial,
                       int32_t(cgk::kVecBlocks), w->sc, int32_t(cgk::kStart), target * target);
    DAMN_HIP_TRY(hipGetLastError());
    st = iterate<float>(A32, w, w->d, w->rh, w->p32, w->q32, opts->check_every, s);
    if (st != DAMN_OK) return st;
    total_inner += w->host[0].iters;
    ++outer;
    hipLaunchKernelGGL(cgk::mixed_correct, dim3(cgk::kVecBlocks), dim3(256), 0, s, n, x, w->d,
                       w->sc + 1);
    DAMN_HIP_TRY(hipGetLastError());
    st = residual(A64, w, b, x, s);
    if (st != DAMN_OK) return st;
    if (w->host[0].breakdown) {
      breakdown = true;
      st = read_scal(w, s);
      if (st != DAMN_OK) return st;
      break;
    }
  }
  const Scal o = w->host[1];
  out.iters = total_inner;
  out.outer = outer;
  out.rel_res = o.b2 > 0 ? std::sqrt(o.rho / o.b2) : 0.0;
  *info = out;
  if (breakdown) return DAMN_ERR_BREAKDOWN;
  return out.converged ? DAMN_OK : DAMN_ERR_NOT_CONVERGED;
}

}  // namespace
}  // namespace damn

using namespace damn;

extern "C" int damn_cg(damn_mat A64, damn_mat A32, const double* b, double* x,
                       const damn_cg_opts* opts, damn_cg_info* info, void* stream) {
  int st = check_args(A64, A32, b, x, opts, info);
  if (st != DAMN_OK) return st;
  damn_cg_work* w = nullptr;
  st = get_work(A64, partial_count(A64, A32), A32 != nullptr, &w);
  if (st != DAMN_OK) return st;
  return solve(A64, A32, b, x, opts, info, w, static_cast<hipStream_t>(stream));
}
