// Launch-configuration selection: the exhaustive autotuner and a small
// multilayer perceptron that predicts its choice from sparsity features.
//
// Classes (DAMN_NCLASS = 70):
//   0..20   vector variant, lanes {1,2,4,...,64} x unroll {1,2,4}  (nrhs = 1)
//   21..41  stream variant, interleaved gathers, lanes {1,...,64} x tile
//           {1024,2048,4096}                                        (nrhs = 1)
//   42..62  stream variant, paired gathers, the same lanes x tiles  (nrhs = 1)
//   63..69  SpMM (stream, 2048-entry tiles), lanes {1,...,64}        (nrhs > 1)
//
// Network: x = (f - mu) / sigma (16 features), h1 = relu(W1 x + b1) (64),
// h2 = relu(W2 h1 + b2) (64), z = W3 h2 + b3 (70); classes that do not apply
// to the sample's nrhs are masked out of the softmax.  Training minimises the
// cross entropy against soft targets q_c ~ exp(-(t_c / t_min - 1) / tau)
// built from autotuner times, with Adam.  All network arithmetic runs in
// float32 on the GPU: one workgroup per sample for the forward and backward
// passes through the activations, one thread per parameter for the weight
// gradients (summed over the minibatch in a fixed order), one thread per
// parameter for the Adam step.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <mutex>
#include <new>
#include <vector>

#include "damn.h"
#include "damn_mat.h"

namespace damn {
namespace sel {

constexpr int F = DAMN_NFEAT;    // 16
constexpr int H = 64;            // hidden width
constexpr int K = DAMN_NCLASS;   // 70
constexpr int kSpmm0 = DAMN_CLASS_SPMM;  // first SpMM class
constexpr int kW1 = 0, kB1 = kW1 + H * F, kW2 = kB1 + H, kB2 = kW2 + H * H, kW3 = kB2 + H,
              kB3 = kW3 + K * H, kMu = kB3 + K, kSigma = kMu + F, kTotal = kSigma + F;
constexpr int kTrained = kMu;    // parameters before mu/sigma are trained
static_assert(kTotal == DAMN_MLP_NPARAMS, "parameter layout");
static_assert(K <= 2 * H, "a workgroup of H threads handles at most two classes per thread");

constexpr int kLanes[7] = {1, 2, 4, 8, 16, 32, 64};
constexpr int kUnrolls[3] = {1, 2, 4};
constexpr int kTiles[3] = {1024, 2048, 4096};

__device__ __forceinline__ bool class_valid(int k, float nrhs) {
  return nrhs > 1.5f ? k >= kSpmm0 : k < kSpmm0;
}

// Forward pass of one sample (H = 64 threads; thread t computes the logits
// of classes t and t + H); leaves x, h1, h2, z in LDS.
__device__ void forward_one(const float* __restrict__ P, const float* __restrict__ f,
                            float* xs, float* h1, float* h2, float* z) {
  const int t = threadIdx.x;
  if (t < F) xs[t] = (f[t] - P[kMu + t]) / P[kSigma + t];
  __syncthreads();
  float a = P[kB1 + t];
  for (int i = 0; i < F; ++i) a += P[kW1 + t * F + i] * xs[i];
  h1[t] = a > 0.f ? a : 0.f;
  __syncthreads();
  a = P[kB2 + t];
  for (int i = 0; i < H; ++i) a += P[kW2 + t * H + i] * h1[i];
  h2[t] = a > 0.f ? a : 0.f;
  __syncthreads();
  for (int k = t; k < K; k += H) {
    a = P[kB3 + k];
    for (int i = 0; i < H; ++i) a += P[kW3 + k * H + i] * h2[i];
    z[k] = a;
  }
  __syncthreads();
}

// Workgroup b handles sample idx[b]: forward, masked softmax, dZ = (p-q)/B,
// per-sample loss, and the back-propagated dH2, dH1.  Activations are kept
// per minibatch row b for the weight gradients.
__global__ __launch_bounds__(64) void fwd_bwd(const float* __restrict__ P,
                                              const float* __restrict__ feats,
                                              const float* __restrict__ targets,
                                              const int32_t* __restrict__ idx, int32_t B,
                                              float* __restrict__ X, float* __restrict__ A1,
                                              float* __restrict__ A2, float* __restrict__ dZ,
                                              float* __restrict__ dH2, float* __restrict__ dH1,
                                              float* __restrict__ loss) {
  __shared__ float xs[F], h1[H], h2[H], z[K], dz[K], dh2[H], terms[K];
  __shared__ float red[2];
  const int b = blockIdx.x, t = threadIdx.x;
  const int s = idx[b];
  const float* f = feats + int64_t(s) * F;
  forward_one(P, f, xs, h1, h2, z);
  const float nrhs = f[9];
  // masked softmax (lane 0 does the small reductions in a fixed order)
  if (t == 0) {
    float m = -INFINITY;
    for (int k = 0; k < K; ++k)
      if (class_valid(k, nrhs)) m = fmaxf(m, z[k]);
    float sum = 0.f;
    for (int k = 0; k < K; ++k)
      if (class_valid(k, nrhs)) sum += expf(z[k] - m);
    red[0] = m;
    red[1] = sum;
  }
  __syncthreads();
  for (int k = t; k < K; k += H) {
    const bool valid = class_valid(k, nrhs);
    const float q = targets[int64_t(s) * K + k];
    const float p = valid ? expf(z[k] - red[0]) / red[1] : 0.f;
    dz[k] = valid ? (p - q) / float(B) : 0.f;
    // loss term -q log p, log p = z - m - log(sum)
    terms[k] = (valid && q > 0.f) ? -q * (z[k] - red[0] - logf(red[1])) : 0.f;
  }
  __syncthreads();
  if (t < F) X[b * F + t] = xs[t];
  A1[b * H + t] = h1[t];
  A2[b * H + t] = h2[t];
  for (int k = t; k < K; k += H) dZ[b * K + k] = dz[k];
  // dH2 = W3^T dZ masked by relu; dH1 = W2^T dH2 masked by relu
  float g = 0.f;
  for (int k = 0; k < K; ++k) g += P[kW3 + k * H + t] * dz[k];
  g = h2[t] > 0.f ? g : 0.f;
  dh2[t] = g;
  dH2[b * H + t] = g;
  __syncthreads();
  g = 0.f;
  for (int j = 0; j < H; ++j) g += P[kW2 + j * H + t] * dh2[j];
  dH1[b * H + t] = h1[t] > 0.f ? g : 0.f;
  // per-sample loss: sum of the class terms in class order
  if (t == 0) {
    float l = 0.f;
    for (int k = 0; k < K; ++k) l += terms[k];
    loss[b] = l;
  }
}

// Weight gradients: thread per trained parameter, summed over the minibatch
// rows 0..B-1 in order.
__global__ __launch_bounds__(256) void grad_params(int32_t B, const float* __restrict__ X,
                                                   const float* __restrict__ A1,
                                                   const float* __restrict__ A2,
                                                   const float* __restrict__ dZ,
                                                   const float* __restrict__ dH2,
                                                   const float* __restrict__ dH1,
                                                   float* __restrict__ G) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= kTrained) return;
  float s = 0.f;
  if (p < kB1) {
    const int j = (p - kW1) / F, i = (p - kW1) % F;
    for (int b = 0; b < B; ++b) s += dH1[b * H + j] * X[b * F + i];
  } else if (p < kW2) {
    const int j = p - kB1;
    for (int b = 0; b < B; ++b) s += dH1[b * H + j];
  } else if (p < kB2) {
    const int j = (p - kW2) / H, i = (p - kW2) % H;
    for (int b = 0; b < B; ++b) s += dH2[b * H + j] * A1[b * H + i];
  } else if (p < kW3) {
    const int j = p - kB2;
    for (int b = 0; b < B; ++b) s += dH2[b * H + j];
  } else if (p < kB3) {
    const int k = (p - kW3) / H, j = (p - kW3) % H;
    for (int b = 0; b < B; ++b) s += dZ[b * K + k] * A2[b * H + j];
  } else {
    const int k = p - kB3;
    for (int b = 0; b < B; ++b) s += dZ[b * K + k];
  }
  G[p] = s;
}

__global__ __launch_bounds__(256) void adam_step(float* __restrict__ P, const float* __restrict__ G,
                                                 float* __restrict__ m, float* __restrict__ v,
                                                 float lr, float c1, float c2) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= kTrained) return;
  const float g = G[p];
  const float mn = 0.9f * m[p] + 0.1f * g;
  const float vn = 0.999f * v[p] + 0.001f * g * g;
  m[p] = mn;
  v[p] = vn;
  P[p] -= lr * (mn / c1) / (sqrtf(vn / c2) + 1e-8f);
}

// sum of the per-sample losses of one minibatch into acc[slot] (one thread)
__global__ void add_loss(const float* __restrict__ loss, int32_t B, float* __restrict__ acc,
                         int32_t slot) {
  float s = 0.f;
  for (int b = 0; b < B; ++b) s += loss[b];
  acc[slot] += s;
}

// inference: most probable valid class (lowest index on ties)
// The most probable applicable class of each row, and (prob != nullptr) its
// probability under the softmax over the applicable classes.
__global__ __launch_bounds__(64) void select_cls(const float* __restrict__ P,
                                                 const float* __restrict__ feats,
                                                 int32_t* __restrict__ out,
                                                 float* __restrict__ prob) {
  __shared__ float xs[F], h1[H], h2[H], z[K];
  const int s = blockIdx.x;
  const float* f = feats + int64_t(s) * F;
  forward_one(P, f, xs, h1, h2, z);
  if (threadIdx.x == 0) {
    int best = -1;
    for (int k = 0; k < K; ++k)
      if (class_valid(k, f[9]) && (best < 0 || z[k] > z[best])) best = k;
    out[s] = best;
    if (prob) {
      float sum = 0.0f;
      for (int k = 0; k < K; ++k)
        if (class_valid(k, f[9])) sum += expf(z[k] - z[best]);
      prob[s] = 1.0f / sum;
    }
  }
}

// Fixed device array of damn_select_noalloc: the feature rows, classes and
// probabilities of up to kNoAllocMax rows.  Every GPU the library runs on
// holds its own copy at its own address, found with hipGetSymbolAddress;
// in host code the array's name is not a device address and is never
// passed to a kernel or a copy.
constexpr int32_t kNoAllocMax = DAMN_SELECT_NOALLOC_MAX_ROWS;
constexpr size_t kNoAllocFeatOff = 0;
constexpr size_t kNoAllocClsOff = kNoAllocFeatOff + sizeof(float) * F * size_t(kNoAllocMax);
constexpr size_t kNoAllocProbOff = kNoAllocClsOff + sizeof(int32_t) * size_t(kNoAllocMax);
constexpr size_t kNoAllocBytes = kNoAllocProbOff + sizeof(float) * size_t(kNoAllocMax);
static_assert(kNoAllocClsOff % 256 == 0 && kNoAllocProbOff % 256 == 0, "scratch layout");
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
unsigned char* g_scratch[kMaxDevices] = {};

// The device address of `scratch` on device `dev` (the current device),
// looked up on the first call there and kept.
int noalloc_scratch(int dev, unsigned char** out) {
  if (dev < 0 || dev >= kMaxDevices) return DAMN_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (g_scratch[dev] == nullptr) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr)
      return DAMN_ERR_HIP;
    g_scratch[dev] = static_cast<unsigned char*>(p);
  }
  *out = g_scratch[dev];
  return DAMN_OK;
}

// splitmix64, for initial weights and minibatch shuffles
inline uint64_t mix(uint64_t& x) {
  uint64_t z = (x += 0x9e3779b97f4a7c15ull);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}
inline double uniform01(uint64_t& x) { return double(mix(x) >> 11) * (1.0 / 9007199254740992.0); }

}  // namespace sel
}  // namespace damn

struct damn_mlp_s {
  int device = 0;
  float* P = nullptr;  // parameters, device
  float* m = nullptr;  // Adam moments
  float* v = nullptr;
  int64_t step = 0;
};

using namespace damn;

namespace {

int mlp_alloc(damn_mlp M) {
  const size_t bytes = sizeof(float) * sel::kTotal;
  if (hipMalloc(&M->P, bytes) != hipSuccess || hipMalloc(&M->m, bytes) != hipSuccess ||
      hipMalloc(&M->v, bytes) != hipSuccess)
    return DAMN_ERR_ALLOC;
  if (hipMemset(M->m, 0, bytes) != hipSuccess || hipMemset(M->v, 0, bytes) != hipSuccess)
    return DAMN_ERR_HIP;
  return DAMN_OK;
}

void mlp_free(damn_mlp M) {
  if (!M) return;
  if (M->P) hipFree(M->P);
  if (M->m) hipFree(M->m);
  if (M->v) hipFree(M->v);
  delete M;
}

// Device buffers of one minibatch pass.
struct Pass {
  float *X = nullptr, *A1 = nullptr, *A2 = nullptr, *dZ = nullptr, *dH2 = nullptr,
        *dH1 = nullptr, *loss = nullptr, *G = nullptr;
  int32_t* idx = nullptr;
  int alloc(int32_t B) {
    using namespace sel;
    bool ok = hipMalloc(&X, sizeof(float) * B * F) == hipSuccess &&
              hipMalloc(&A1, sizeof(float) * B * H) == hipSuccess &&
              hipMalloc(&A2, sizeof(float) * B * H) == hipSuccess &&
              hipMalloc(&dZ, sizeof(float) * B * K) == hipSuccess &&
              hipMalloc(&dH2, sizeof(float) * B * H) == hipSuccess &&
              hipMalloc(&dH1, sizeof(float) * B * H) == hipSuccess &&
              hipMalloc(&loss, sizeof(float) * B) == hipSuccess &&
              hipMalloc(&G, sizeof(float) * kTotal) == hipSuccess &&
              hipMalloc(&idx, sizeof(int32_t) * B) == hipSuccess;
    return ok ? DAMN_OK : DAMN_ERR_ALLOC;
  }
  ~Pass() {
    for (void* p : {(void*)X, (void*)A1, (void*)A2, (void*)dZ, (void*)dH2, (void*)dH1,
                    (void*)loss, (void*)G, (void*)idx})
      if (p) hipFree(p);
  }
  // forward + backward over B samples feats/targets (device) rows idx
  void run(const float* P, const float* feats, const float* targets, int32_t B,
           hipStream_t s) {
    hipLaunchKernelGGL(sel::fwd_bwd, dim3(B), dim3(64), 0, s, P, feats, targets, idx, B, X, A1,
                       A2, dZ, dH2, dH1, loss);
    hipLaunchKernelGGL(sel::grad_params, dim3((sel::kTrained + 255) / 256), dim3(256), 0, s, B,
                       X, A1, A2, dZ, dH2, dH1, G);
  }
};

// soft targets from times (+inf or NaN = not applicable); false if a sample
// has no finite time
bool soft_targets(int32_t N, const float* times, float tau, std::vector<float>& Q) {
  using namespace sel;
  Q.assign(size_t(N) * K, 0.f);
  for (int32_t s = 0; s < N; ++s) {
    const float* t = times + int64_t(s) * K;
    double tmin = INFINITY;
    for (int k = 0; k < K; ++k)
      if (std::isfinite(t[k]) && t[k] > 0) tmin = std::min(tmin, double(t[k]));
    if (!std::isfinite(tmin)) return false;
    double sum = 0;
    for (int k = 0; k < K; ++k)
      if (std::isfinite(t[k]) && t[k] > 0) sum += std::exp(-(double(t[k]) / tmin - 1.0) / tau);
    for (int k = 0; k < K; ++k)
      if (std::isfinite(t[k]) && t[k] > 0)
        Q[size_t(s) * K + k] = float(std::exp(-(double(t[k]) / tmin - 1.0) / tau) / sum);
  }
  return true;
}

}  // namespace

extern "C" {

int damn_class_config(int32_t cls, damn_config* cfg, int32_t* spmm) {
  if (cfg == nullptr || cls < 0 || cls >= DAMN_NCLASS) return DAMN_ERR_INVALID_ARG;
  damn_config c{};
  int32_t mm = 0;
  if (cls < 21) {
    c.variant = DAMN_VAR_VECTOR;
    c.lanes = sel::kLanes[cls / 3];
    c.unroll = sel::kUnrolls[cls % 3];
    c.tile = 2048;
  } else if (cls < sel::kSpmm0) {
    const int32_t j = (cls - 21) % 21;
    c.variant = DAMN_VAR_STREAM;
    c.lanes = sel::kLanes[j / 3];
    c.unroll = cls < 42 ? 1 : 2;  // interleaved or paired gathers
    c.tile = sel::kTiles[j % 3];
  } else {
    c.variant = DAMN_VAR_STREAM;  // the stream SpMM, 2048-entry tiles
    c.lanes = sel::kLanes[cls - sel::kSpmm0];
    c.unroll = 1;
    c.tile = 2048;
    mm = 1;
  }
  *cfg = c;
  if (spmm) *spmm = mm;
  return DAMN_OK;
}

int damn_autotune(damn_mat A, int32_t nrhs, const void* X, void* Y, int32_t reps, float* times,
                  void* stream) {
  if (A == nullptr || times == nullptr || nrhs < 1 || nrhs > 8 || reps < 1)
    return DAMN_ERR_INVALID_ARG;
  if (nrhs > 1 && A->dtype != DAMN_F64) return DAMN_ERR_UNSUPPORTED;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) hipEventDestroy(e0);
    return DAMN_ERR_HIP;
  }
  const damn_config saved = A->cfg;
  int best = -1;
  int st = DAMN_OK;
  for (int k = 0; k < DAMN_NCLASS && st == DAMN_OK; ++k) {
    times[k] = std::numeric_limits<float>::infinity();
    damn_config c;
    int32_t mm;
    damn_class_config(k, &c, &mm);
    if ((nrhs > 1) != (mm != 0)) continue;
    st = damn_set_config(A, &c);
    if (st == DAMN_ERR_UNSUPPORTED && c.unroll == 2 && c.variant == DAMN_VAR_STREAM) {
      st = DAMN_OK;  // paired gathers do not apply to this handle's cell
      continue;
    }
    if (st != DAMN_OK) break;
    auto once = [&]() {
      if (nrhs > 1) return damn_spmm(A, X, Y, nrhs, 1.0, 0.0, stream);
      return A->format == DAMN_FORMAT_DA16 || A->format == DAMN_FORMAT_DA8
                 ? damn_spmv(A, X, Y, 1.0, 0.0, stream)
                 : damn_csr_spmv(A, X, Y, 1.0, 0.0, stream);
    };
    st = once();  // warm
    if (st != DAMN_OK) break;
    if (hipEventRecord(e0, s) != hipSuccess) { st = DAMN_ERR_HIP; break; }
    for (int r = 0; r < reps && st == DAMN_OK; ++r) st = once();
    if (st != DAMN_OK) break;
    float ms = 0;
    if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
      st = DAMN_ERR_HIP;
      break;
    }
    times[k] = ms * 1e-3f / float(reps);
    if (best < 0 || times[k] < times[best]) best = k;
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (st != DAMN_OK || best < 0) {
    damn_set_config(A, &saved);
    return st != DAMN_OK ? st : DAMN_ERR_HIP;
  }
  damn_config c;
  damn_class_config(best, &c, nullptr);
  return damn_set_config(A, &c);
}

int damn_mlp_create(damn_mlp* out, const float* params, uint64_t seed) {
  if (out == nullptr) return DAMN_ERR_INVALID_ARG;
  damn_mlp M = new (std::nothrow) damn_mlp_s();
  if (!M) return DAMN_ERR_ALLOC;
  hipGetDevice(&M->device);
  int st = mlp_alloc(M);
  if (st != DAMN_OK) {
    mlp_free(M);
    return st;
  }
  std::vector<float> h(sel::kTotal, 0.f);
  if (params) {
    std::memcpy(h.data(), params, sizeof(float) * sel::kTotal);
  } else {
    // He-uniform weights, zero biases, identity standardisation
    uint64_t x = seed;
    auto fill = [&](int off, int rows, int fan_in) {
      const double a = std::sqrt(6.0 / fan_in);
      for (int i = 0; i < rows * fan_in; ++i) h[off + i] = float((2 * sel::uniform01(x) - 1) * a);
    };
    fill(sel::kW1, sel::H, sel::F);
    fill(sel::kW2, sel::H, sel::H);
    fill(sel::kW3, sel::K, sel::H);
    for (int i = 0; i < sel::F; ++i) h[sel::kSigma + i] = 1.f;
  }
  if (hipMemcpy(M->P, h.data(), sizeof(float) * sel::kTotal, hipMemcpyHostToDevice) != hipSuccess) {
    mlp_free(M);
    return DAMN_ERR_HIP;
  }
  *out = M;
  return DAMN_OK;
}

int damn_mlp_get_params(damn_mlp M, float* params) {
  if (M == nullptr || params == nullptr) return DAMN_ERR_INVALID_ARG;
  return hipMemcpy(params, M->P, sizeof(float) * sel::kTotal, hipMemcpyDeviceToHost) ==
                 hipSuccess
             ? DAMN_OK
             : DAMN_ERR_HIP;
}

int damn_mlp_grad(damn_mlp M, int32_t B, const float* feats, const float* targets, float* loss,
                  float* grads, void* stream) {
  if (M == nullptr || B < 1 || feats == nullptr || targets == nullptr || loss == nullptr ||
      grads == nullptr)
    return DAMN_ERR_INVALID_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  Pass pass;
  float *df = nullptr, *dq = nullptr;
  int st = pass.alloc(B);
  if (st == DAMN_OK && (hipMalloc(&df, sizeof(float) * B * sel::F) != hipSuccess ||
                        hipMalloc(&dq, sizeof(float) * B * sel::K) != hipSuccess))
    st = DAMN_ERR_ALLOC;
  std::vector<int32_t> idx(B);
  for (int32_t b = 0; b < B; ++b) idx[b] = b;
  std::vector<float> lb(B);
  if (st == DAMN_OK) {
    bool ok =
        hipMemcpyAsync(df, feats, sizeof(float) * B * sel::F, hipMemcpyHostToDevice, s) ==
            hipSuccess &&
        hipMemcpyAsync(dq, targets, sizeof(float) * B * sel::K, hipMemcpyHostToDevice, s) ==
            hipSuccess &&
        hipMemcpyAsync(pass.idx, idx.data(), sizeof(int32_t) * B, hipMemcpyHostToDevice, s) ==
            hipSuccess;
    if (ok) {
      pass.run(M->P, df, dq, B, s);
      ok = hipGetLastError() == hipSuccess &&
           hipMemcpyAsync(lb.data(), pass.loss, sizeof(float) * B, hipMemcpyDeviceToHost, s) ==
               hipSuccess &&
           hipMemcpyAsync(grads, pass.G, sizeof(float) * sel::kTrained, hipMemcpyDeviceToHost,
                          s) == hipSuccess &&
           hipStreamSynchronize(s) == hipSuccess;
    }
    if (!ok) st = DAMN_ERR_HIP;
  }
  if (df) hipFree(df);
  if (dq) hipFree(dq);
  if (st != DAMN_OK) return st;
  float l = 0.f;
  for (int32_t b = 0; b < B; ++b) l += lb[b];
  *loss = l / float(B);
  for (int i = sel::kTrained; i < sel::kTotal; ++i) grads[i] = 0.f;
  return DAMN_OK;
}

int damn_mlp_train(damn_mlp M, int32_t N, const float* feats, const float* times,
                   int32_t epochs, int32_t batch, float lr, float tau, uint64_t seed,
                   float* epoch_loss, void* stream) {
  if (M == nullptr || N < 1 || feats == nullptr || times == nullptr || epochs < 1 ||
      batch < 1 || !(lr > 0.f) || !(tau > 0.f))
    return DAMN_ERR_INVALID_ARG;
  using namespace sel;
  hipStream_t s = static_cast<hipStream_t>(stream);
  std::vector<float> Q;
  if (!soft_targets(N, times, tau, Q)) return DAMN_ERR_INVALID_ARG;
  // standardisation from the training features (population statistics)
  std::vector<float> P(kTotal);
  if (hipMemcpy(P.data(), M->P, sizeof(float) * kTotal, hipMemcpyDeviceToHost) != hipSuccess)
    return DAMN_ERR_HIP;
  for (int j = 0; j < F; ++j) {
    double mu = 0, sq = 0;
    for (int32_t i = 0; i < N; ++i) mu += feats[int64_t(i) * F + j];
    mu /= N;
    for (int32_t i = 0; i < N; ++i) {
      const double d = feats[int64_t(i) * F + j] - mu;
      sq += d * d;
    }
    const double sd = std::sqrt(sq / N);
    P[kMu + j] = float(mu);
    P[kSigma + j] = sd > 1e-6 ? float(sd) : 1.f;
  }
  if (hipMemcpy(M->P, P.data(), sizeof(float) * kTotal, hipMemcpyHostToDevice) != hipSuccess)
    return DAMN_ERR_HIP;
  const int32_t B = std::min(batch, N);
  Pass pass;
  float *df = nullptr, *dq = nullptr, *dl = nullptr;
  int32_t* dperm = nullptr;
  int st = pass.alloc(B);
  if (st == DAMN_OK && (hipMalloc(&df, sizeof(float) * size_t(N) * F) != hipSuccess ||
                        hipMalloc(&dq, sizeof(float) * size_t(N) * K) != hipSuccess ||
                        hipMalloc(&dl, sizeof(float) * epochs) != hipSuccess ||
                        hipMalloc(&dperm, sizeof(int32_t) * N) != hipSuccess))
    st = DAMN_ERR_ALLOC;
  bool ok = st == DAMN_OK &&
            hipMemcpyAsync(df, feats, sizeof(float) * size_t(N) * F, hipMemcpyHostToDevice, s) ==
                hipSuccess &&
            hipMemcpyAsync(dq, Q.data(), sizeof(float) * size_t(N) * K, hipMemcpyHostToDevice,
                           s) == hipSuccess &&
            hipMemsetAsync(dl, 0, sizeof(float) * epochs, s) == hipSuccess;
  std::vector<int32_t> perm(N);
  for (int32_t i = 0; i < N; ++i) perm[i] = i;
  uint64_t rs = seed;
  for (int32_t e = 0; ok && e < epochs; ++e) {
    for (int32_t i = N - 1; i > 0; --i) {  // Fisher-Yates
      const int32_t j = int32_t(mix(rs) % uint64_t(i + 1));
      std::swap(perm[i], perm[j]);
    }
    ok = hipMemcpyAsync(dperm, perm.data(), sizeof(int32_t) * N, hipMemcpyHostToDevice, s) ==
             hipSuccess &&
         hipStreamSynchronize(s) == hipSuccess;
    for (int32_t b0 = 0; ok && b0 + B <= N; b0 += B) {  // full minibatches only
      ok = hipMemcpyAsync(pass.idx, dperm + b0, sizeof(int32_t) * B, hipMemcpyDeviceToDevice,
                          s) == hipSuccess;
      if (!ok) break;
      pass.run(M->P, df, dq, B, s);
      hipLaunchKernelGGL(add_loss, dim3(1), dim3(1), 0, s, pass.loss, B, dl, e);
      ++M->step;
      const float c1 = float(1.0 - std::pow(0.9, double(M->step)));
      const float c2 = float(1.0 - std::pow(0.999, double(M->step)));
      hipLaunchKernelGGL(adam_step, dim3((kTrained + 255) / 256), dim3(256), 0, s, M->P, pass.G,
                         M->m, M->v, lr, c1, c2);
      ok = hipGetLastError() == hipSuccess;
    }
  }
  std::vector<float> hl(epochs, 0.f);
  if (ok)
    ok = hipMemcpyAsync(hl.data(), dl, sizeof(float) * epochs, hipMemcpyDeviceToHost, s) ==
             hipSuccess &&
         hipStreamSynchronize(s) == hipSuccess;
  if (df) hipFree(df);
  if (dq) hipFree(dq);
  if (dl) hipFree(dl);
  if (dperm) hipFree(dperm);
  if (st != DAMN_OK) return st;
  if (!ok) return DAMN_ERR_HIP;
  const int32_t per_epoch = (N / B) * B;
  if (epoch_loss)
    for (int32_t e = 0; e < epochs; ++e) epoch_loss[e] = hl[e] / float(per_epoch);
  return DAMN_OK;
}

int damn_select_prob(damn_mlp M, int32_t N, const float* feats, int32_t* cls, float* prob,
                     void* stream) {
  if (M == nullptr || N < 0 || (N > 0 && (feats == nullptr || cls == nullptr)))
    return DAMN_ERR_INVALID_ARG;
  if (N == 0) return DAMN_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  float* df = nullptr;
  int32_t* dc = nullptr;
  float* dp = nullptr;
  int st = DAMN_OK;
  if (hipMalloc(&df, sizeof(float) * size_t(N) * sel::F) != hipSuccess ||
      hipMalloc(&dc, sizeof(int32_t) * N) != hipSuccess ||
      (prob && hipMalloc(&dp, sizeof(float) * N) != hipSuccess))
    st = DAMN_ERR_ALLOC;
  if (st == DAMN_OK) {
    bool ok = hipMemcpyAsync(df, feats, sizeof(float) * size_t(N) * sel::F,
                             hipMemcpyHostToDevice, s) == hipSuccess;
    if (ok) {
      hipLaunchKernelGGL(sel::select_cls, dim3(N), dim3(64), 0, s, M->P, df, dc, dp);
      ok = hipGetLastError() == hipSuccess &&
           hipMemcpyAsync(cls, dc, sizeof(int32_t) * N, hipMemcpyDeviceToHost, s) ==
               hipSuccess &&
           (!prob || hipMemcpyAsync(prob, dp, sizeof(float) * N, hipMemcpyDeviceToHost, s) ==
                         hipSuccess) &&
           hipStreamSynchronize(s) == hipSuccess;
    }
    if (!ok) st = DAMN_ERR_HIP;
  }
  if (df) hipFree(df);
  if (dc) hipFree(dc);
  if (dp) hipFree(dp);
  return st;
}

int damn_select_noalloc(damn_mlp M, int32_t N, const float* feats, int32_t* cls, float* prob,
                        void* stream) {
  using damn::sel::kNoAllocMax;
  if (M == nullptr || N < 0 || (N > 0 && (feats == nullptr || cls == nullptr)))
    return DAMN_ERR_INVALID_ARG;
  if (N > kNoAllocMax) return DAMN_ERR_TOO_LARGE;
  if (N == 0) return DAMN_OK;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return DAMN_ERR_HIP;
  if (dev != M->device) return DAMN_ERR_INVALID_ARG;
  unsigned char* base = nullptr;
  const int st = damn::sel::noalloc_scratch(dev, &base);
  if (st != DAMN_OK) return st;
  float* df = reinterpret_cast<float*>(base + damn::sel::kNoAllocFeatOff);
  int32_t* dc = reinterpret_cast<int32_t*>(base + damn::sel::kNoAllocClsOff);
  float* dp = prob ? reinterpret_cast<float*>(base + damn::sel::kNoAllocProbOff) : nullptr;
  hipStream_t s = static_cast<hipStream_t>(stream);
  bool ok = hipMemcpyAsync(df, feats, sizeof(float) * size_t(N) * damn::sel::F,
                           hipMemcpyHostToDevice, s) == hipSuccess;
  if (ok) {
    hipLaunchKernelGGL(damn::sel::select_cls, dim3(N), dim3(64), 0, s, M->P, df, dc, dp);
    ok = hipGetLastError() == hipSuccess &&
         hipMemcpyAsync(cls, dc, sizeof(int32_t) * N, hipMemcpyDeviceToHost, s) == hipSuccess &&
         (!prob || hipMemcpyAsync(prob, dp, sizeof(float) * N, hipMemcpyDeviceToHost, s) ==
                       hipSuccess) &&
         hipStreamSynchronize(s) == hipSuccess;
  }
  return ok ? DAMN_OK : DAMN_ERR_HIP;
}

int damn_select(damn_mlp M, int32_t N, const float* feats, int32_t* cls, void* stream) {
  return damn_select_prob(M, N, feats, cls, nullptr, stream);
}

int damn_mlp_destroy(damn_mlp M) {
  if (M == nullptr) return DAMN_ERR_INVALID_ARG;
  hipDeviceSynchronize();
  mlp_free(M);
  return DAMN_OK;
}

}  // extern "C"
