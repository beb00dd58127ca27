// Row reduction of the SpMM stream kernel:
// Y[r, :] <- alpha * A[r, :] X + beta * Y[r, :] for the rows of one tile
// whose entries, indices and row pointers already sit in LDS (Sec. 4's
// product repeated over NRHS vectors).  X is ncols x NRHS and Y nrows x NRHS,
// row-major, so the NRHS values of one row are adjacent.
//
// Each row gets G lanes of a wave.  The NRHS values of a row are cut into
// pieces of PW = 2 doubles (PAIRS: 16-byte loads and stores; NRHS even, X
// and Y 16-byte aligned) or of one double.  When the piece count NP is a
// power of two, the row's lanes split over pieces first: PL = min(G, NP)
// lanes take neighbouring pieces of the same entry and G / PL lanes step
// through the entries.  One gather instruction then reads whole runs of
// neighbouring X rows (the rows r + off for neighbouring r), instead of one
// piece of each; a wavefront touches a quarter as many cache lines at
// NRHS = 8.  Other piece counts keep all pieces in every lane (PL = 1).
//
// Where a lane holds at most two sums (NRHS <= 4), spmm_tile_rows_deep
// (compile-time G) loads up to eight entries' X pieces before using any.
//
// The batched kernel keeps its own unsplit reduction: it inlines every
// right-hand-side count into one kernel, and with this reduction the merged
// kernel needs about 96 VGPRs instead of 60, which costs it more occupancy
// than the split gains.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "damn_device.h"

namespace damn {
namespace kern {

typedef double spmm_d2 __attribute__((ext_vector_type(2)));

template <typename I, bool DA, int NRHS, bool PAIRS>
__device__ __forceinline__ void spmm_tile_rows(int G, int32_t r0, int32_t r1, int32_t a0,
                                               int32_t ar, const double* __restrict__ val_s,
                                               const I* __restrict__ idx_s,
                                               const int32_t* __restrict__ rp_s,
                                               const double* __restrict__ X,
                                               double* __restrict__ Y, double alpha, double beta,
                                               bool read_y) {
  constexpr int PW = PAIRS ? 2 : 1;
  constexpr int NP = NRHS / PW;
  constexpr bool kSplit = (NP & (NP - 1)) == 0;
  const int PL = kSplit ? (G < NP ? G : NP) : 1;  // lanes over pieces
  const int npl = NP / PL;                         // pieces per lane
  // A wave holds 64 / G rows.  Lane l takes piece l mod PL, row
  // (l / PL) mod (64 / G) of the wave's rows and entry group l / (PL * 64/G):
  // the lanes of one entry group read the pieces of neighbouring rows'
  // X rows, a contiguous run for banded matrices.
  const int RPW = 64 / G;
  const int wl = int(threadIdx.x & 63);
  const int p = wl % PL;                // first piece of this lane
  const int EL = G / PL;                // lanes over entries
  const int g = wl / (PL * RPW);        // this lane's first entry
  const int rw = (wl / PL) % RPW;       // this lane's row in the wave
  // two entries in flight when a lane holds at most 4 sums (the second set
  // in acc2); more would cost occupancy
  constexpr int T = NRHS < 4 ? NRHS : 4;
  const bool twin = npl * PW <= T;
  for (int32_t r = r0 + int32_t(threadIdx.x >> 6) * RPW + rw; r < r1; r += 256 / G) {
    const int32_t s = rp_s[r - ar] - a0, e = rp_s[r + 1 - ar] - a0;
    const double* Xs = DA ? X + int64_t(r) * NRHS : X;
    double acc[NRHS], acc2[T];
#pragma unroll
    for (int j = 0; j < NRHS; ++j) acc[j] = 0.0;
#pragma unroll
    for (int j = 0; j < T; ++j) acc2[j] = 0.0;
    auto add = [&](auto& a, int32_t k) {
      constexpr int N = sizeof(a) / sizeof(double);
      const double v = val_s[k];
      const double* xr = Xs + int64_t(idx_s[k]) * NRHS;
#pragma unroll
      for (int i = 0; i < NP; ++i) {
        if ((i + 1) * PW <= N && i < npl) {
          const int q = p + i * PL;
          if (PAIRS) {
            const spmm_d2 xv = reinterpret_cast<const spmm_d2*>(xr)[q];
            a[2 * i] += v * xv.x;
            a[2 * i + 1] += v * xv.y;
          } else {
            a[i] += v * xr[q];
          }
        }
      }
    };
    int32_t k = s + g;
    if (twin) {
      for (; k + EL < e; k += 2 * EL) {
        add(acc, k);
        add(acc2, k + EL);
      }
    }
    for (; k < e; k += EL) add(acc, k);
#pragma unroll
    for (int j = 0; j < NRHS; ++j) {
      if (j < npl * PW) {
        if (j < T) acc[j] += acc2[j];
        // sum over the lanes of this row that hold the same pieces
        for (int o = 32; o >= PL * RPW; o >>= 1) acc[j] += __shfl_xor(acc[j], o, 64);
      }
    }
    if (g == 0) {
      double* yr = Y + int64_t(r) * NRHS;
#pragma unroll
      for (int i = 0; i < NP; ++i) {
        if (i < npl) {
          const int q = p + i * PL;
          if (PAIRS) {
            spmm_d2 out;
            out.x = finish(acc[2 * i], alpha, beta, read_y, yr + 2 * q);
            out.y = finish(acc[2 * i + 1], alpha, beta, read_y, yr + 2 * q + 1);
            reinterpret_cast<spmm_d2*>(yr)[q] = out;
          } else {
            yr[q] = finish(acc[i], alpha, beta, read_y, yr + q);
          }
        }
      }
    }
  }
}


// The same reduction with compile-time G for small per-lane sum counts:
// when a lane holds at most two sums (NRHS <= 4 split over the row's
// lanes), it loads the X pieces of up to eight of its entries before using
// any, so a 27-point row's share is in flight at once (27-point 128^3,
// four lanes, 2048-entry tiles: nrhs 2 116.0 -> 110.8 us, nrhs 4
// 143.5 -> 136.1 us; with six entries in flight no gain, and nrhs 8, at
// four sums per lane, is bound by the data its gathers return).
template <int G, int NRHS, bool PAIRS>
struct SpmmDeep {
  static constexpr int PW = PAIRS ? 2 : 1;
  static constexpr int NP = NRHS / PW;
  static constexpr bool kSplit = (NP & (NP - 1)) == 0;
  static constexpr int PL = kSplit ? (G < NP ? G : NP) : 1;
  static constexpr int NS = (NP / PL) * PW;  // sums per lane
  static constexpr bool kUse = NRHS <= 4 && NS <= 2;
};

template <typename I, bool DA, int G, int NRHS, bool PAIRS>
__device__ __forceinline__ void spmm_tile_rows_deep(int32_t r0, int32_t r1, int32_t a0,
                                                    int32_t ar, const double* __restrict__ val_s,
                                                    const I* __restrict__ idx_s,
                                                    const int32_t* __restrict__ rp_s,
                                                    const double* __restrict__ X,
                                                    double* __restrict__ Y, double alpha,
                                                    double beta, bool read_y) {
  using K = SpmmDeep<G, NRHS, PAIRS>;
  constexpr int PL = K::PL, NS = K::NS, npl = K::NP / K::PL;
  constexpr int UE = 16 / NS;  // entries in flight per lane
  constexpr int RPW = 64 / G;
  constexpr int EL = G / PL;   // lanes over entries
  const int wl = int(threadIdx.x & 63);
  const int p = wl % PL;
  const int g = wl / (PL * RPW);
  const int rw = (wl / PL) % RPW;
  for (int32_t r = r0 + int32_t(threadIdx.x >> 6) * RPW + rw; r < r1; r += 256 / G) {
    const int32_t s = rp_s[r - ar] - a0, e = rp_s[r + 1 - ar] - a0;
    const double* Xs = DA ? X + int64_t(r) * NRHS : X;
    double acc[NS];
#pragma unroll
    for (int j = 0; j < NS; ++j) acc[j] = 0.0;
    for (int32_t k0 = s + g; k0 < e; k0 += UE * EL) {
      double xv[UE][NS];
      double vv[UE];
#pragma unroll
      for (int u = 0; u < UE; ++u) {
        const int32_t k = k0 + u * EL;
        if (k < e) {
          vv[u] = val_s[k];
          const double* xr = Xs + int64_t(idx_s[k]) * NRHS;
#pragma unroll
          for (int i = 0; i < npl; ++i) {
            const int q = p + i * PL;
            if (PAIRS) {
              const spmm_d2 t = reinterpret_cast<const spmm_d2*>(xr)[q];
              xv[u][2 * i] = t.x;
              xv[u][2 * i + 1] = t.y;
            } else {
              xv[u][i] = xr[q];
            }
          }
        } else {
          vv[u] = 0.0;
#pragma unroll
          for (int j = 0; j < NS; ++j) xv[u][j] = 0.0;
        }
      }
#pragma unroll
      for (int u = 0; u < UE; ++u) {
        if (k0 + u * EL < e) {
#pragma unroll
          for (int j = 0; j < NS; ++j) acc[j] += vv[u] * xv[u][j];
        }
      }
    }
#pragma unroll
    for (int j = 0; j < NS; ++j)
      for (int o = 32; o >= PL * RPW; o >>= 1) acc[j] += __shfl_xor(acc[j], o, 64);
    if (g == 0) {
      double* yr = Y + int64_t(r) * NRHS;
#pragma unroll
      for (int i = 0; i < npl; ++i) {
        const int q = p + i * PL;
        if (PAIRS) {
          spmm_d2 out;
          out.x = finish(acc[2 * i], alpha, beta, read_y, yr + 2 * q);
          out.y = finish(acc[2 * i + 1], alpha, beta, read_y, yr + 2 * q + 1);
          reinterpret_cast<spmm_d2*>(yr)[q] = out;
        } else {
          yr[q] = finish(acc[i], alpha, beta, read_y, yr + q);
        }
      }
    }
  }
}

}  // namespace kern
}  // namespace damn
