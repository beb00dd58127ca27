// Native CPU baseline of the products, for comparison only (not part of
// libdamn.so and never a fallback for it): DA-CSR (int16 offsets) and CSR
// (int32 columns) SpMV y = A x in float64, rows split statically over
// OpenMP threads, each row summed with four independent partial sums.  The
// DA rows shift x once per row and index it with the offset (the shifted-x
// access of Sec. 4); the paper's own CPU kernels use 1-8 accumulators and
// OpenMP (Sec. 4.1).
#include <omp.h>

#include <cstdint>

namespace {

template <typename I, bool DA>
void spmv(int32_t nrows, const int32_t* rowptr, const I* idx, const double* val, const double* x,
          double* y, int threads) {
#pragma omp parallel for schedule(static) num_threads(threads)
  for (int32_t r = 0; r < nrows; ++r) {
    const double* xs = DA ? x + r : x;
    const int32_t e = rowptr[r + 1];
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int32_t k = rowptr[r];
    for (; k + 3 < e; k += 4) {
      a0 += val[k] * xs[idx[k]];
      a1 += val[k + 1] * xs[idx[k + 1]];
      a2 += val[k + 2] * xs[idx[k + 2]];
      a3 += val[k + 3] * xs[idx[k + 3]];
    }
    for (; k < e; ++k) a0 += val[k] * xs[idx[k]];
    y[r] = (a0 + a1) + (a2 + a3);
  }
}

}  // namespace

extern "C" {

int damn_cpu_threads(void) { return omp_get_max_threads(); }

void damn_cpu_spmv_da(int32_t nrows, const int32_t* rowptr, const int16_t* off, const double* val,
                      const double* x, double* y, int threads) {
  spmv<int16_t, true>(nrows, rowptr, off, val, x, y, threads);
}

void damn_cpu_spmv_csr(int32_t nrows, const int32_t* rowptr, const int32_t* col,
                       const double* val, const double* x, double* y, int threads) {
  spmv<int32_t, false>(nrows, rowptr, col, val, x, y, threads);
}

}  // extern "C"
