// The remaining cells of the storage grid of Fig. 3: 8-bit DA offsets and
// 16-bit CSR columns with float64, float32 and float16 values, and float16
// values with 16-bit DA offsets and 32-bit CSR columns.  Float16 values are
// widened to float32 as they are used; x, y and the sums are float32.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "damn_kernels.h"
#include "spmv_templates.h"

namespace damn {
namespace {

template <typename I, bool DA>
hipError_t by_store(const SpmvArgs& a, int variant, int lanes, int unroll) {
  switch (a.store) {
    case DAMN_F64: return launch::product<I, DA, double, double>(a, variant, lanes, unroll);
    case DAMN_F32: return launch::product<I, DA, float, float>(a, variant, lanes, unroll);
    default: return launch::product<I, DA, _Float16, float>(a, variant, lanes, unroll);
  }
}

}  // namespace

hipError_t launch_spmv_grid(const SpmvArgs& a, int variant, int lanes, int unroll) {
  switch (a.format) {
    case DAMN_FORMAT_DA8: return by_store<int8_t, true>(a, variant, lanes, unroll);
    case DAMN_FORMAT_CSR16: return by_store<int16_t, false>(a, variant, lanes, unroll);
    case DAMN_FORMAT_DA16:  // float16 values only (the others are in spmv_kernels.hip)
      return launch::product<int16_t, true, _Float16, float>(a, variant, lanes, unroll);
    default:
      return launch::product<int32_t, false, _Float16, float>(a, variant, lanes, unroll);
  }
}

}  // namespace damn
