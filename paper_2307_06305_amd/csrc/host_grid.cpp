// Host-side conversion into the storage grid of Fig. 3: column indices of
// 8, 16 or 32 bits (DA offsets c - r of Sec. 2, or absolute columns) and
// scalars of 64, 32 or 16 bits.  Pure C++; no GPU calls.
#include <cmath>
#include <cstdint>
#include <cstring>

#include "damn.h"
#include "damn_internal.h"

namespace damn {

int index_bytes(int32_t format) {
  switch (format) {
    case DAMN_FORMAT_DA16: return 2;
    case DAMN_FORMAT_CSR32: return 4;
    case DAMN_FORMAT_DA8: return 1;
    case DAMN_FORMAT_CSR16: return 2;
    case DAMN_FORMAT_DABSR16: return 2;
    case DAMN_FORMAT_BSR32: return 4;
    case DAMN_FORMAT_DACOO16: return 2;
    case DAMN_FORMAT_COO32: return 4;
    default: return 0;
  }
}

bool format_is_da(int32_t format) {
  return format == DAMN_FORMAT_DA16 || format == DAMN_FORMAT_DA8 ||
         format == DAMN_FORMAT_DABSR16 || format == DAMN_FORMAT_DACOO16;
}

bool format_is_coo(int32_t format) {
  return format == DAMN_FORMAT_DACOO16 || format == DAMN_FORMAT_COO32;
}

bool format_is_block(int32_t format) {
  return format == DAMN_FORMAT_DABSR16 || format == DAMN_FORMAT_BSR32;
}

int value_bytes(int32_t dtype) {
  switch (dtype) {
    case DAMN_F64: return 8;
    case DAMN_F32: return 4;
    case DAMN_F16: return 2;
    default: return 0;
  }
}

// IEEE 754 binary64 -> binary16 bits, round to nearest with ties to even,
// in one step from the binary64 value.  binary16: sign, 5-bit exponent with
// bias 15, 10-bit fraction; normal numbers 2^-14 .. 65504, subnormals in
// steps of 2^-24.  *overflow is set when a finite value rounds to infinity.
uint16_t f64_to_f16_bits(double d, bool* overflow) {
  uint64_t b;
  std::memcpy(&b, &d, sizeof b);
  const uint16_t sign = uint16_t((b >> 48) & 0x8000u);
  const int e = int((b >> 52) & 0x7FF);
  const uint64_t frac = b & ((uint64_t(1) << 52) - 1);
  if (e == 0x7FF) return uint16_t(sign | (frac ? 0x7E00u : 0x7C00u));  // NaN, infinity
  if (e == 0) return sign;  // zero or binary64 subnormal: far below 2^-25, rounds to 0
  const int E = e - 1023;   // value = sig * 2^(E - 52), sig in [2^52, 2^53)
  if (E > 15) {
    *overflow = true;
    return uint16_t(sign | 0x7C00u);
  }
  const uint64_t sig = frac | (uint64_t(1) << 52);
  // q = value / 2^s rounded, with s = E - 10 for normals and -24 below 2^-14
  const int s = E >= -14 ? E - 10 : -24;
  const int shift = 52 + s - E;  // 42 for normals, more for subnormals
  if (shift > 60) return sign;    // value < 2^-32: rounds to 0
  uint64_t q = sig >> shift;
  const uint64_t rem = sig & ((uint64_t(1) << shift) - 1);
  const uint64_t half = uint64_t(1) << (shift - 1);
  if (rem > half || (rem == half && (q & 1))) ++q;
  uint32_t bits;
  if (E >= -14) {
    // q in [2^10, 2^11]; q == 2^11 carries into the exponent
    bits = (uint32_t(E + 14) << 10) + uint32_t(q);
  } else {
    bits = uint32_t(q);  // subnormal; q == 2^10 is the smallest normal
  }
  if (bits >= 0x7C00u) {
    *overflow = true;
    bits = 0x7C00u;
  }
  return uint16_t(sign | bits);
}

// IEEE 754 binary32 -> binary16 bits, same rounding (the binary32 value is
// exactly representable in binary64, so one rounding step results).
uint16_t f32_to_f16_bits(float f, bool* overflow) { return f64_to_f16_bits(double(f), overflow); }

}  // namespace damn

using namespace damn;

extern "C" {

int damn_encode_index(int32_t format, int32_t nrows, int32_t ncols, const int32_t* rowptr,
                      const int32_t* colids, void* idx_out, int32_t* w_out) {
  const int ib = index_bytes(format);
  if (ib == 0 || format_is_block(format) || format_is_coo(format) || w_out == nullptr)
    return DAMN_ERR_INVALID_ARG;
  const int st = check_csr(nrows, ncols, rowptr, colids);
  if (st != DAMN_OK) return st;
  const int64_t nnz = rowptr[nrows];
  if (nnz > 0 && idx_out == nullptr) return DAMN_ERR_INVALID_ARG;
  const int64_t limit = int64_t(1) << (8 * ib - 1);
  int64_t w = 0;
  if (format_is_da(format)) {
    int64_t lo = 0, hi = 0;
    bandwidth(nrows, rowptr, colids, &lo, &hi);
    w = std::max(lo, hi);
  } else {
    for (int64_t i = 0; i < nnz; ++i) w = std::max<int64_t>(w, colids[i]);
  }
  *w_out = int32_t(w);
  if (w >= limit) return DAMN_ERR_NO_FIT;
  const bool da = format_is_da(format);
  parallel_for(nrows, [&](int64_t b, int64_t e) {
    for (int64_t r = b; r < e; ++r)
      for (int64_t i = rowptr[r]; i < rowptr[r + 1]; ++i) {
        const int64_t v = da ? int64_t(colids[i]) - r : int64_t(colids[i]);
        if (ib == 1)
          static_cast<int8_t*>(idx_out)[i] = int8_t(v);
        else if (ib == 2)
          static_cast<int16_t*>(idx_out)[i] = int16_t(v);
        else
          static_cast<int32_t*>(idx_out)[i] = int32_t(v);
      }
  }, 4096);
  return DAMN_OK;
}

int damn_coo_encode(int32_t format, int32_t nrows, int32_t ncols, const int32_t* rowptr,
                    const int32_t* colids, int32_t* rows_out, void* idx_out, int32_t* w_out) {
  if (!format_is_coo(format) || w_out == nullptr) return DAMN_ERR_INVALID_ARG;
  const int st = check_csr(nrows, ncols, rowptr, colids);
  if (st != DAMN_OK) return st;
  const int64_t nnz = rowptr[nrows];
  if (nnz > 0 && (rows_out == nullptr || idx_out == nullptr)) return DAMN_ERR_INVALID_ARG;
  const bool da = format == DAMN_FORMAT_DACOO16;
  int64_t w = 0;
  if (da) {
    int64_t lo = 0, hi = 0;
    bandwidth(nrows, rowptr, colids, &lo, &hi);
    w = std::max(lo, hi);
    *w_out = int32_t(w);
    if (w >= kInt16BandwidthLimit) return DAMN_ERR_NO_FIT;
  } else {
    for (int64_t i = 0; i < nnz; ++i) w = std::max<int64_t>(w, colids[i]);
    *w_out = int32_t(w);
  }
  parallel_for(nrows, [&](int64_t b, int64_t e) {
    for (int64_t r = b; r < e; ++r)
      for (int64_t i = rowptr[r]; i < rowptr[r + 1]; ++i) {
        rows_out[i] = int32_t(r);
        if (da)
          static_cast<int16_t*>(idx_out)[i] = int16_t(colids[i] - r);
        else
          static_cast<int32_t*>(idx_out)[i] = colids[i];
      }
  }, 4096);
  return DAMN_OK;
}

int damn_store_values(int64_t n, const void* vals, int32_t vals_dtype, int32_t dtype,
                      void* out) {
  if (n < 0 || (n > 0 && (vals == nullptr || out == nullptr))) return DAMN_ERR_INVALID_ARG;
  if (value_bytes(vals_dtype) == 0 || value_bytes(dtype) == 0) return DAMN_ERR_INVALID_ARG;
  if (value_bytes(dtype) > value_bytes(vals_dtype)) return DAMN_ERR_UNSUPPORTED;
  int32_t over = 0;
  parallel_for(n, [&](int64_t b, int64_t e) {
    bool o = false;
    for (int64_t i = b; i < e; ++i) {
      if (vals_dtype == dtype) {
        std::memcpy(static_cast<char*>(out) + i * value_bytes(dtype),
                    static_cast<const char*>(vals) + i * value_bytes(dtype), value_bytes(dtype));
      } else if (dtype == DAMN_F32) {  // from float64; the host rounds to nearest even
        const double v = static_cast<const double*>(vals)[i];
        const float f = float(v);
        o |= std::isinf(f) && std::isfinite(v);
        static_cast<float*>(out)[i] = f;
      } else if (vals_dtype == DAMN_F64) {  // float64 -> float16
        static_cast<uint16_t*>(out)[i] = f64_to_f16_bits(static_cast<const double*>(vals)[i], &o);
      } else {  // float32 -> float16
        static_cast<uint16_t*>(out)[i] = f32_to_f16_bits(static_cast<const float*>(vals)[i], &o);
      }
    }
    if (o) __atomic_store_n(&over, 1, __ATOMIC_RELAXED);
  });
  return over ? DAMN_ERR_NO_FIT : DAMN_OK;
}

}  // extern "C"
