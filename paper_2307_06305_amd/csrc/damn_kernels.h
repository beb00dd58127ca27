// Launch interface between the C ABI layer and the product kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "damn.h"

namespace damn {

// Rows per stream tile are capped so one workgroup's second step stays short
// and the tile's row pointers fit a fixed LDS area.
constexpr int32_t kMaxTileRows = 512;
// Start of a stream tile: its first row and that row's first entry (for
// block formats: block row and block), so a workgroup knows its rows and
// entry range after one load.  Tiles are listed in order, followed by the
// end record (nrows, nnz).
struct alignas(8) TileStart {
  int32_t row;
  int32_t entry;
};

// Row-pointer arrays are allocated with this many spare (zero) entries so
// 16-byte copies of a tile's row pointers stay inside the allocation.
constexpr int32_t kRowptrPad = 16;

// Coordinate formats: entries per workgroup.
constexpr int32_t kCooChunk = 1024;

struct SpmvArgs {
  int32_t nrows = 0;
  int32_t ncols = 0;
  const int32_t* rowptr = nullptr;
  const void* idx = nullptr;  // indices of `format` (damn_format)
  const void* val = nullptr;  // values of `store` (damn_dtype)
  const void* x = nullptr;
  void* y = nullptr;
  double alpha = 1.0;
  double beta = 0.0;
  int32_t read_y = 0;  // beta != 0
  int32_t format = DAMN_FORMAT_DA16;
  int32_t store = DAMN_F64;  // x, y and sums are float64 for DAMN_F64, else float32
  int32_t block = 1;         // block formats: b (rowptr and tiles count block rows)
  // coordinate formats: entries, their rows, per chunk the end of the row
  // holding its last entry
  int64_t nnz = 0;
  const int32_t* coo_rows = nullptr;
  const int32_t* coo_cross = nullptr;
  int64_t nchunks = 0;
  // stream variant
  int32_t cache = DAMN_CACHE_NT;  // cache policy of the matrix stream (damn_cache)
  int32_t gather = 1;             // x values per gather load: 1 interleaved, 2 paired
  const TileStart* tile_row = nullptr;
  int64_t ntiles = 0;
  int32_t cap = 0;
  int32_t tile_rows = kMaxTileRows;  // most rows (block rows) of any tile
  hipStream_t stream = nullptr;
};

// variant 0 = vector (lanes, unroll), 1 = stream (lanes = G, tiles in args)
hipError_t launch_spmv(const SpmvArgs& a, int variant, int lanes, int unroll);
// The same for 8-bit DA, 16-bit CSR and float16 values (spmv_grid.hip).
hipError_t launch_spmv_grid(const SpmvArgs& a, int variant, int lanes, int unroll);
// Block formats (spmv_bsr.hip): the stream variant over tiles of block rows
// with `cap` blocks; lanes in {1, 2, 4, 8, 16}; block in {2, 3, 4, 6}.
hipError_t launch_spmv_bsr(const SpmvArgs& a, int lanes);
// Coordinate formats (spmv_coo.hip): one chunk kernel (y <- beta*y alone
// when alpha == 0 or there are no entries); entries in row order.
hipError_t launch_spmv_coo(const SpmvArgs& a);
// Stream variant with the conjugate-gradient epilogue: partial[t] = sum of
// y_r * w_r over tile t (w = nullptr: w = y), skipped entirely when *done.
// lanes in {1, 2, 4, 8, 16}; alpha != 0; DA16 or CSR32, float64 or float32.
hipError_t launch_spmv_dot(const SpmvArgs& a, int lanes, const void* w, double* partial,
                           const int32_t* done);
// float64 DA16 or CSR32 only; 1 <= nrhs <= 8; vector variant
hipError_t launch_spmm(const SpmvArgs& a, int lanes, int nrhs);
// The same with the stream variant's tiles (spmm_stream.hip)
hipError_t launch_spmm_stream(const SpmvArgs& a, int lanes, int nrhs);
hipError_t launch_stream_read(const void* src, int64_t bytes, int32_t passes, double* sink,
                              int mode, int32_t tile_bytes, hipStream_t s);
hipError_t launch_stream_copy(const void* src, void* dst, int64_t bytes, hipStream_t s);
hipError_t launch_gather_read(const double* x, int64_t n, int64_t rows, int32_t per_row,
                              int32_t hw, const int32_t* offs, double* sink, hipStream_t s);

}  // namespace damn
