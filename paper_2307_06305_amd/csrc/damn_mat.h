// The device matrix handle, shared by the library's HIP translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "damn.h"
#include "damn_kernels.h"

struct damn_cg_work;  // conjugate-gradient workspace, allocated on first use

struct damn_mat_s {
  int device = 0;
  int32_t nrows = 0, ncols = 0;
  int64_t nnz = 0;
  int32_t format = DAMN_FORMAT_DA16;
  int32_t dtype = DAMN_F64;
  int32_t block = 1;  // b of block formats (rowptr, idx and tiles count block rows)
  int32_t* d_rows = nullptr;  // coordinate formats: row of each entry, padded
  int32_t* d_cross = nullptr;  // coordinate formats: per chunk, the end of the row of its last entry
  int64_t nchunks = 0;
  int32_t* d_rowptr = nullptr;
  void* d_idx = nullptr;  // int16 offsets or int32 columns, padded
  void* d_val = nullptr;  // float64 or float32 values, padded
  std::vector<int32_t> h_rowptr;  // host copy, for building stream tiles
  damn_config cfg{};
  damn::TileStart* d_tiles = nullptr;  // stream tiles, then the end record
  int64_t ntiles = 0;
  int32_t tiles_req = 0;  // entry cap the tiles were built for
  int32_t tiles_cap = 0;  // largest entry count of a tile that is not one long row
  int32_t tiles_rows = 0;  // most rows of any tile
  damn_cg_work* cg = nullptr;
};

namespace damn {
// x values per gather load of a stream configuration: its `unroll` (1
// interleaved, 2 paired); 1 for the vector variant.
inline int32_t gather_of(const damn_config& c) {
  return c.variant == DAMN_VAR_STREAM && c.unroll == 2 ? 2 : 1;
}
// Build (or reuse) the stream tiles of A for entry cap `cap`; synchronises.
int build_tiles(damn_mat A, int32_t cap, hipStream_t s);
// Free the conjugate-gradient workspace of A, if any.
void release_cg_work(damn_mat A);
}  // namespace damn
