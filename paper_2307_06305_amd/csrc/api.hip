// C ABI of libdamn.so: device matrices, products and configuration.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "damn.h"
#include "damn_internal.h"
#include "damn_kernels.h"
#include "damn_mat.h"

namespace damn {

// Cut rows into tiles of consecutive rows with at most `cap` entries and at
// most kMaxTileRows rows; a longer row is a tile of its own.  A tile that
// does not reach the last row is cut back to a power-of-two number of rows:
// on grids whose lines have power-of-two length the tiles then cover whole
// lines or equal parts of them, and every row slot of the workgroup's row
// loop is used (7-point 128 x 128 x 1024 stencil, one lane per row: 274 us
// with 256-row tiles against 294 us with the greedy 292-row tiles, whose
// second pass over the rows leaves most lanes idle).
//
// The kernels size LDS by A->tiles_cap and A->tiles_rows, the most entries
// and rows of a regular tile, so small tiles leave room for more resident
// workgroups; they also take a tile with more than tiles_cap entries for one
// long row (every long row exceeds `cap`, hence tiles_cap).
//
// Tiles are built when a handle is created and when damn_set_config picks a
// new cap, never inside a product call: the table is uploaded on `s` and
// waited for, and a table it replaces is freed only after the device has
// drained every launch queued so far (any of them may still read it).
int build_tiles(damn_mat A, int32_t cap, hipStream_t s) {
  if (A->d_tiles && A->tiles_req == cap) return DAMN_OK;
  std::vector<TileStart> starts;
  int32_t largest = 0, most_rows = 1;
  try {
    // rows of the stored structure: block rows for block formats
    const int32_t nr = int32_t(A->h_rowptr.size()) - 1;
    starts.reserve(size_t(nr / 8 + 2));
    const int32_t* rp = A->h_rowptr.data();
    int32_t r = 0;
    while (r < nr) {
      starts.push_back({r, rp[r]});
      const int32_t first = r;
      if (rp[r + 1] - rp[r] > cap) {
        ++r;
        continue;
      }
      while (r < nr && r - first < kMaxTileRows && rp[r + 1] - rp[first] <= cap) ++r;
      if (r < nr) {
        int32_t m = 1;
        while (2 * m <= r - first) m *= 2;
        r = first + m;
      }
      largest = std::max(largest, rp[r] - rp[first]);
      most_rows = std::max(most_rows, r - first);
    }
    starts.push_back({nr, rp[nr]});
  } catch (const std::bad_alloc&) {
    return DAMN_ERR_ALLOC;
  }
  TileStart* d = nullptr;
  if (hipMalloc(&d, sizeof(TileStart) * starts.size()) != hipSuccess) return DAMN_ERR_ALLOC;
  if (hipMemcpyAsync(d, starts.data(), sizeof(TileStart) * starts.size(), hipMemcpyHostToDevice,
                     s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess) {
    hipFree(d);
    return DAMN_ERR_HIP;
  }
  if (A->d_tiles) {
    if (hipDeviceSynchronize() != hipSuccess) {
      hipFree(d);
      return DAMN_ERR_HIP;
    }
    hipFree(A->d_tiles);
  }
  A->d_tiles = d;
  A->ntiles = int64_t(starts.size()) - 1;
  A->tiles_req = cap;
  A->tiles_cap = largest;
  A->tiles_rows = most_rows;
  return DAMN_OK;
}

int host_threads() {
  static int n = [] {
    int t = int(std::thread::hardware_concurrency());
    if (const char* e = std::getenv("DAMN_THREADS")) t = std::atoi(e);
    if (t < 1) t = 1;
    if (t > 64) t = 64;
    return t;
  }();
  return n;
}

namespace {

// Entry arrays are padded (and zero-filled) so the stream variant's 16-byte
// pieces, which may run up to 15 entries past the last one, stay inside.
inline int64_t padded_entries(int64_t nnz) { return ((nnz + 15) / 16) * 16 + 32; }

// Default launch shape: the stream variant with 2048-entry tiles; one lane
// per row for very short rows, two otherwise, and more lanes for long rows
// (about one lane per 16 entries).
damn_config default_config(int32_t nrows, int64_t nnz) {
  damn_config c{};
  c.variant = DAMN_VAR_STREAM;
  c.unroll = 1;
  c.tile = 2048;
  const double mean = nrows > 0 ? double(nnz) / nrows : 0.0;
  int lanes = mean < 4.0 ? 1 : 2;
  while (lanes < 64 && lanes * 16 < mean) lanes *= 2;
  c.lanes = lanes;
  return c;
}

bool valid_pow2_lanes(int32_t l) { return l >= 1 && l <= 64 && (l & (l - 1)) == 0; }

// Tile cap of the stream variant for a configured tile size: entries, or
// for block formats blocks of about `tile` values (at least 8).
int32_t tile_cap(damn_mat A, int32_t tile) {
  if (A->block <= 1) return tile;
  const int32_t c = tile / (A->block * A->block);
  return c < 8 ? 8 : c;
}

void free_mat(damn_mat A) {
  if (!A) return;
  int cur = 0;
  hipGetDevice(&cur);
  hipSetDevice(A->device);
  if (A->d_rowptr) hipFree(A->d_rowptr);
  if (A->d_idx) hipFree(A->d_idx);
  if (A->d_val) hipFree(A->d_val);
  if (A->d_tiles) hipFree(A->d_tiles);
  if (A->d_rows) hipFree(A->d_rows);
  if (A->d_cross) hipFree(A->d_cross);
  release_cg_work(A);
  hipSetDevice(cur);
  delete A;
}

// Last step of every create call for the tiled formats: the stream tiles of
// the default configuration, so no product call has to build them.
int create_tiles(damn_mat A, hipStream_t s) {
  const int st = build_tiles(A, tile_cap(A, A->cfg.tile), s);
  if (st != DAMN_OK) {
    free_mat(A);
    return st;
  }
  return DAMN_OK;
}

// Upload a validated matrix: indices of `format` as given, values rounded
// from vals_dtype to store_dtype (damn_store_values).
int create_common(damn_mat* out, int32_t nrows, int32_t ncols, const int32_t* rowptr,
                  const void* idx, const void* vals, int32_t vals_dtype, int32_t store_dtype,
                  void* stream, int32_t format, int64_t vals_per_entry = 1) {
  if (out == nullptr || rowptr == nullptr) return DAMN_ERR_INVALID_ARG;
  if (value_bytes(vals_dtype) == 0 || value_bytes(store_dtype) == 0) return DAMN_ERR_INVALID_ARG;
  if (value_bytes(store_dtype) > value_bytes(vals_dtype)) return DAMN_ERR_UNSUPPORTED;
  const size_t idx_size = size_t(index_bytes(format));
  const int64_t nnz = rowptr[nrows];
  if (nnz > 0 && (idx == nullptr || vals == nullptr)) return DAMN_ERR_INVALID_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);

  damn_mat A = nullptr;
  try {
    A = new damn_mat_s();
    A->h_rowptr.assign(rowptr, rowptr + nrows + 1);
  } catch (const std::bad_alloc&) {
    delete A;
    return DAMN_ERR_ALLOC;
  }
  hipGetDevice(&A->device);
  A->nrows = nrows;
  A->ncols = ncols;
  A->nnz = nnz;
  A->format = format;
  A->dtype = store_dtype;
  A->cfg = default_config(nrows, nnz);

  const size_t vsize = size_t(value_bytes(store_dtype));
  const int64_t pe = padded_entries(nnz);
  const int64_t nv = nnz * vals_per_entry;  // values: b*b per block for block formats
  const int64_t pv = padded_entries(nv);
  if (hipMalloc(&A->d_rowptr, sizeof(int32_t) * (size_t(nrows) + 1 + kRowptrPad)) != hipSuccess ||
      hipMalloc(&A->d_idx, idx_size * pe) != hipSuccess ||
      hipMalloc(&A->d_val, vsize * pv) != hipSuccess) {
    free_mat(A);
    return DAMN_ERR_ALLOC;
  }
  std::vector<unsigned char> conv;
  const void* src_vals = vals;
  if (store_dtype != vals_dtype) {
    try {
      conv.resize(size_t(nv) * vsize);
    } catch (const std::bad_alloc&) {
      free_mat(A);
      return DAMN_ERR_ALLOC;
    }
    const int st = damn_store_values(nv, vals, vals_dtype, store_dtype, conv.data());
    if (st != DAMN_OK) {
      free_mat(A);
      return st;
    }
    src_vals = conv.data();
  }
  bool ok = hipMemsetAsync(A->d_rowptr, 0, sizeof(int32_t) * (size_t(nrows) + 1 + kRowptrPad),
                           s) == hipSuccess &&
            hipMemsetAsync(A->d_idx, 0, idx_size * pe, s) == hipSuccess &&
            hipMemsetAsync(A->d_val, 0, vsize * pv, s) == hipSuccess &&
            hipMemcpyAsync(A->d_rowptr, rowptr, sizeof(int32_t) * (size_t(nrows) + 1),
                           hipMemcpyHostToDevice, s) == hipSuccess;
  if (ok && nnz > 0)
    ok = hipMemcpyAsync(A->d_idx, idx, idx_size * nnz, hipMemcpyHostToDevice, s) == hipSuccess &&
         hipMemcpyAsync(A->d_val, src_vals, vsize * nv, hipMemcpyHostToDevice, s) ==
             hipSuccess;
  if (ok) ok = hipStreamSynchronize(s) == hipSuccess;
  if (!ok) {
    free_mat(A);
    return DAMN_ERR_HIP;
  }
  *out = A;
  return DAMN_OK;
}

// create_common, then the stream tiles of the default configuration
int create_tiled(damn_mat* out, int32_t nrows, int32_t ncols, const int32_t* rowptr,
                 const void* idx, const void* vals, int32_t vals_dtype, int32_t store_dtype,
                 void* stream, int32_t format) {
  damn_mat A = nullptr;
  int st = create_common(&A, nrows, ncols, rowptr, idx, vals, vals_dtype, store_dtype, stream,
                         format);
  if (st != DAMN_OK) return st;
  st = create_tiles(A, static_cast<hipStream_t>(stream));
  if (st != DAMN_OK) return st;
  *out = A;
  return DAMN_OK;
}

int run_spmv(damn_mat A, const void* x, void* y, double alpha, double beta, void* stream,
             bool want_da) {
  if (A == nullptr || format_is_da(A->format) != want_da) return DAMN_ERR_INVALID_ARG;
  if ((x == nullptr && A->ncols > 0 && alpha != 0.0) || (y == nullptr && A->nrows > 0))
    return DAMN_ERR_INVALID_ARG;
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
  a.stream = static_cast<hipStream_t>(stream);
  if (format_is_coo(A->format)) {
    a.nnz = A->nnz;
    a.coo_rows = A->d_rows;
    a.coo_cross = A->d_cross;
    a.nchunks = A->nchunks;
    const hipError_t e = launch_spmv_coo(a);
    return e == hipSuccess ? DAMN_OK : DAMN_ERR_HIP;
  }
  if (A->block > 1) {
    // block formats: the stream variant only, at most 16 lanes per row
    if (alpha == 0.0) {  // y <- beta*y: no tiles needed
      const hipError_t e = launch_spmv(a, DAMN_VAR_VECTOR, 1, 1);
      return e == hipSuccess ? DAMN_OK : DAMN_ERR_HIP;
    }
    if (A->d_tiles == nullptr) return DAMN_ERR_INVALID_ARG;
    a.block = A->block;
    a.tile_row = A->d_tiles;
    a.ntiles = A->ntiles;
    a.cap = A->tiles_cap;
    a.tile_rows = A->tiles_rows;
    const hipError_t e = launch_spmv_bsr(a, A->cfg.lanes > 16 ? 16 : A->cfg.lanes);
    return e == hipSuccess ? DAMN_OK : DAMN_ERR_HIP;
  }
  if (A->cfg.variant == DAMN_VAR_STREAM) {
    if (A->d_tiles == nullptr) return DAMN_ERR_INVALID_ARG;
    a.tile_row = A->d_tiles;
    a.ntiles = A->ntiles;
    a.cap = A->tiles_cap;
    a.tile_rows = A->tiles_rows;
    a.cache = A->cfg.cache;
    a.gather = gather_of(A->cfg);
  }
  const hipError_t e = launch_spmv(a, A->cfg.variant, A->cfg.lanes, A->cfg.unroll);
  return e == hipSuccess ? DAMN_OK : DAMN_ERR_HIP;
}

}  // namespace
}  // namespace damn

using namespace damn;

extern "C" {

const char* damn_status_string(int status) {
  switch (status) {
    case DAMN_OK: return "ok";
    case DAMN_ERR_INVALID_ARG: return "invalid argument";
    case DAMN_ERR_BAD_CSR: return "malformed CSR structure";
    case DAMN_ERR_NO_FIT:
      return "index or value does not fit its storage type (16-bit offsets need bandwidth "
             "< 2^15)";
    case DAMN_ERR_HIP: return "HIP runtime error";
    case DAMN_ERR_ALLOC: return "allocation failed";
    case DAMN_ERR_UNSUPPORTED: return "unsupported combination";
    case DAMN_ERR_NOT_CONVERGED: return "iteration limit reached";
    case DAMN_ERR_BREAKDOWN: return "breakdown: matrix not positive definite";
    case DAMN_ERR_TOO_LARGE: return "more rows than the fixed scratch area holds";
    default: return "unknown status";
  }
}

const char* damn_version(void) { return "damn 0.1.0 (gfx950)"; }

int damn_create(damn_mat* out, int32_t nrows, int32_t ncols, const int32_t* rowptr,
                const int16_t* off, const void* vals, int32_t vals_dtype, int32_t store_dtype,
                void* stream) {
  if (nrows < 0 || ncols < 0 || rowptr == nullptr) return DAMN_ERR_INVALID_ARG;
  // structure, plus every r + off[i] inside [0, ncols)
  if (rowptr[0] != 0) return DAMN_ERR_BAD_CSR;
  for (int32_t r = 0; r < nrows; ++r)
    if (rowptr[r + 1] < rowptr[r]) return DAMN_ERR_BAD_CSR;
  const int64_t nnz = rowptr[nrows];
  if (nnz > 0 && off == nullptr) return DAMN_ERR_INVALID_ARG;
  int32_t bad = 0;
  parallel_for(nrows, [&](int64_t b, int64_t e) {
    int32_t local = 0;
    for (int64_t r = b; r < e; ++r)
      for (int64_t i = rowptr[r]; i < rowptr[r + 1]; ++i) {
        const int64_t c = r + off[i];
        local |= (c < 0) | (c >= ncols);
      }
    if (local) __atomic_store_n(&bad, 1, __ATOMIC_RELAXED);
  }, 4096);
  if (bad) return DAMN_ERR_BAD_CSR;
  return create_tiled(out, nrows, ncols, rowptr, off, vals, vals_dtype, store_dtype, stream,
                      DAMN_FORMAT_DA16);
}

int damn_csr_create(damn_mat* out, int32_t nrows, int32_t ncols, const int32_t* rowptr,
                    const int32_t* colids, const void* vals, int32_t vals_dtype,
                    int32_t store_dtype, void* stream) {
  const int st = check_csr(nrows, ncols, rowptr, colids);
  if (st != DAMN_OK) return st;
  return create_tiled(out, nrows, ncols, rowptr, colids, vals, vals_dtype, store_dtype, stream,
                      DAMN_FORMAT_CSR32);
}

int damn_bsr_create(damn_mat* out, int32_t format, int32_t nbrows, int32_t nbcols, int32_t b,
                    const int32_t* browptr, const void* bidx, const void* bvals,
                    int32_t vals_dtype, int32_t store_dtype, void* stream) {
  if (!format_is_block(format) || nbrows < 0 || nbcols < 0 || browptr == nullptr ||
      out == nullptr)
    return DAMN_ERR_INVALID_ARG;
  if (b != 2 && b != 3 && b != 4 && b != 6) return DAMN_ERR_UNSUPPORTED;
  if (store_dtype == DAMN_F16) return DAMN_ERR_UNSUPPORTED;
  if (int64_t(nbrows) * b > INT32_MAX || int64_t(nbcols) * b > INT32_MAX)
    return DAMN_ERR_UNSUPPORTED;
  if (browptr[0] != 0) return DAMN_ERR_BAD_CSR;
  for (int32_t r = 0; r < nbrows; ++r)
    if (browptr[r + 1] < browptr[r]) return DAMN_ERR_BAD_CSR;
  const int64_t nnzb = browptr[nbrows];
  if (nnzb > 0 && (bidx == nullptr || bvals == nullptr)) return DAMN_ERR_INVALID_ARG;
  if (nnzb * b * b >= (int64_t(1) << 31)) return DAMN_ERR_UNSUPPORTED;
  const bool da = format == DAMN_FORMAT_DABSR16;
  int32_t bad = 0;
  parallel_for(nbrows, [&](int64_t lo, int64_t hi) {
    int32_t local = 0;
    for (int64_t r = lo; r < hi; ++r)
      for (int64_t k = browptr[r]; k < browptr[r + 1]; ++k) {
        const int64_t c = da ? r + static_cast<const int16_t*>(bidx)[k]
                             : int64_t(static_cast<const int32_t*>(bidx)[k]);
        local |= (c < 0) | (c >= nbcols);
      }
    if (local) __atomic_store_n(&bad, 1, __ATOMIC_RELAXED);
  }, 4096);
  if (bad) return DAMN_ERR_BAD_CSR;
  // the values are nnzb*b*b scalars: upload as a matrix with that many
  // entries, then describe the blocks
  std::vector<int32_t> vrp;
  try {
    vrp.assign(browptr, browptr + nbrows + 1);
  } catch (const std::bad_alloc&) {
    return DAMN_ERR_ALLOC;
  }
  damn_mat A = nullptr;
  int st = create_common(&A, nbrows, nbcols, vrp.data(), bidx, bvals, vals_dtype, store_dtype,
                         stream, format, int64_t(b) * b);
  if (st != DAMN_OK) return st;
  A->block = b;
  A->nrows = nbrows * b;
  A->ncols = nbcols * b;
  st = create_tiles(A, static_cast<hipStream_t>(stream));
  if (st != DAMN_OK) return st;
  *out = A;
  return DAMN_OK;
}

int damn_coo_create(damn_mat* out, int32_t format, int32_t nrows, int32_t ncols, int64_t nnz,
                    const int32_t* rows, const void* idx, const void* vals, int32_t vals_dtype,
                    int32_t store_dtype, void* stream) {
  if (!format_is_coo(format) || out == nullptr || nrows < 0 || ncols < 0 || nnz < 0)
    return DAMN_ERR_INVALID_ARG;
  if (store_dtype == DAMN_F16 || nnz >= (int64_t(1) << 31)) return DAMN_ERR_UNSUPPORTED;
  if (nnz > 0 && (rows == nullptr || idx == nullptr || vals == nullptr))
    return DAMN_ERR_INVALID_ARG;
  // rows in order and range, columns in range; the row pointers follow
  std::vector<int32_t> rp;
  try {
    rp.assign(size_t(nrows) + 1, 0);
  } catch (const std::bad_alloc&) {
    return DAMN_ERR_ALLOC;
  }
  const bool da = format == DAMN_FORMAT_DACOO16;
  for (int64_t i = 0; i < nnz; ++i) {
    const int32_t r = rows[i];
    if (r < 0 || r >= nrows || (i > 0 && r < rows[i - 1])) return DAMN_ERR_BAD_CSR;
    const int64_t c = da ? int64_t(r) + static_cast<const int16_t*>(idx)[i]
                         : int64_t(static_cast<const int32_t*>(idx)[i]);
    if (c < 0 || c >= ncols) return DAMN_ERR_BAD_CSR;
    ++rp[size_t(r) + 1];
  }
  for (int32_t r = 0; r < nrows; ++r) rp[r + 1] += rp[r];
  damn_mat A = nullptr;
  int st = create_common(&A, nrows, ncols, rp.data(), idx, vals, vals_dtype, store_dtype, stream,
                         format);
  if (st != DAMN_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  A->nchunks = (nnz + kCooChunk - 1) / kCooChunk;
  // per chunk, the end of the row holding its last entry: the chunk where a
  // row begins sums it to there
  std::vector<int32_t> cross;
  try {
    cross.resize(size_t(A->nchunks > 0 ? A->nchunks : 1), 0);
  } catch (const std::bad_alloc&) {
    free_mat(A);
    return DAMN_ERR_ALLOC;
  }
  for (int64_t t = 0; t < A->nchunks; ++t) {
    const int64_t last = std::min<int64_t>((t + 1) * kCooChunk, nnz) - 1;
    cross[size_t(t)] = rp[size_t(rows[last]) + 1];
  }
  const int64_t pe = padded_entries(nnz);
  bool ok = hipMalloc(&A->d_rows, sizeof(int32_t) * pe) == hipSuccess &&
            hipMalloc(&A->d_cross, sizeof(int32_t) * cross.size()) == hipSuccess;
  if (!ok) {
    free_mat(A);
    return DAMN_ERR_ALLOC;
  }
  ok = hipMemsetAsync(A->d_rows, 0, sizeof(int32_t) * pe, s) == hipSuccess &&
       (nnz == 0 || hipMemcpyAsync(A->d_rows, rows, sizeof(int32_t) * nnz,
                                   hipMemcpyHostToDevice, s) == hipSuccess) &&
       hipMemcpyAsync(A->d_cross, cross.data(), sizeof(int32_t) * cross.size(),
                      hipMemcpyHostToDevice, s) == hipSuccess &&
       hipStreamSynchronize(s) == hipSuccess;
  if (!ok) {
    free_mat(A);
    return DAMN_ERR_HIP;
  }
  *out = A;
  return DAMN_OK;
}

int damn_create_format(damn_mat* out, int32_t format, int32_t nrows, int32_t ncols,
                       const int32_t* rowptr, const void* idx, const void* vals,
                       int32_t vals_dtype, int32_t store_dtype, void* stream) {
  const int ib = index_bytes(format);
  if (ib == 0 || format_is_block(format) || format_is_coo(format) || nrows < 0 || ncols < 0 ||
      rowptr == nullptr)
    return DAMN_ERR_INVALID_ARG;
  if (rowptr[0] != 0) return DAMN_ERR_BAD_CSR;
  for (int32_t r = 0; r < nrows; ++r)
    if (rowptr[r + 1] < rowptr[r]) return DAMN_ERR_BAD_CSR;
  const int64_t nnz = rowptr[nrows];
  if (nnz > 0 && (idx == nullptr || vals == nullptr)) return DAMN_ERR_INVALID_ARG;
  // every column (r + off for DA) inside [0, ncols), so no kernel reads outside x
  const bool da = format_is_da(format);
  int32_t bad = 0;
  parallel_for(nrows, [&](int64_t b, int64_t e) {
    int32_t local = 0;
    for (int64_t r = b; r < e; ++r)
      for (int64_t i = rowptr[r]; i < rowptr[r + 1]; ++i) {
        const int64_t v = ib == 1   ? int64_t(static_cast<const int8_t*>(idx)[i])
                          : ib == 2 ? int64_t(static_cast<const int16_t*>(idx)[i])
                                    : int64_t(static_cast<const int32_t*>(idx)[i]);
        const int64_t c = da ? r + v : v;
        local |= (c < 0) | (c >= ncols);
      }
    if (local) __atomic_store_n(&bad, 1, __ATOMIC_RELAXED);
  }, 4096);
  if (bad) return DAMN_ERR_BAD_CSR;
  return create_tiled(out, nrows, ncols, rowptr, idx, vals, vals_dtype, store_dtype, stream,
                      format);
}

int damn_destroy(damn_mat A) {
  if (A == nullptr) return DAMN_ERR_INVALID_ARG;
  int cur = 0;
  hipGetDevice(&cur);
  hipSetDevice(A->device);
  hipDeviceSynchronize();
  hipSetDevice(cur);
  free_mat(A);
  return DAMN_OK;
}

int damn_mat_info(damn_mat A, int32_t* nrows, int32_t* ncols, int64_t* nnz, int32_t* format,
                  int32_t* dtype) {
  if (A == nullptr) return DAMN_ERR_INVALID_ARG;
  if (nrows) *nrows = A->nrows;
  if (ncols) *ncols = A->ncols;
  if (nnz) *nnz = A->nnz;
  if (format) *format = A->format;
  if (dtype) *dtype = A->dtype;
  return DAMN_OK;
}

int damn_spmv(damn_mat A, const void* x, void* y, double alpha, double beta, void* stream) {
  return run_spmv(A, x, y, alpha, beta, stream, true);
}

int damn_csr_spmv(damn_mat A, const void* x, void* y, double alpha, double beta,
                  void* stream) {
  return run_spmv(A, x, y, alpha, beta, stream, false);
}

int damn_spmm(damn_mat A, const void* X, void* Y, int32_t nrhs, double alpha, double beta,
              void* stream) {
  if (A == nullptr || nrhs < 1) return DAMN_ERR_INVALID_ARG;
  if (nrhs > 8) return DAMN_ERR_UNSUPPORTED;
  if (A->dtype != DAMN_F64 || (A->format != DAMN_FORMAT_DA16 && A->format != DAMN_FORMAT_CSR32))
    return DAMN_ERR_UNSUPPORTED;
  if ((X == nullptr && A->ncols > 0 && alpha != 0.0) || (Y == nullptr && A->nrows > 0))
    return DAMN_ERR_INVALID_ARG;
  SpmvArgs a;
  a.nrows = A->nrows;
  a.ncols = A->ncols;
  a.rowptr = A->d_rowptr;
  a.idx = A->d_idx;
  a.val = A->d_val;
  a.x = X;
  a.y = Y;
  a.alpha = alpha;
  a.beta = beta;
  a.read_y = beta != 0.0;
  a.format = A->format;
  a.store = A->dtype;
  a.stream = static_cast<hipStream_t>(stream);
  if (alpha == 0.0) {  // Y <- beta*Y over nrows*nrhs values; A and X are not read
    if (int64_t(A->nrows) * nrhs > INT32_MAX) return DAMN_ERR_UNSUPPORTED;
    a.nrows = int32_t(int64_t(A->nrows) * nrhs);
    const hipError_t e = launch_spmv(a, DAMN_VAR_VECTOR, 1, 1);
    return e == hipSuccess ? DAMN_OK : DAMN_ERR_HIP;
  }
  if (A->cfg.variant == DAMN_VAR_STREAM) {
    // one right-hand side: the SpMV kernels (X and Y are vectors)
    if (nrhs == 1) return run_spmv(A, X, Y, alpha, beta, stream, format_is_da(A->format));
    if (A->d_tiles == nullptr) return DAMN_ERR_INVALID_ARG;
    a.tile_row = A->d_tiles;
    a.ntiles = A->ntiles;
    a.cap = A->tiles_cap;
    a.tile_rows = A->tiles_rows;
    const hipError_t e = launch_spmm_stream(a, A->cfg.lanes, nrhs);
    return e == hipSuccess ? DAMN_OK : DAMN_ERR_HIP;
  }
  const hipError_t e = launch_spmm(a, A->cfg.lanes, nrhs);
  return e == hipSuccess ? DAMN_OK : DAMN_ERR_HIP;
}

int damn_set_config(damn_mat A, const damn_config* cfg) {
  if (A == nullptr || cfg == nullptr) return DAMN_ERR_INVALID_ARG;
  if (cfg->variant != DAMN_VAR_VECTOR && cfg->variant != DAMN_VAR_STREAM)
    return DAMN_ERR_INVALID_ARG;
  if (!valid_pow2_lanes(cfg->lanes)) return DAMN_ERR_INVALID_ARG;
  damn_config c = *cfg;
  if (c.variant == DAMN_VAR_VECTOR) {
    if (c.unroll != 1 && c.unroll != 2 && c.unroll != 4) return DAMN_ERR_INVALID_ARG;
    // the tiles of the last stream configuration stay: block formats and
    // conjugate gradients run the stream kernels on them
    if (c.tile == 0) c.tile = A->cfg.tile;
    c.cache = DAMN_CACHE_NT;
  } else {
    if (c.tile < 256 || c.tile > 4096 || (c.tile % 8) != 0) return DAMN_ERR_UNSUPPORTED;
    if (c.cache != DAMN_CACHE_NT && c.cache != DAMN_CACHE_PLAIN) return DAMN_ERR_INVALID_ARG;
    const bool plain_cell = A->block == 1 &&
                            (A->format == DAMN_FORMAT_DA16 || A->format == DAMN_FORMAT_CSR32) &&
                            (A->dtype == DAMN_F64 || A->dtype == DAMN_F32);
    if (c.cache == DAMN_CACHE_PLAIN && !plain_cell) return DAMN_ERR_UNSUPPORTED;
    if (c.unroll == 0) c.unroll = 1;
    if (c.unroll != 1 && c.unroll != 2) return DAMN_ERR_INVALID_ARG;
    if (c.unroll == 2 && (A->block > 1 || format_is_coo(A->format))) return DAMN_ERR_UNSUPPORTED;
    const int st = build_tiles(A, tile_cap(A, c.tile), nullptr);
    if (st != DAMN_OK) return st;
  }
  A->cfg = c;
  return DAMN_OK;
}

int damn_get_config(damn_mat A, damn_config* cfg) {
  if (A == nullptr || cfg == nullptr) return DAMN_ERR_INVALID_ARG;
  *cfg = A->cfg;
  return DAMN_OK;
}

int damn_stream_read(const void* src, size_t bytes, int32_t passes, double* sink, int32_t mode,
                     int32_t tile_bytes, void* stream) {
  if ((src == nullptr && bytes > 0) || sink == nullptr || bytes % 16 != 0 || passes < 1)
    return DAMN_ERR_INVALID_ARG;
  if (mode < DAMN_READ_NT || mode > DAMN_READ_LDS_PLAIN) return DAMN_ERR_INVALID_ARG;
  const bool lds = mode == DAMN_READ_LDS_NT || mode == DAMN_READ_LDS_PLAIN;
  if (lds && (tile_bytes < 1024 || tile_bytes > 65536 || tile_bytes % 16 != 0))
    return DAMN_ERR_INVALID_ARG;
  // workgroups per pass: one per tile (LDS modes), at most 65536 slices otherwise
  const int64_t per_pass =
      lds ? int64_t(bytes / 16 + tile_bytes / 16 - 1) / (tile_bytes / 16) : int64_t(65536);
  if (per_pass * passes > INT32_MAX) return DAMN_ERR_UNSUPPORTED;
  const hipError_t e = launch_stream_read(src, int64_t(bytes), passes, sink, mode, tile_bytes,
                                          static_cast<hipStream_t>(stream));
  return e == hipSuccess ? DAMN_OK : DAMN_ERR_HIP;
}

int damn_gather_read(const double* x, int64_t n, int64_t rows, int32_t per_row,
                     int32_t halfwidth, const int32_t* offs, double* sink, void* stream) {
  if (x == nullptr || sink == nullptr || n < 1 || rows < 0 || per_row < 0 || halfwidth < 0 ||
      halfwidth > (1 << 30))
    return DAMN_ERR_INVALID_ARG;
  if ((rows + 255) / 256 > INT32_MAX) return DAMN_ERR_UNSUPPORTED;
  const hipError_t e = launch_gather_read(x, n, rows, per_row, halfwidth, offs, sink,
                                          static_cast<hipStream_t>(stream));
  return e == hipSuccess ? DAMN_OK : DAMN_ERR_HIP;
}

int damn_stream_copy(const void* src, void* dst, size_t bytes, void* stream) {
  if (((src == nullptr || dst == nullptr) && bytes > 0) || bytes % 16 != 0)
    return DAMN_ERR_INVALID_ARG;
  const hipError_t e =
      launch_stream_copy(src, dst, int64_t(bytes), static_cast<hipStream_t>(stream));
  return e == hipSuccess ? DAMN_OK : DAMN_ERR_HIP;
}

}  // extern "C"
