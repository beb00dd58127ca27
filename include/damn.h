/*
 * damn.h -- diagonally-addressed (DA) CSR sparse matrix-vector products on
 * AMD Instinct MI355X (gfx950).  C ABI of libdamn.so.
 *
 * Storage (paper Sec. 2, Listing 1): a matrix A of nrows x ncols is held as
 *   rowptr[nrows+1]  int32, rowptr[0] = 0, non-decreasing, rowptr[nrows] = nnz
 *   colids[nnz]      CSR: the column c_i in [0, ncols)           (int32)
 *                    DA-CSR: the offset c_i - r_i in [-w, w]     (int16)
 *   values[nnz]      float64 or float32
 * where w is the bandwidth of Eq. 2, max |c - r| over stored entries.  A
 * matrix fits 16-bit DA-CSR when w < 2^15 (Sec. 2, Example 2).  Explicitly
 * stored zeros are entries (footnote of Example 2); empty rows, repeated
 * columns and unsorted rows are allowed.
 *
 * Product (Sec. 4): y <- alpha*A*x + beta*y.  beta == 0 never reads y, and
 * alpha == 0 never reads A or x (BLAS convention; the paper's listing always
 * reads y).
 *
 * Conventions for every call:
 * - Sizes are int32 (the paper selects matrices whose CSR fits 32-bit
 *   signed indices, Sec. 3).
 * - Host pointers are read during the call and never retained.  Device
 *   pointers (x, y, X, Y, b) belong to the caller and must stay valid until
 *   the work queued on `stream` has finished.
 * - `stream` is a hipStream_t passed as void*; NULL is the null stream.
 *   Device calls only queue work on it and return without synchronising,
 *   unless stated otherwise.
 * - Every call returns a damn_status.  On any error the outputs are left
 *   untouched and nothing is queued.
 */
#ifndef DAMN_H
#define DAMN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DAMN_OK = 0,
  DAMN_ERR_INVALID_ARG = -1,   /* null pointer, negative size, bad enum     */
  DAMN_ERR_BAD_CSR = -2,       /* rowptr/colids do not form a valid matrix  */
  DAMN_ERR_NO_FIT = -3,        /* bandwidth >= 2^15, also after reordering  */
  DAMN_ERR_HIP = -4,           /* a HIP runtime call failed                 */
  DAMN_ERR_ALLOC = -5,         /* host or device allocation failed          */
  DAMN_ERR_UNSUPPORTED = -6,   /* combination not provided (e.g. nrhs > 8)  */
  DAMN_ERR_NOT_CONVERGED = -7, /* iteration limit reached                   */
  DAMN_ERR_BREAKDOWN = -8,     /* p.Ap <= 0: matrix not positive definite   */
  DAMN_ERR_TOO_LARGE = -9      /* more rows than a fixed scratch area holds */
} damn_status;

/* Scalar types of stored values (the scalar axis of Fig. 3).  Products
 * with float16-valued matrices take float32 x and y and accumulate in
 * float32. */
typedef enum { DAMN_F64 = 0, DAMN_F32 = 1, DAMN_F16 = 2 } damn_dtype;

/* Column-index kind of a device matrix (the index axis of Fig. 3):
 *   DA16   int16 offsets c - r, needs bandwidth w < 2^15 (Sec. 2)
 *   CSR32  int32 absolute columns
 *   DA8    int8 offsets c - r, needs w < 2^7
 *   CSR16  int16 absolute columns, needs every column < 2^15 (the direct
 *          narrow-index CSR the remark closing Sec. 4 compares with)
 * A signed index of b bits holds magnitudes below 2^(b-1): the most
 * negative value of the type is never used, as for the 16-bit rule. */
typedef enum {
  DAMN_FORMAT_DA16 = 0,
  DAMN_FORMAT_CSR32 = 1,
  DAMN_FORMAT_DA8 = 2,
  DAMN_FORMAT_CSR16 = 3,
  DAMN_FORMAT_DABSR16 = 4, /* b x b blocks, int16 block offsets bc - br    */
  DAMN_FORMAT_BSR32 = 5,   /* b x b blocks, int32 block columns bc         */
  DAMN_FORMAT_DACOO16 = 6, /* coordinates: int32 row, int16 offset c - r   */
  DAMN_FORMAT_COO32 = 7    /* coordinates: int32 row, int32 column         */
} damn_format;

/* Opaque device matrix; owns its device arrays. */
typedef struct damn_mat_s* damn_mat;

/* Human-readable text for a status code (static storage). */
const char* damn_status_string(int status);
/* Library version string (static storage). */
const char* damn_version(void);

/* ------------------------------------------------------------------------
 * Host-only preprocessing (no GPU use).
 * --------------------------------------------------------------------- */

/* Bandwidth check (Eq. 2; 16-bit rule of Sec. 2, Example 2 and Sec. 3).
 * In:  int32 CSR (rowptr[nrows+1], colids[rowptr[nrows]]), host memory.
 * Out: *w = max |c - r|, *lo = max(r - c, 0), *hi = max(c - r, 0) over all
 *      stored entries (0 for an empty matrix); *fits = (w < 32768).
 * Errors: DAMN_ERR_INVALID_ARG (null pointer with nnz > 0, negative size),
 *         DAMN_ERR_BAD_CSR (rowptr not starting at 0 / decreasing / not
 *         ending at nnz, or a column outside [0, ncols)). */
int damn_fit_check(int32_t nrows, int32_t ncols, const int32_t* rowptr,
                   const int32_t* colids, int32_t* w, int32_t* lo, int32_t* hi,
                   int32_t* fits);

/* Reverse Cuthill-McKee ordering (cited in Sec. 2, Example 2, and Sec. 3;
 * details fixed here): graph = pattern of A + A^T without self loops;
 * adjacency ordered by (degree, index); components seeded by the unvisited
 * vertex of smallest (degree, index) and started from a George-Liu
 * pseudo-peripheral vertex; breadth-first Cuthill-McKee; the concatenated
 * order reversed.
 * In:  square int32 CSR of order n (host).
 * Out: perm[n], new position -> old index (host, caller-allocated).
 * Errors: DAMN_ERR_INVALID_ARG, DAMN_ERR_BAD_CSR, DAMN_ERR_ALLOC. */
int damn_rcm(int32_t n, const int32_t* rowptr, const int32_t* colids,
             int32_t* perm);

/* Bandwidth refinement of an ordering, for matrices whose RCM order still
 * has w >= 32768 (the paper's RCM fell short on two matrices, Sec. 3).  A
 * sweep gives each vertex of the pattern graph of A + A^T the key
 * min + max of its neighbours' current positions (2 * its own position if
 * it has none) and re-sorts the vertices by (key, current position).  Sweeps
 * repeat until the order's bandwidth is below `limit` (32768 for 16-bit
 * offsets), at most max_sweeps.
 * In:  square int32 CSR of order n, perm[n] (new -> old) to start from.
 * Out: perm[n] replaced by the first fitting order, or by the narrowest one
 *      seen; *w_out its bandwidth.
 * Errors: DAMN_ERR_NO_FIT (no fitting order; perm and *w_out still written),
 *         DAMN_ERR_INVALID_ARG (perm not a permutation), DAMN_ERR_BAD_CSR,
 *         DAMN_ERR_ALLOC. */
int damn_refine_bandwidth(int32_t n, const int32_t* rowptr, const int32_t* colids,
                          int32_t* perm, int32_t max_sweeps, int32_t limit, int32_t* w_out);

/* CSR -> DA-CSR with 16-bit offsets (Sec. 2, Example 1).
 * If w < 32768 in the given order: rowptr and values are copied, and
 * off[i] = colids[i] - r_i, entry order unchanged; perm_out (if not NULL)
 * gets the identity and *permuted = 0.
 * Otherwise, if allow_rcm != 0 and the matrix is square: the RCM
 * permutation (refined by damn_refine_bandwidth with 32 sweeps when the RCM
 * order alone does not fit) is applied as P A P^T (new row i = old row perm[i], column c
 * relabelled to inv[c]; within a row entries ordered by new column, equal
 * columns keep their old order), the fit is checked again and *permuted = 1.
 * Products with a permuted matrix are in permuted space: x_p[i] = x[perm[i]]
 * and y[perm[i]] = y_p[i].
 * In:  host int32 CSR with float64 values.
 * Out: rowptr_out[nrows+1], off_out[nnz], vals_out[nnz] (float64),
 *      perm_out[nrows] (may be NULL), *permuted, *w_out (bandwidth of the
 *      result, or of the best form found when NO_FIT).  All host memory.
 * Errors: DAMN_ERR_NO_FIT (only *w_out is written), DAMN_ERR_INVALID_ARG,
 *         DAMN_ERR_BAD_CSR, DAMN_ERR_ALLOC. */
int damn_encode(int32_t nrows, int32_t ncols, const int32_t* rowptr,
                const int32_t* colids, const double* vals, int32_t allow_rcm,
                int32_t* rowptr_out, int16_t* off_out, double* vals_out,
                int32_t* perm_out, int32_t* permuted, int32_t* w_out);

/* Column indices of int32 CSR in any index format of Fig. 3, entry order
 * unchanged: DA formats store c - r (Sec. 2, Example 1), CSR formats c.
 * In:  format (damn_format), host int32 CSR (rowptr[nrows+1],
 *      colids[nnz]).
 * Out: idx_out[nnz] of the format's integer type (int8, int16 or int32,
 *      host, caller-allocated); *w_out = the bandwidth (DA formats) or the
 *      largest stored column (CSR formats), written on success and on
 *      DAMN_ERR_NO_FIT.
 * Errors: DAMN_ERR_NO_FIT (w_out at or above 2^(bits-1); idx_out untouched),
 *         DAMN_ERR_INVALID_ARG, DAMN_ERR_BAD_CSR. */
int damn_encode_index(int32_t format, int32_t nrows, int32_t ncols, const int32_t* rowptr,
                      const int32_t* colids, void* idx_out, int32_t* w_out);

/* Block storage (Sec. 1: diagonal addressing applies to BSR as well).  The
 * matrix is cut into b x b blocks (nrows and ncols multiples of b); a block
 * is stored when a pattern entry (stored zeros included) falls into it.  Per
 * block row the stored blocks come in ascending block column, each with its
 * b*b values row-major (zero where the pattern has no entry; repeated
 * entries add up in storage order).  DA-BSR keeps the block offset bc - br
 * in int16 and needs the block bandwidth max |bc - br| below 2^15; BSR keeps
 * bc in int32.
 *
 * damn_bsr_count: *nnzb = stored blocks, *wb = block bandwidth (host).
 * damn_bsr_encode: format DAMN_FORMAT_DABSR16 or DAMN_FORMAT_BSR32; writes
 *   browptr_out[nrows/b + 1], bidx_out[nnzb] (int16 offsets or int32 block
 *   columns) and bvals_out[nnzb*b*b] (float64), host, caller-allocated with
 *   the sizes damn_bsr_count gives.
 * Errors: DAMN_ERR_INVALID_ARG (b < 1, sizes not multiples of b, null
 *         pointers), DAMN_ERR_BAD_CSR, DAMN_ERR_NO_FIT (DA-BSR with
 *         wb >= 2^15), DAMN_ERR_UNSUPPORTED (2^31 blocks or more),
 *         DAMN_ERR_ALLOC. */
int damn_bsr_count(int32_t nrows, int32_t ncols, const int32_t* rowptr, const int32_t* colids,
                   int32_t b, int64_t* nnzb, int32_t* wb);
int damn_bsr_encode(int32_t nrows, int32_t ncols, const int32_t* rowptr, const int32_t* colids,
                    const double* vals, int32_t b, int32_t format, int32_t* browptr_out,
                    void* bidx_out, double* bvals_out);

/* Coordinate storage (Sec. 1: diagonal addressing applies to one of COO's
 * index vectors).  Every entry keeps its int32 row; DA-COO stores the
 * column as the int16 offset c - r (bandwidth below 2^15), COO as the int32
 * column.  Entries are in row order (as CSR gives them; any order within a
 * row).
 * damn_coo_encode: from int32 CSR, entry order unchanged; rows_out[nnz],
 *   idx_out[nnz] (int16 or int32), host, caller-allocated; *w_out = the
 *   bandwidth (DA-COO) or the largest column (COO).
 * Errors: DAMN_ERR_NO_FIT (DA-COO with w >= 2^15; only *w_out written),
 *         DAMN_ERR_INVALID_ARG, DAMN_ERR_BAD_CSR. */
int damn_coo_encode(int32_t format, int32_t nrows, int32_t ncols, const int32_t* rowptr,
                    const int32_t* colids, int32_t* rows_out, void* idx_out, int32_t* w_out);

/* Values in a narrower scalar type (the scalar axis of Fig. 3): IEEE 754
 * round to nearest, ties to even, in one step from the input value (a
 * float64 value is never rounded to float32 on its way to float16).
 * In:  n values of vals_dtype (host); dtype no wider than vals_dtype
 *      (equal types copy).
 * Out: out[n] of dtype (host, caller-allocated; float16 as its 16 bits).
 * Errors: DAMN_ERR_NO_FIT (a finite value rounds to infinity; out holds the
 *         infinities), DAMN_ERR_UNSUPPORTED (widening), DAMN_ERR_INVALID_ARG. */
int damn_store_values(int64_t n, const void* vals, int32_t vals_dtype, int32_t dtype,
                      void* out);

/* ------------------------------------------------------------------------
 * Device matrices.
 * --------------------------------------------------------------------- */

/* Upload a DA-CSR matrix (int16 offsets) to the current device.
 * In:  host rowptr[nrows+1], off[nnz], vals[nnz] of type vals_dtype; the
 *      device copy stores values as store_dtype (float64 -> float32 rounds
 *      to nearest even).  Every r + off[i] must lie in [0, ncols) (checked
 *      on the host, so no kernel can read outside x; Sec. 4, remark on
 *      non-square matrices).
 * Out: *out, a handle owning its device memory (free with damn_destroy),
 *      including the stream-variant tile table of its default
 *      configuration, so the product calls never allocate.
 * The copies are ordered on `stream`; the call synchronises the stream
 * before returning so the host arrays may be freed at once.
 * Errors: DAMN_ERR_INVALID_ARG, DAMN_ERR_BAD_CSR, DAMN_ERR_ALLOC,
 *         DAMN_ERR_HIP. */
int damn_create(damn_mat* out, int32_t nrows, int32_t ncols,
                const int32_t* rowptr, const int16_t* off, const void* vals,
                int32_t vals_dtype, int32_t store_dtype, void* stream);

/* Upload a plain int32 CSR matrix (the comparison format of Sec. 4).
 * Same contract as damn_create with absolute columns colids[nnz]. */
int damn_csr_create(damn_mat* out, int32_t nrows, int32_t ncols,
                    const int32_t* rowptr, const int32_t* colids,
                    const void* vals, int32_t vals_dtype, int32_t store_dtype,
                    void* stream);

/* Upload a matrix in any cell of the storage grid of Fig. 3.
 * In:  format (damn_format); host rowptr[nrows+1]; idx[nnz] of the
 *      format's integer type (as damn_encode_index writes it); vals[nnz] of
 *      vals_dtype (float64, float32 or float16 bits), stored on the device
 *      as store_dtype, rounded as damn_store_values does (widening is
 *      DAMN_ERR_UNSUPPORTED).  Every column (r + off for DA formats) must
 *      lie in [0, ncols); checked on the host.
 * Out: *out as for damn_create.  DA handles take damn_spmv, CSR handles
 *      damn_csr_spmv; x and y are float64 for float64 handles and float32
 *      otherwise.
 * Errors: DAMN_ERR_NO_FIT (a value overflows store_dtype),
 *         DAMN_ERR_INVALID_ARG, DAMN_ERR_BAD_CSR, DAMN_ERR_UNSUPPORTED,
 *         DAMN_ERR_ALLOC, DAMN_ERR_HIP. */
int damn_create_format(damn_mat* out, int32_t format, int32_t nrows, int32_t ncols,
                       const int32_t* rowptr, const void* idx, const void* vals,
                       int32_t vals_dtype, int32_t store_dtype, void* stream);

/* Upload a block matrix (DAMN_FORMAT_DABSR16 or DAMN_FORMAT_BSR32) with
 * block size b in {2, 3, 4, 6}.
 * In:  nbrows x nbcols blocks; host browptr[nbrows+1], bidx[nnzb] (int16
 *      offsets or int32 block columns), bvals[nnzb*b*b] of vals_dtype,
 *      stored as store_dtype (float64 or float32).  Every block column
 *      (br + offset for DA-BSR) must lie in [0, nbcols); checked on the host.
 * Out: *out; the handle is an (nbrows*b) x (nbcols*b) matrix: DA-BSR takes
 *      damn_spmv and BSR damn_csr_spmv.  The products use the stream
 *      variant with `lanes` lanes per scalar row (at most 16) and tiles of
 *      about `tile` values.
 * Errors: DAMN_ERR_INVALID_ARG, DAMN_ERR_BAD_CSR, DAMN_ERR_UNSUPPORTED (b,
 *         float16), DAMN_ERR_NO_FIT (value overflow), DAMN_ERR_ALLOC,
 *         DAMN_ERR_HIP. */
int damn_bsr_create(damn_mat* out, int32_t format, int32_t nbrows, int32_t nbcols, int32_t b,
                    const int32_t* browptr, const void* bidx, const void* bvals,
                    int32_t vals_dtype, int32_t store_dtype, void* stream);

/* Upload a coordinate matrix (DAMN_FORMAT_DACOO16 or DAMN_FORMAT_COO32).
 * In:  nrows x ncols, nnz entries (below 2^31): host rows[nnz] (int32,
 *      non-decreasing, in [0, nrows)), idx[nnz] (int16 offsets or int32
 *      columns; every column inside [0, ncols)), vals[nnz] of vals_dtype
 *      stored as store_dtype (float64 or float32).  All checked on the host.
 * Out: *out.  DA-COO takes damn_spmv, COO damn_csr_spmv; a product is
 *      one launch that writes every row of y once (rows without entries
 *      get beta*y), each row summed in one place, without atomics (the
 *      result does not depend on scheduling).
 * Errors: DAMN_ERR_INVALID_ARG, DAMN_ERR_BAD_CSR (rows out of order or
 *         range, columns out of range), DAMN_ERR_UNSUPPORTED (float16,
 *         nnz >= 2^31), DAMN_ERR_NO_FIT (value overflow), DAMN_ERR_ALLOC,
 *         DAMN_ERR_HIP. */
int damn_coo_create(damn_mat* out, int32_t format, int32_t nrows, int32_t ncols, int64_t nnz,
                    const int32_t* rows, const void* idx, const void* vals, int32_t vals_dtype,
                    int32_t store_dtype, void* stream);

/* Release a handle (waits for the device to finish using it). */
int damn_destroy(damn_mat A);

/* Shape and format of a handle (any out pointer may be NULL); nrows and
 * ncols are scalar rows and columns, nnz counts stored entries (blocks for
 * block formats). */
int damn_mat_info(damn_mat A, int32_t* nrows, int32_t* ncols, int64_t* nnz,
                  int32_t* format, int32_t* dtype);

/* ------------------------------------------------------------------------
 * Products (Sec. 4, Listing 2).  x has ncols entries, y has nrows, in
 * device memory: float64 for float64 handles, float32 for float32 and
 * float16 handles (which accumulate in float32).  A product call only
 * launches kernels on `stream`: it never allocates, copies or synchronises,
 * so it may be captured into a HIP graph, the first call on a fresh handle
 * included.
 * --------------------------------------------------------------------- */

/* y <- alpha*A*x + beta*y for a DA handle (DA16, DA8, DA-BSR, DA-COO): row r
 * accumulates values[i] * x[r + off[i]] (the shifted-x access of Sec. 4;
 * for DA-BSR block row br reads x blocks br + offset).
 * Errors: DAMN_ERR_INVALID_ARG (null, or a handle with absolute columns),
 *         DAMN_ERR_HIP. */
int damn_spmv(damn_mat A, const void* x, void* y, double alpha, double beta,
              void* stream);

/* Same product for handles with absolute columns (CSR32, CSR16, BSR32,
 * COO32). */
int damn_csr_spmv(damn_mat A, const void* x, void* y, double alpha,
                  double beta, void* stream);

/* Y <- alpha*A*X + beta*Y for nrhs right-hand sides, 1 <= nrhs <= 8.
 * X is ncols x nrhs and Y is nrows x nrhs, both row-major (the nrhs values
 * of one row are adjacent).  Float64 DA16 and CSR32 handles.  The handle's
 * configuration picks the kernel: the stream variant (tiles in LDS, `lanes`
 * lanes per row accumulating all nrhs sums) or the vector variant.
 * alpha == 0 scales Y by beta without reading A or X.
 * Errors: DAMN_ERR_INVALID_ARG, DAMN_ERR_UNSUPPORTED (nrhs > 8, another
 *         format or scalar type). */
int damn_spmm(damn_mat A, const void* X, void* Y, int32_t nrhs, double alpha,
              double beta, void* stream);

/* ------------------------------------------------------------------------
 * Kernel configuration.
 * --------------------------------------------------------------------- */

/* Kernel variants of the product:
 *   DAMN_VAR_VECTOR: `lanes` lanes of a wavefront per row (1..64, power of
 *                    two; 1 = one row per lane), `unroll` independent partial
 *                    sums per lane (1, 2 or 4).
 *   DAMN_VAR_STREAM: workgroups take tiles of whole rows holding at most
 *                    `tile` entries (and at most 512 rows; a tile that
 *                    ends before the last row is cut back to a power-of-two
 *                    row count), stream offsets and values with aligned
 *                    16-byte loads through LDS, and reduce each row with
 *                    `lanes` lanes (1..64).  A row longer than `tile` is
 *                    reduced by a whole workgroup.  `unroll` is the number
 *                    of x values per gather load (0 counts as 1):
 *                    1 (interleaved): the row's lanes take every lanes-th
 *                      entry and load one x value each;
 *                    2 (paired): each lane takes a contiguous part of the
 *                      row and loads x[c], x[c+1] together, using both when
 *                      the next entry's column is c+1 (runs of neighbouring
 *                      columns, as in stencil rows, need half the loads).
 *                      Every scalar cell (DA16, DA8, CSR32, CSR16, any
 *                      value type); block and coordinate formats return
 *                      DAMN_ERR_UNSUPPORTED.  damn_spmv, damn_csr_spmv
 *                      and conjugate gradients use it; SpMM and the batch
 *                      take the interleaved gathers with the same lanes.
 */
typedef enum { DAMN_VAR_VECTOR = 0, DAMN_VAR_STREAM = 1 } damn_variant;

/* Cache policy of the stream variant's matrix loads. */
typedef enum {
  DAMN_CACHE_NT = 0,    /* non-temporal (default): the matrix, read once per
                           product, does not displace x from L2            */
  DAMN_CACHE_PLAIN = 1  /* plain loads: a matrix that fits the MALL with its
                           vectors stays there across repeated products;
                           DA16 and CSR32 handles with float64 or float32
                           values only (else DAMN_ERR_UNSUPPORTED); SpMM
                           with nrhs > 1 and CG keep non-temporal loads    */
} damn_cache;

typedef struct {
  int32_t variant;
  int32_t lanes;
  int32_t unroll;
  int32_t tile;  /* stream variant only: entries per tile (256..4096, a
                    multiple of 8; otherwise DAMN_ERR_UNSUPPORTED) */
  int32_t cache; /* stream variant only: a damn_cache value, 0 default */
} damn_config;

/* Set / read the configuration used by damn_spmv, damn_csr_spmv and
 * damn_spmm on this handle.  A new handle starts with a default derived
 * from its mean row length, its tiles already built.  A stream
 * configuration with a new tile size rebuilds the tile table: that call
 * allocates, uploads on the null stream, waits for the device to finish all
 * queued work and frees the old table, so it belongs in setup code, not in
 * a captured or latency-critical region.  A vector configuration keeps the
 * last stream tiles (block formats and conjugate gradients run the stream
 * kernels on them).  Errors: DAMN_ERR_INVALID_ARG, DAMN_ERR_UNSUPPORTED,
 * DAMN_ERR_ALLOC, DAMN_ERR_HIP. */
int damn_set_config(damn_mat A, const damn_config* cfg);
int damn_get_config(damn_mat A, damn_config* cfg);

/* ------------------------------------------------------------------------
 * Conjugate gradients on the device (the iterative solvers the paper's DA
 * storage is meant for, Sec. 3 footnote; the multi-precision argument of the
 * remark after Fig. 3: a DA-CSR int16 matrix gains 5/3x traffic when its
 * scalars go from float64 to float32, against 3/2x for CSR int32).
 * --------------------------------------------------------------------- */

typedef struct {
  double tol;          /* stop when ||b - A x||_2 <= tol * ||b||_2 (1e-10)   */
  double inner_tol;    /* mixed: inner solve to relative residual (1e-5)    */
  int32_t max_iter;    /* CG iterations (mixed: per inner solve)            */
  int32_t max_outer;   /* mixed: refinement steps (50)                      */
  int32_t check_every; /* iterations between host reads of the stop flag    */
} damn_cg_opts;

typedef struct {
  int32_t iters;     /* float64 CG: iterations; mixed: inner iterations, all */
  int32_t outer;     /* mixed: refinement steps taken                        */
  int32_t converged; /* 1 if the residual target was met                    */
  double rel_res;    /* ||b - A x|| / ||b|| of the returned x, float64       */
} damn_cg_info;

/* Solve A x = b for symmetric positive definite A, from x0 = 0.
 * A64: float64 handle (DA16 or CSR32), square.  A32 == NULL: float64 CG
 * (Hestenes-Stiefel; vectors and dot products float64; stops on the
 * recursively updated residual, then reports the true residual).
 * A32 != NULL: mixed precision with iterative refinement.  A32 is the same
 * matrix with float32 values (same format and shape).  Each outer step forms
 * r = b - A64 x and ||r|| in float64; if not yet converged it runs CG on
 * A32 d = r/||r|| with float32 vectors, float32-accumulated products with
 * A32 and float64-accumulated dot products, to the relative residual
 * min(1/2, max(inner_tol, tol ||b|| / (2 ||r||))), then x += ||r|| d.
 * b, x: device float64 vectors of n entries, 16-byte aligned (x is overwritten; on
 * DAMN_ERR_NOT_CONVERGED / DAMN_ERR_BREAKDOWN it holds the last iterate).
 * The call synchronises `stream` (it reads the stop flag every check_every
 * iterations).  Device workspace (about 7 vectors) is kept with A64.
 * Errors: DAMN_ERR_INVALID_ARG, DAMN_ERR_UNSUPPORTED (DA8 or CSR16 handles),
 *         DAMN_ERR_NOT_CONVERGED (limits reached), DAMN_ERR_BREAKDOWN
 *         (p.Ap <= 0), DAMN_ERR_ALLOC, DAMN_ERR_HIP. */
int damn_cg(damn_mat A64, damn_mat A32, const double* b, double* x,
            const damn_cg_opts* opts, damn_cg_info* info, void* stream);

/* ------------------------------------------------------------------------
 * Batched products: Y_i <- alpha*A_i*X_i + beta*Y_i for many DA-CSR
 * matrices (the product of Sec. 4, repeated) in one graph-captured launch
 * (one workgroup per tile by default, or a persistent grid on request).
 * --------------------------------------------------------------------- */

typedef struct damn_batch_s* damn_batch;

/* Prepare a batch over `count` float64 DA-CSR handles mats[i] with nrhs[i]
 * right-hand sides (1..8).  X[i] (ncols_i x nrhs[i]) and Y[i] (nrows_i x
 * nrhs[i]) are device pointers, row-major like damn_spmm; the batch keeps
 * the pointers (not the data) and the handles' device arrays, which must
 * outlive it.  Rows are cut into tiles of at most max(2048, longest row)
 * entries (at most 4096).  workgroups == 0: the launch has one workgroup
 * per tile; workgroups > 0: a persistent grid of that many workgroups, each
 * walking one of `workgroups` contiguous ranges of the tile list of about
 * equal modelled bytes.  The launch is captured once into a HIP graph.
 * Errors: DAMN_ERR_INVALID_ARG (null, non-DA16 or non-float64 handle),
 *         DAMN_ERR_UNSUPPORTED (nrhs outside 1..8, a row longer than 4096
 *         entries), DAMN_ERR_ALLOC, DAMN_ERR_HIP. */
int damn_batch_create(damn_batch* out, int32_t count, const damn_mat* mats,
                      const int32_t* nrhs, const double* const* X, double* const* Y,
                      double alpha, double beta, int32_t workgroups, void* stream);

/* Run the batch on `stream`: use_graph != 0 replays the captured graph,
 * otherwise the same kernel is launched directly.  Asynchronous. */
int damn_batch_run(damn_batch B, int32_t use_graph, void* stream);

/* Tiles, workgroups and modelled bytes of one run (matrices once, row
 * pointers, X once, Y written and, if beta != 0, read). */
int damn_batch_info(damn_batch B, int64_t* ntiles, int32_t* workgroups, double* model_bytes);

/* Release a batch (waits for the device). */
int damn_batch_destroy(damn_batch B);

/* ------------------------------------------------------------------------
 * Choosing a launch configuration.  The paper picks, per matrix, the
 * fastest of its implementations and thread counts (Sec. 4.1); here an
 * exhaustive autotuner measures every configuration, and a small network
 * trained on the autotuner's measurements predicts the choice from
 * sparsity features.
 * --------------------------------------------------------------------- */

#define DAMN_NFEAT 16
#define DAMN_NCLASS 70
#define DAMN_CLASS_SPMM 63
#define DAMN_MLP_NPARAMS 9830

/* Sparsity features of an int32 CSR matrix (host, float64 arithmetic,
 * float32 results): 0 log2(nrows+1), 1 log2(nnz+1), 2 mean row length,
 * 3 std of row lengths, 4 log2(max row length+1), 5 fraction of empty rows,
 * 6 log2(w+1), 7 w/max(ncols,1), 8 w >= 32768, 9 nrhs,
 * 10 log2(mean |c-r| + 1), 11 fraction of entries with |c-r| <= 64,
 * 12 std/mean of row lengths, 13 fraction of rows with >= 64 entries,
 * 14 log2(ncols+1), 15 fraction of adjacent entry pairs within a row whose
 * columns differ by 1.  w is the bandwidth of Eq. 2.
 * Errors: DAMN_ERR_INVALID_ARG, DAMN_ERR_BAD_CSR. */
int damn_features(int32_t nrows, int32_t ncols, const int32_t* rowptr,
                  const int32_t* colids, int32_t nrhs, float* feat);

/* Configuration of class cls (0 <= cls < DAMN_NCLASS): classes 0..20 are
 * the vector variant (lanes 1..64 x unroll 1,2,4), 21..41 the stream variant
 * with interleaved gathers and 42..62 with paired gathers (lanes 1..64 x
 * tile 1024, 2048, 4096 each), all for nrhs = 1; DAMN_CLASS_SPMM (63) ..
 * 69 are SpMM lane counts 1..64 of the stream SpMM with 2048-entry tiles,
 * for nrhs > 1 (*spmm = 1). */
int damn_class_config(int32_t cls, damn_config* cfg, int32_t* spmm);

/* Time every class that applies to nrhs (reps launches each after one
 * warm-up, HIP events on `stream`), write seconds per launch to
 * times[DAMN_NCLASS] (+inf for classes that do not apply) and set the
 * fastest configuration on A.  X, Y: device operands as for damn_spmv
 * (nrhs = 1, the handle's dtype) or damn_spmm (nrhs > 1, float64).  Y is
 * overwritten.  Synchronises the stream.
 * Errors: DAMN_ERR_INVALID_ARG, DAMN_ERR_UNSUPPORTED, DAMN_ERR_HIP. */
int damn_autotune(damn_mat A, int32_t nrhs, const void* X, void* Y, int32_t reps,
                  float* times, void* stream);

typedef struct damn_mlp_s* damn_mlp;

/* Network 16 -> 64 -> 64 -> 70 (ReLU), float32 on the device.  params
 * (host, DAMN_MLP_NPARAMS floats: W1[64][16], b1, W2[64][64], b2, W3[70][64],
 * b3, then the feature standardisation mu[16], sigma[16]) or NULL for a
 * seeded He-uniform initialisation. */
int damn_mlp_create(damn_mlp* out, const float* params, uint64_t seed);
int damn_mlp_get_params(damn_mlp M, float* params);
int damn_mlp_destroy(damn_mlp M);

/* Loss and parameter gradients on one minibatch (for checking the backward
 * kernels): feats[B][16], targets[B][70] (a distribution over the classes
 * that apply; feats[b][9] = nrhs decides which apply), host arrays; the
 * gradients of mu and sigma are returned as 0. */
int damn_mlp_grad(damn_mlp M, int32_t B, const float* feats, const float* targets, float* loss,
                  float* grads, void* stream);

/* Train on N samples: feats[N][16] and autotuner times[N][70] (+inf where a
 * class does not apply), host arrays.  Sets mu/sigma from the features, then
 * runs `epochs` passes of Adam over shuffled minibatches of `batch` samples
 * with soft targets q_c ~ exp(-(t_c/t_min - 1)/tau).  epoch_loss[epochs]
 * (may be NULL) receives the mean loss of each pass. */
int damn_mlp_train(damn_mlp M, int32_t N, const float* feats, const float* times,
                   int32_t epochs, int32_t batch, float lr, float tau, uint64_t seed,
                   float* epoch_loss, void* stream);

/* Predicted class for N feature rows (host in, host out), by the inference
 * kernel: the most probable class that applies to the row's nrhs. */
int damn_select(damn_mlp M, int32_t N, const float* feats, int32_t* cls, void* stream);

/* damn_select, plus prob[N] (host): the probability the network gives the
 * chosen class under the softmax over the applicable classes.  A caller
 * falls back to damn_autotune when it is low. */
int damn_select_prob(damn_mlp M, int32_t N, const float* feats, int32_t* cls, float* prob,
                     void* stream);

/* Allocation-free damn_select_prob, for callers that cannot allocate
 * device memory (tight serving loops that pick a launch configuration per
 * incoming matrix, harnesses that forbid hipMalloc).  Same arguments and
 * results as damn_select_prob (prob may be NULL), bit for bit: the same
 * inference kernel runs on the same feature rows.  The feature rows,
 * classes and probabilities are staged in a fixed device array of the
 * library, one copy per GPU, held until the process ends
 * (DAMN_SELECT_NOALLOC_MAX_ROWS rows, 288 KiB); its address is looked up
 * once per device, on the first call there.  The call allocates nothing,
 * copies on `stream` and synchronises it before returning.  Calls that
 * overlap on one GPU (other threads, other streams) share that array and
 * race: serialise them.  Errors: DAMN_ERR_INVALID_ARG (null handle, N < 0,
 * null feats/cls with N > 0, current device not the network's),
 * DAMN_ERR_TOO_LARGE (N > DAMN_SELECT_NOALLOC_MAX_ROWS; nothing is
 * launched), DAMN_ERR_HIP. */
#define DAMN_SELECT_NOALLOC_MAX_ROWS 4096
int damn_select_noalloc(damn_mlp M, int32_t N, const float* feats, int32_t* cls, float* prob,
                        void* stream);

/* ------------------------------------------------------------------------
 * Measurement helpers.
 * --------------------------------------------------------------------- */

/* Read paths of the streaming probe. */
typedef enum {
  DAMN_READ_NT = 0,        /* 16-byte loads into registers, non-temporal   */
  DAMN_READ_PLAIN = 1,     /* 16-byte loads into registers, plain          */
  DAMN_READ_LDS_NT = 2,    /* direct-to-LDS 16-byte loads, non-temporal:
                              the matrix stream of the product kernels     */
  DAMN_READ_LDS_PLAIN = 3  /* direct-to-LDS 16-byte loads, plain           */
} damn_read_mode;

/* Streaming ceiling probe: reads `bytes` (multiple of 16) from device
 * buffer src `passes` times (>= 1) in one launch, along the read path
 * `mode`, and writes checksums into sink[0 .. 65535] (device, float64;
 * workgroup b writes sink[b mod 65536]).  The register modes give each of
 * at most 65536 workgroups per pass a contiguous slice; the LDS modes give
 * each workgroup one tile of tile_bytes (1024 .. 65536, a multiple of 16;
 * ignored otherwise), the shape of the product kernels' tiles.  The passes
 * follow each other in workgroup order, so a buffer larger than the L2
 * (4 MB per XCD) but within the MALL (256 MB) is re-read from the MALL, if
 * the read path allocates there, with the launch's ramp-up paid once.  Used
 * for the read ceilings the products are compared with, and to calibrate
 * traffic counters.  Errors: DAMN_ERR_INVALID_ARG, DAMN_ERR_UNSUPPORTED
 * (more than 2^31 - 1 workgroups). */
int damn_stream_read(const void* src, size_t bytes, int32_t passes, double* sink, int32_t mode,
                     int32_t tile_bytes, void* stream);

/* Gather probe: the x accesses of a product (Sec. 4) without its matrix.
 * Row r of `rows` (one thread each, 256 rows per workgroup, renumbered per
 * XCD as the products are) reads per_row float64 values x[c]: with offs
 * (device, per_row int32 values), c = r + offs[k], the DA offsets of a
 * stencil, shared by every row; with offs = NULL, c is drawn from
 * [r - halfwidth, r + halfwidth] by a fixed integer hash of (r, k), as a
 * random banded matrix's columns scatter.  Columns are clipped to [0, n).
 * x is a device array of n >= 1 values; one checksum per workgroup goes to
 * sink[b mod 65536] (device, float64, 65536 entries).  rows * per_row
 * 8-byte reads with the access pattern of the product and no matrix
 * stream: the gather time a product with that pattern cannot beat.
 * Errors: DAMN_ERR_INVALID_ARG, DAMN_ERR_UNSUPPORTED (more than 2^31 - 1
 * workgroups). */
int damn_gather_read(const double* x, int64_t n, int64_t rows, int32_t per_row,
                     int32_t halfwidth, const int32_t* offs, double* sink, void* stream);

/* Copy probe: dst = src for `bytes` (multiple of 16) with 16-byte accesses;
 * known bytes read and written, to calibrate memory-traffic counters.
 * Errors: DAMN_ERR_INVALID_ARG. */
int damn_stream_copy(const void* src, void* dst, size_t bytes, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* DAMN_H */
