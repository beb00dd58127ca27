"""Python binding of libdamn.so (diagonally-addressed CSR SpMV on MI355X).

Argument marshalling only: every step runs in the C++/HIP library.  Host
arrays are NumPy; device vectors are torch tensors on a HIP device, passed
by pointer together with the current torch stream.  Importing the package
loads the library and raises if it has not been built
(`python -m paper_2307_06305_amd.build`).

Names follow the C ABI of include/damn.h without the `damn_` prefix.
"""

from __future__ import annotations

import ctypes as C
import os

import numpy as np

from ._lib import DamnError, NoFit, lib, LIB_PATH  # noqa: F401

F64, F32, F16 = 0, 1, 2
FORMAT_DA16, FORMAT_CSR32, FORMAT_DA8, FORMAT_CSR16 = 0, 1, 2, 3
FORMAT_DABSR16, FORMAT_BSR32 = 4, 5
FORMAT_DACOO16, FORMAT_COO32 = 6, 7
VAR_VECTOR, VAR_STREAM = 0, 1
SELECT_NOALLOC_MAX_ROWS = 4096  # DAMN_SELECT_NOALLOC_MAX_ROWS

# the storage grid of Fig. 3: format -> (index dtype, holds DA offsets)
FORMATS = {FORMAT_DA16: (np.int16, True), FORMAT_CSR32: (np.int32, False),
           FORMAT_DA8: (np.int8, True), FORMAT_CSR16: (np.int16, False),
           FORMAT_DABSR16: (np.int16, True), FORMAT_BSR32: (np.int32, False),
           FORMAT_DACOO16: (np.int16, True), FORMAT_COO32: (np.int32, False)}
VALUE_DTYPES = {F64: np.float64, F32: np.float32, F16: np.float16}

_I32P = C.POINTER(C.c_int32)


def _check(st, what):
    if st != 0:
        raise DamnError(st, what)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _ptr(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


def _csr_arrays(nrows, rowptr, *entry_arrays):
    """The C ABI takes nnz from rowptr[nrows]: check the array lengths
    against it before handing the pointers over."""
    rp = _i32(rowptr)
    if nrows < 0 or rp.shape != (nrows + 1,):
        raise DamnError(-2, "rowptr must have nrows+1 entries")
    nnz = int(rp[nrows])
    for a in entry_arrays:
        if nnz < 0 or len(a) != nnz:
            raise DamnError(-2, "entry arrays must have rowptr[nrows] entries")
    return rp


def version() -> str:
    return lib.damn_version().decode()


def status_string(code: int) -> str:
    return lib.damn_status_string(int(code)).decode()


# ---------------------------------------------------------------------------
# host preprocessing
# ---------------------------------------------------------------------------

def fit_check(nrows, ncols, rowptr, colids):
    """(w, lo, hi, fits) of Eq. 2 for an int32 CSR matrix (host)."""
    c = _i32(colids)
    rp = _csr_arrays(nrows, rowptr, c)
    w, lo, hi, f = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
    _check(lib.damn_fit_check(nrows, ncols, _ptr(rp, C.c_int32), _ptr(c, C.c_int32),
                              C.byref(w), C.byref(lo), C.byref(hi), C.byref(f)), "fit_check")
    return w.value, lo.value, hi.value, bool(f.value)


def rcm(n, rowptr, colids):
    """Reverse Cuthill-McKee permutation (new -> old), int32 (host)."""
    c = _i32(colids)
    rp = _csr_arrays(n, rowptr, c)
    perm = np.empty(n, dtype=np.int32)
    _check(lib.damn_rcm(n, _ptr(rp, C.c_int32), _ptr(c, C.c_int32), _ptr(perm, C.c_int32)),
           "rcm")
    return perm


def refine_bandwidth(n, rowptr, colids, perm, max_sweeps=32, limit=2**15):
    """Midpoint refinement of an ordering (host).  Returns (perm, w, fits)."""
    c = _i32(colids)
    rp = _csr_arrays(n, rowptr, c)
    p = np.array(perm, dtype=np.int32, copy=True)
    if p.shape != (n,):
        raise DamnError(-1, "perm must have n entries")
    w = C.c_int32()
    st = lib.damn_refine_bandwidth(n, _ptr(rp, C.c_int32), _ptr(c, C.c_int32),
                                   _ptr(p, C.c_int32), int(max_sweeps), int(limit), C.byref(w))
    if st not in (0, -3):
        raise DamnError(st, "refine_bandwidth")
    return p, w.value, st == 0


def encode(nrows, ncols, rowptr, colids, vals, allow_rcm=True):
    """CSR -> DA-CSR int16 (host).  Returns dict(rowptr, off, vals, perm,
    permuted, w); raises NoFit (with .w) when no fitting form exists."""
    c = _i32(colids)
    v = np.ascontiguousarray(vals, dtype=np.float64)
    rp = _csr_arrays(nrows, rowptr, c, v)
    nnz = int(rp[nrows])
    rp_out = np.empty(nrows + 1, dtype=np.int32)
    off = np.empty(nnz, dtype=np.int16)
    v_out = np.empty(nnz, dtype=np.float64)
    perm = np.empty(nrows, dtype=np.int32)
    permuted, w = C.c_int32(), C.c_int32()
    st = lib.damn_encode(nrows, ncols, _ptr(rp, C.c_int32), _ptr(c, C.c_int32),
                         _ptr(v, C.c_double), int(allow_rcm), _ptr(rp_out, C.c_int32),
                         _ptr(off, C.c_int16), _ptr(v_out, C.c_double), _ptr(perm, C.c_int32),
                         C.byref(permuted), C.byref(w))
    if st == -3:
        raise NoFit(w.value)
    _check(st, "encode")
    return {"rowptr": rp_out, "off": off, "vals": v_out, "perm": perm,
            "permuted": bool(permuted.value), "w": w.value}


def encode_index(fmt, nrows, ncols, rowptr, colids):
    """Column indices of int32 CSR in format fmt (FORMAT_*), entry order
    unchanged (host).  Returns (idx, w); raises NoFit (with .w)."""
    c = _i32(colids)
    rp = _csr_arrays(nrows, rowptr, c)
    if fmt not in FORMATS:
        raise DamnError(-1, "encode_index: unknown format")
    dt, _ = FORMATS[fmt]
    idx = np.empty(int(rp[nrows]), dtype=dt)
    w = C.c_int32()
    st = lib.damn_encode_index(int(fmt), nrows, ncols, _ptr(rp, C.c_int32), _ptr(c, C.c_int32),
                               idx.ctypes.data_as(C.c_void_p), C.byref(w))
    if st == -3:
        raise NoFit(w.value, "bandwidth" if FORMATS[fmt][1] else "column",
                    8 * np.dtype(dt).itemsize)
    _check(st, "encode_index")
    return idx, w.value


def bsr_encode(nrows, ncols, rowptr, colids, vals, b, fmt=FORMAT_DABSR16):
    """int32 CSR -> BSR / DA-BSR with b x b blocks (host).  Returns
    dict(browptr, bidx, bvals (nnzb, b, b), wb); raises NoFit (with .w = the
    block bandwidth) for DA-BSR when it does not fit int16."""
    c = _i32(colids)
    v = np.ascontiguousarray(vals, dtype=np.float64)
    rp = _csr_arrays(nrows, rowptr, c, v)
    nnzb, wb = C.c_int64(), C.c_int32()
    _check(lib.damn_bsr_count(nrows, ncols, _ptr(rp, C.c_int32), _ptr(c, C.c_int32), int(b),
                              C.byref(nnzb), C.byref(wb)), "bsr_count")
    if fmt not in (FORMAT_DABSR16, FORMAT_BSR32):
        raise DamnError(-1, "bsr_encode: not a block format")
    nb = nnzb.value
    brp = np.empty(nrows // b + 1, dtype=np.int32)
    bidx = np.empty(nb, dtype=FORMATS[fmt][0])
    bvals = np.empty((nb, b, b), dtype=np.float64)
    st = lib.damn_bsr_encode(nrows, ncols, _ptr(rp, C.c_int32), _ptr(c, C.c_int32),
                             _ptr(v, C.c_double), int(b), int(fmt), _ptr(brp, C.c_int32),
                             bidx.ctypes.data_as(C.c_void_p), _ptr(bvals, C.c_double))
    if st == -3:
        raise NoFit(wb.value, "block bandwidth")
    _check(st, "bsr_encode")
    return {"browptr": brp, "bidx": bidx, "bvals": bvals, "wb": wb.value}


def coo_encode(nrows, ncols, rowptr, colids, fmt=FORMAT_DACOO16):
    """int32 CSR -> coordinates, entry order unchanged (host).  Returns
    (rows int32, idx) with idx the int16 offsets (DA-COO) or int32 columns;
    raises NoFit for DA-COO when the bandwidth does not fit int16."""
    c = _i32(colids)
    rp = _csr_arrays(nrows, rowptr, c)
    if fmt not in (FORMAT_DACOO16, FORMAT_COO32):
        raise DamnError(-1, "coo_encode: not a coordinate format")
    nnz = int(rp[nrows])
    rows = np.empty(nnz, dtype=np.int32)
    idx = np.empty(nnz, dtype=FORMATS[fmt][0])
    w = C.c_int32()
    st = lib.damn_coo_encode(int(fmt), nrows, ncols, _ptr(rp, C.c_int32), _ptr(c, C.c_int32),
                             _ptr(rows, C.c_int32), idx.ctypes.data_as(C.c_void_p), C.byref(w))
    if st == -3:
        raise NoFit(w.value)
    _check(st, "coo_encode")
    return rows, idx


def store_values(vals, dtype):
    """Values rounded to dtype (F64/F32/F16) as the library stores them
    (host).  Raises NoFit on overflow."""
    v = np.ascontiguousarray(vals)
    src = {np.dtype(np.float64): F64, np.dtype(np.float32): F32,
           np.dtype(np.float16): F16}.get(v.dtype)
    if src is None:
        v = v.astype(np.float64)
        src = F64
    out = np.empty(v.shape, dtype=VALUE_DTYPES[dtype])
    st = lib.damn_store_values(v.size, v.ctypes.data_as(C.c_void_p), src, int(dtype),
                               out.ctypes.data_as(C.c_void_p))
    if st == -3:
        raise NoFit(None, bits=8 * out.itemsize)
    _check(st, "store_values")
    return out


# ---------------------------------------------------------------------------
# device side
# ---------------------------------------------------------------------------

def _stream_ptr(stream):
    import torch

    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def _dev_ptr(t, dtype, numel, name):
    import torch

    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a tensor on a HIP device")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements, got {t.numel()}")
    return C.c_void_p(t.data_ptr())


class Matrix:
    """A device matrix in one cell of the storage grid of Fig. 3 (DA-CSR
    int16 or int8 offsets, CSR int32 or int16 columns; float64, float32 or
    float16 values) owned by the library."""

    def __init__(self, handle, nrows, ncols, nnz, fmt, dtype):
        self._h = handle
        self.nrows, self.ncols, self.nnz = nrows, ncols, nnz
        self.format, self.dtype = fmt, dtype
        self.block = 1

    # construction -----------------------------------------------------------
    @classmethod
    def create(cls, nrows, ncols, rowptr, off, vals, store=F64, stream=None):
        """Upload DA-CSR (int16 offsets) from host arrays."""
        o = np.ascontiguousarray(off, dtype=np.int16)
        v = np.ascontiguousarray(vals)
        rp = _csr_arrays(nrows, rowptr, o, v)
        vd = F32 if v.dtype == np.float32 else F64
        v = v.astype(np.float64 if vd == F64 else np.float32, copy=False)
        h = C.c_void_p()
        _check(lib.damn_create(C.byref(h), nrows, ncols, _ptr(rp, C.c_int32), _ptr(o, C.c_int16),
                               v.ctypes.data_as(C.c_void_p), vd, store, _stream_ptr(stream)),
               "create")
        return cls(h, nrows, ncols, int(rp[nrows]), FORMAT_DA16, store)

    @classmethod
    def create_format(cls, fmt, nrows, ncols, rowptr, idx, vals, store=F64, stream=None):
        """Upload any format of the grid: idx as encode_index returns it,
        vals float64/float32/float16 (rounded to `store` by the library)."""
        if fmt not in FORMATS:
            raise DamnError(-1, "create_format: unknown format")
        ix = np.ascontiguousarray(idx, dtype=FORMATS[fmt][0])
        v = np.ascontiguousarray(vals)
        vd = {np.dtype(np.float64): F64, np.dtype(np.float32): F32,
              np.dtype(np.float16): F16}.get(v.dtype)
        if vd is None:
            v, vd = v.astype(np.float64), F64
        rp = _csr_arrays(nrows, rowptr, ix, v)
        h = C.c_void_p()
        _check(lib.damn_create_format(C.byref(h), int(fmt), nrows, ncols, _ptr(rp, C.c_int32),
                                      ix.ctypes.data_as(C.c_void_p), v.ctypes.data_as(C.c_void_p),
                                      vd, int(store), _stream_ptr(stream)), "create_format")
        return cls(h, nrows, ncols, int(rp[nrows]), fmt, store)

    @classmethod
    def bsr_create(cls, fmt, nbrows, nbcols, b, browptr, bidx, bvals, store=F64, stream=None):
        """Upload BSR (FORMAT_BSR32) or DA-BSR (FORMAT_DABSR16) with b x b
        blocks; bvals has nnzb*b*b values (float64 or float32)."""
        if fmt not in (FORMAT_DABSR16, FORMAT_BSR32):
            raise DamnError(-1, "bsr_create: not a block format")
        ix = np.ascontiguousarray(bidx, dtype=FORMATS[fmt][0])
        v = np.ascontiguousarray(bvals).reshape(-1)
        vd = F32 if v.dtype == np.float32 else F64
        v = v.astype(np.float64 if vd == F64 else np.float32, copy=False)
        rp = _csr_arrays(nbrows, browptr, ix)
        if v.size != ix.size * b * b:
            raise DamnError(-2, "bvals must hold nnzb*b*b values")
        h = C.c_void_p()
        _check(lib.damn_bsr_create(C.byref(h), int(fmt), nbrows, nbcols, int(b),
                                   _ptr(rp, C.c_int32), ix.ctypes.data_as(C.c_void_p),
                                   v.ctypes.data_as(C.c_void_p), vd, int(store),
                                   _stream_ptr(stream)), "bsr_create")
        M = cls(h, nbrows * b, nbcols * b, int(rp[nbrows]), fmt, store)
        M.block = b
        return M

    @classmethod
    def coo_create(cls, fmt, nrows, ncols, rows, idx, vals, store=F64, stream=None):
        """Upload coordinates (FORMAT_DACOO16 or FORMAT_COO32), entries in row
        order; vals float64 or float32."""
        if fmt not in (FORMAT_DACOO16, FORMAT_COO32):
            raise DamnError(-1, "coo_create: not a coordinate format")
        r = _i32(rows)
        ix = np.ascontiguousarray(idx, dtype=FORMATS[fmt][0])
        v = np.ascontiguousarray(vals)
        vd = F32 if v.dtype == np.float32 else F64
        v = v.astype(np.float64 if vd == F64 else np.float32, copy=False)
        if not (r.size == ix.size == v.size):
            raise DamnError(-2, "rows, idx and vals must have the same length")
        h = C.c_void_p()
        _check(lib.damn_coo_create(C.byref(h), int(fmt), nrows, ncols, r.size,
                                   _ptr(r, C.c_int32), ix.ctypes.data_as(C.c_void_p),
                                   v.ctypes.data_as(C.c_void_p), vd, int(store),
                                   _stream_ptr(stream)), "coo_create")
        return cls(h, nrows, ncols, int(r.size), fmt, store)

    @classmethod
    def csr_create(cls, nrows, ncols, rowptr, colids, vals, store=F64, stream=None):
        """Upload plain CSR (int32 columns) from host arrays."""
        c = _i32(colids)
        v = np.ascontiguousarray(vals)
        rp = _csr_arrays(nrows, rowptr, c, v)
        vd = F32 if v.dtype == np.float32 else F64
        v = v.astype(np.float64 if vd == F64 else np.float32, copy=False)
        h = C.c_void_p()
        _check(lib.damn_csr_create(C.byref(h), nrows, ncols, _ptr(rp, C.c_int32),
                                   _ptr(c, C.c_int32), v.ctypes.data_as(C.c_void_p), vd, store,
                                   _stream_ptr(stream)), "csr_create")
        return cls(h, nrows, ncols, int(rp[nrows]), FORMAT_CSR32, store)

    def destroy(self):
        if self._h is not None and self._h.value:
            _check(lib.damn_destroy(self._h), "destroy")
        self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    @property
    def torch_dtype(self):
        import torch

        return torch.float64 if self.dtype == F64 else torch.float32

    # products ---------------------------------------------------------------
    def spmv(self, x, y, alpha=1.0, beta=0.0, stream=None):
        """y <- alpha*A*x + beta*y (DA-CSR handle)."""
        dt = self.torch_dtype
        _check(lib.damn_spmv(self._h, _dev_ptr(x, dt, self.ncols, "x"),
                             _dev_ptr(y, dt, self.nrows, "y"), float(alpha), float(beta),
                             _stream_ptr(stream)), "spmv")

    def csr_spmv(self, x, y, alpha=1.0, beta=0.0, stream=None):
        """y <- alpha*A*x + beta*y (CSR handle)."""
        dt = self.torch_dtype
        _check(lib.damn_csr_spmv(self._h, _dev_ptr(x, dt, self.ncols, "x"),
                                 _dev_ptr(y, dt, self.nrows, "y"), float(alpha), float(beta),
                                 _stream_ptr(stream)), "csr_spmv")

    @property
    def is_da(self):
        return FORMATS[self.format][1]

    @property
    def takes_paired(self):
        """Whether the stream variant's paired gathers apply (unroll 2):
        every scalar cell (DA16, DA8, CSR32, CSR16, any value type)."""
        return (self.format in (FORMAT_DA16, FORMAT_CSR32, FORMAT_DA8, FORMAT_CSR16)
                and self.block == 1)

    def apply(self, x, y, alpha=1.0, beta=0.0, stream=None):
        """spmv or csr_spmv, whichever matches the handle's format."""
        f = self.spmv if self.is_da else self.csr_spmv
        f(x, y, alpha, beta, stream)

    def spmm(self, X, Y, alpha=1.0, beta=0.0, stream=None):
        """Y <- alpha*A*X + beta*Y; X (ncols, nrhs), Y (nrows, nrhs) row-major."""
        import torch

        if X.dim() != 2 or Y.dim() != 2 or X.shape[1] != Y.shape[1]:
            raise ValueError("X and Y must be 2-D with the same number of columns")
        nrhs = int(X.shape[1])
        _check(lib.damn_spmm(self._h, _dev_ptr(X, torch.float64, self.ncols * nrhs, "X"),
                             _dev_ptr(Y, torch.float64, self.nrows * nrhs, "Y"), nrhs,
                             float(alpha), float(beta), _stream_ptr(stream)), "spmm")

    # configuration ----------------------------------------------------------
    def set_config(self, variant=VAR_VECTOR, lanes=8, unroll=1, tile=2048, cache=0):
        cfg = _lib_config(variant, lanes, unroll, tile, cache)
        _check(lib.damn_set_config(self._h, C.addressof(cfg)), "set_config")

    def get_config(self):
        cfg = _Config()
        _check(lib.damn_get_config(self._h, C.addressof(cfg)), "get_config")
        return {"variant": cfg.variant, "lanes": cfg.lanes, "unroll": cfg.unroll,
                "tile": cfg.tile, "cache": cfg.cache}


CACHE_NT, CACHE_PLAIN = 0, 1


class _Config(C.Structure):
    _fields_ = [("variant", C.c_int32), ("lanes", C.c_int32), ("unroll", C.c_int32),
                ("tile", C.c_int32), ("cache", C.c_int32)]


def _lib_config(variant, lanes, unroll, tile, cache=0):
    return _Config(int(variant), int(lanes), int(unroll), int(tile), int(cache))


class _CgOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("inner_tol", C.c_double), ("max_iter", C.c_int32),
                ("max_outer", C.c_int32), ("check_every", C.c_int32)]


class _CgInfo(C.Structure):
    _fields_ = [("iters", C.c_int32), ("outer", C.c_int32), ("converged", C.c_int32),
                ("rel_res", C.c_double)]


def cg(A64, b, x, A32=None, tol=1e-10, inner_tol=1e-5, max_iter=20000, max_outer=50,
       check_every=16, stream=None):
    """Solve A x = b on the device (float64 CG, or mixed precision when A32,
    the float32-valued copy, is given).  b, x: float64 device vectors.
    Returns dict(iters, outer, converged, rel_res); raises DamnError on
    breakdown or invalid input (not on reaching the iteration limit)."""
    import torch

    n = A64.nrows
    opts = _CgOpts(float(tol), float(inner_tol), int(max_iter), int(max_outer),
                   int(check_every))
    info = _CgInfo()
    st = lib.damn_cg(A64.handle, None if A32 is None else A32.handle,
                     _dev_ptr(b, torch.float64, n, "b"), _dev_ptr(x, torch.float64, n, "x"),
                     C.addressof(opts), C.addressof(info), _stream_ptr(stream))
    if st not in (0, -7):
        raise DamnError(st, "cg")
    return {"iters": info.iters, "outer": info.outer, "converged": bool(info.converged),
            "rel_res": info.rel_res}


class Batch:
    """Many DA-CSR products in one persistent, graph-captured launch.
    mats: float64 DA-CSR Matrix objects; Xs/Ys: float64 device tensors of
    shape (ncols, nrhs) / (nrows, nrhs); the tensors and matrices must
    outlive the batch."""

    def __init__(self, mats, Xs, Ys, alpha=1.0, beta=0.0, workgroups=0, stream=None):
        import torch

        count = len(mats)
        if len(Xs) != count or len(Ys) != count:
            raise ValueError("one X and one Y per matrix")
        nrhs = np.array([int(X.shape[1]) for X in Xs], dtype=np.int32)
        hs = (C.c_void_p * max(count, 1))(*[m.handle for m in mats])
        xp = (C.c_void_p * max(count, 1))()
        yp = (C.c_void_p * max(count, 1))()
        for i, (m, X, Y) in enumerate(zip(mats, Xs, Ys)):
            if X.dim() != 2 or Y.dim() != 2 or Y.shape[1] != X.shape[1]:
                raise ValueError("X and Y must be 2-D with the same number of columns")
            xp[i] = _dev_ptr(X, torch.float64, m.ncols * int(nrhs[i]), "X")
            yp[i] = _dev_ptr(Y, torch.float64, m.nrows * int(nrhs[i]), "Y")
        h = C.c_void_p()
        _check(lib.damn_batch_create(C.byref(h), count, C.cast(hs, C.c_void_p),
                                     nrhs.ctypes.data_as(C.c_void_p), C.cast(xp, C.c_void_p),
                                     C.cast(yp, C.c_void_p), float(alpha), float(beta),
                                     int(workgroups), _stream_ptr(stream)), "batch_create")
        self._h = h
        self._keep = (mats, Xs, Ys)

    def run(self, use_graph=True, stream=None):
        _check(lib.damn_batch_run(self._h, int(bool(use_graph)), _stream_ptr(stream)),
               "batch_run")

    def info(self):
        nt, wg, mb = C.c_int64(), C.c_int32(), C.c_double()
        _check(lib.damn_batch_info(self._h, C.byref(nt), C.byref(wg), C.byref(mb)), "batch_info")
        return {"ntiles": nt.value, "workgroups": wg.value, "model_bytes": mb.value}

    def destroy(self):
        if self._h is not None and self._h.value:
            _check(lib.damn_batch_destroy(self._h), "batch_destroy")
        self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


NFEAT, NCLASS, MLP_NPARAMS = 16, 70, 9830
CLASS_SPMM = 63  # first SpMM class; 0..62 are single-vector products


def features(nrows, ncols, rowptr, colids, nrhs):
    """The 16 sparsity features of an int32 CSR matrix (host), float32."""
    c = _i32(colids)
    rp = _csr_arrays(nrows, rowptr, c)
    f = np.empty(NFEAT, dtype=np.float32)
    _check(lib.damn_features(nrows, ncols, _ptr(rp, C.c_int32), _ptr(c, C.c_int32), int(nrhs),
                             f.ctypes.data_as(C.c_void_p)), "features")
    return f


def class_config(cls):
    """(variant, lanes, unroll, tile, spmm) of selector class cls."""
    cfg = _Config()
    mm = C.c_int32()
    _check(lib.damn_class_config(int(cls), C.addressof(cfg), C.byref(mm)), "class_config")
    return cfg.variant, cfg.lanes, cfg.unroll, cfg.tile, bool(mm.value)


def autotune(mat, nrhs, X, Y, reps=3, stream=None):
    """Time every applicable class on the device and set the fastest on mat.
    Returns float32 seconds per launch for the NCLASS classes (+inf where a
    class does not apply)."""
    import torch

    if nrhs == 1:
        dt = mat.torch_dtype
        xp = _dev_ptr(X, dt, mat.ncols, "x")
        yp = _dev_ptr(Y, dt, mat.nrows, "y")
    else:
        xp = _dev_ptr(X, torch.float64, mat.ncols * nrhs, "X")
        yp = _dev_ptr(Y, torch.float64, mat.nrows * nrhs, "Y")
    t = np.empty(NCLASS, dtype=np.float32)
    _check(lib.damn_autotune(mat.handle, int(nrhs), xp, yp, int(reps), t.ctypes.data_as(C.c_void_p),
                             _stream_ptr(stream)), "autotune")
    return t


class Mlp:
    """The selector network on the device."""

    def __init__(self, params=None, seed=0):
        h = C.c_void_p()
        p = None
        if params is not None:
            p = np.ascontiguousarray(params, dtype=np.float32)
            if p.shape != (MLP_NPARAMS,):
                raise ValueError(f"params must have {MLP_NPARAMS} floats")
        _check(lib.damn_mlp_create(C.byref(h), None if p is None else p.ctypes.data_as(C.c_void_p),
                                   C.c_uint64(seed)), "mlp_create")
        self._h = h

    def params(self):
        out = np.empty(MLP_NPARAMS, dtype=np.float32)
        _check(lib.damn_mlp_get_params(self._h, out.ctypes.data_as(C.c_void_p)), "mlp_get_params")
        return out

    def grad(self, feats, targets, stream=None):
        F = np.ascontiguousarray(feats, dtype=np.float32)
        Q = np.ascontiguousarray(targets, dtype=np.float32)
        B = F.shape[0]
        if F.shape != (B, NFEAT) or Q.shape != (B, NCLASS):
            raise ValueError(f"feats (B, 16) and targets (B, {NCLASS})")
        loss = C.c_float()
        g = np.empty(MLP_NPARAMS, dtype=np.float32)
        _check(lib.damn_mlp_grad(self._h, B, F.ctypes.data_as(C.c_void_p),
                                 Q.ctypes.data_as(C.c_void_p), C.byref(loss),
                                 g.ctypes.data_as(C.c_void_p), _stream_ptr(stream)), "mlp_grad")
        return loss.value, g

    def train(self, feats, times, epochs=200, batch=256, lr=3e-3, tau=0.05, seed=0,
              stream=None):
        F = np.ascontiguousarray(feats, dtype=np.float32)
        T = np.ascontiguousarray(times, dtype=np.float32)
        N = F.shape[0]
        if F.shape != (N, NFEAT) or T.shape != (N, NCLASS):
            raise ValueError(f"feats (N, 16) and times (N, {NCLASS})")
        losses = np.empty(epochs, dtype=np.float32)
        _check(lib.damn_mlp_train(self._h, N, F.ctypes.data_as(C.c_void_p),
                                  T.ctypes.data_as(C.c_void_p), int(epochs), int(batch),
                                  C.c_float(lr), C.c_float(tau), C.c_uint64(seed),
                                  losses.ctypes.data_as(C.c_void_p), _stream_ptr(stream)),
               "mlp_train")
        return losses

    def select(self, feats, stream=None, with_prob=False):
        """Most probable applicable class per feature row; with_prob also
        returns the probability the network gives it."""
        F = np.ascontiguousarray(np.atleast_2d(feats), dtype=np.float32)
        out = np.empty(F.shape[0], dtype=np.int32)
        prob = np.empty(F.shape[0], dtype=np.float32)
        _check(lib.damn_select_prob(self._h, F.shape[0], F.ctypes.data_as(C.c_void_p),
                                    out.ctypes.data_as(C.c_void_p),
                                    prob.ctypes.data_as(C.c_void_p) if with_prob else None,
                                    _stream_ptr(stream)), "select")
        return (out, prob) if with_prob else out

    def select_noalloc(self, feats, stream=None, with_prob=False):
        """select() through damn_select_noalloc: the same results, staged in
        the library's fixed device array (at most SELECT_NOALLOC_MAX_ROWS
        rows), with no device allocation."""
        F = np.ascontiguousarray(np.atleast_2d(feats), dtype=np.float32)
        out = np.empty(F.shape[0], dtype=np.int32)
        prob = np.empty(F.shape[0], dtype=np.float32)
        _check(lib.damn_select_noalloc(self._h, F.shape[0], F.ctypes.data_as(C.c_void_p),
                                       out.ctypes.data_as(C.c_void_p),
                                       prob.ctypes.data_as(C.c_void_p) if with_prob else None,
                                       _stream_ptr(stream)), "select_noalloc")
        return (out, prob) if with_prob else out

    def destroy(self):
        if self._h is not None and self._h.value:
            _check(lib.damn_mlp_destroy(self._h), "mlp_destroy")
        self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


READ_NT, READ_PLAIN, READ_LDS_NT, READ_LDS_PLAIN = 0, 1, 2, 3


def stream_read(src, sink, mode=READ_NT, tile_bytes=8192, stream=None, passes=1):
    """Streaming-read probe over a contiguous device tensor (bytes % 16 == 0)
    along read path `mode` (READ_*; the LDS modes in tiles of tile_bytes),
    `passes` times over in one launch; sink: float64 device tensor with at
    least 65536 entries."""
    import torch

    if not src.is_cuda or not src.is_contiguous():
        raise ValueError("src must be a contiguous device tensor")
    nbytes = src.numel() * src.element_size()
    _dev_ptr(sink, torch.float64, sink.numel(), "sink")
    if sink.numel() < 65536:
        raise ValueError("sink needs 65536 entries")
    _check(lib.damn_stream_read(C.c_void_p(src.data_ptr()), C.c_size_t(nbytes), int(passes),
                                C.c_void_p(sink.data_ptr()), int(mode), int(tile_bytes),
                                _stream_ptr(stream)), "stream_read")


def gather_read(x, sink, rows, per_row, halfwidth=0, offs=None, stream=None):
    """Gather probe: rows * per_row reads of the float64 device vector x,
    row r's at r + offs[k] (offs: int32 device tensor of per_row DA
    offsets) or, without offs, scattered within +-halfwidth of r; sink:
    float64 device tensor with at least 65536 entries."""
    import torch

    _dev_ptr(x, torch.float64, x.numel(), "x")
    _dev_ptr(sink, torch.float64, sink.numel(), "sink")
    if sink.numel() < 65536:
        raise ValueError("sink needs 65536 entries")
    op = None
    if offs is not None:
        op = _dev_ptr(offs, torch.int32, int(per_row), "offs")
    _check(lib.damn_gather_read(C.c_void_p(x.data_ptr()), int(x.numel()), int(rows),
                                int(per_row), int(halfwidth), op, C.c_void_p(sink.data_ptr()),
                                _stream_ptr(stream)), "gather_read")


def stream_copy(src, dst, stream=None):
    """Copy probe between two contiguous device tensors of equal byte size
    (a multiple of 16)."""
    nbytes = src.numel() * src.element_size()
    if not (src.is_cuda and dst.is_cuda and src.is_contiguous() and dst.is_contiguous()):
        raise ValueError("src and dst must be contiguous device tensors")
    if dst.numel() * dst.element_size() != nbytes:
        raise ValueError("src and dst sizes differ")
    _check(lib.damn_stream_copy(C.c_void_p(src.data_ptr()), C.c_void_p(dst.data_ptr()),
                                C.c_size_t(nbytes), _stream_ptr(stream)), "stream_copy")


def library_path() -> str:
    return os.path.abspath(LIB_PATH)
