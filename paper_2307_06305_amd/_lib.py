"""Loading libdamn.so and declaring its C signatures (ctypes)."""

from __future__ import annotations

import ctypes as C
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libdamn.so")


class DamnError(RuntimeError):
    def __init__(self, code, what=""):
        self.code = code
        try:
            msg = lib.damn_status_string(int(code)).decode()
        except Exception:  # library not loaded yet
            msg = f"status {code}"
        super().__init__(f"{what}: {msg} ({code})")


class NoFit(Exception):
    """An index or value does not fit its storage type: for 16-bit DA
    offsets, bandwidth >= 2^15 also after reordering.  .w is the bandwidth
    (or largest column) found, None for a value overflow."""

    def __init__(self, w, what="bandwidth", bits=16):
        if w is None:
            super().__init__(f"a value overflows float{bits}")
        else:
            super().__init__(f"{what} {w} does not fit a {bits}-bit index")
        self.w = w


def _load():
    # torch ships its own HIP runtime with the same soname as ROCm's
    # (libamdhip64.so.7).  Loading torch first makes libdamn.so bind to that
    # runtime, so device pointers and streams from torch are valid in the
    # library; loading the library first would put two HIP runtimes in the
    # process.
    import torch  # noqa: F401

    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with `python -m paper_2307_06305_amd.build`")
    return C.CDLL(LIB_PATH)


_i32, _i64, _f64, _vp = C.c_int32, C.c_int64, C.c_double, C.c_void_p
_pi32, _pi16, _pf64 = C.POINTER(C.c_int32), C.POINTER(C.c_int16), C.POINTER(C.c_double)
_pi64 = C.POINTER(C.c_int64)

_SIGS = {
    "damn_status_string": (C.c_char_p, [C.c_int]),
    "damn_version": (C.c_char_p, []),
    "damn_fit_check": (C.c_int, [_i32, _i32, _pi32, _pi32, _pi32, _pi32, _pi32, _pi32]),
    "damn_rcm": (C.c_int, [_i32, _pi32, _pi32, _pi32]),
    "damn_refine_bandwidth": (C.c_int, [_i32, _pi32, _pi32, _pi32, _i32, _i32, _pi32]),
    "damn_encode": (C.c_int, [_i32, _i32, _pi32, _pi32, _pf64, _i32, _pi32, _pi16, _pf64, _pi32,
                              _pi32, _pi32]),
    "damn_create": (C.c_int, [C.POINTER(_vp), _i32, _i32, _pi32, _pi16, _vp, _i32, _i32, _vp]),
    "damn_csr_create": (C.c_int, [C.POINTER(_vp), _i32, _i32, _pi32, _pi32, _vp, _i32, _i32,
                                  _vp]),
    "damn_encode_index": (C.c_int, [_i32, _i32, _i32, _pi32, _pi32, _vp, _pi32]),
    "damn_store_values": (C.c_int, [_i64, _vp, _i32, _i32, _vp]),
    "damn_create_format": (C.c_int, [C.POINTER(_vp), _i32, _i32, _i32, _pi32, _vp, _vp, _i32,
                                     _i32, _vp]),
    "damn_bsr_count": (C.c_int, [_i32, _i32, _pi32, _pi32, _i32, _pi64, _pi32]),
    "damn_bsr_encode": (C.c_int, [_i32, _i32, _pi32, _pi32, _pf64, _i32, _i32, _pi32, _vp,
                                  _pf64]),
    "damn_bsr_create": (C.c_int, [C.POINTER(_vp), _i32, _i32, _i32, _i32, _pi32, _vp, _vp, _i32,
                                  _i32, _vp]),
    "damn_coo_encode": (C.c_int, [_i32, _i32, _i32, _pi32, _pi32, _pi32, _vp, _pi32]),
    "damn_coo_create": (C.c_int, [C.POINTER(_vp), _i32, _i32, _i32, _i64, _pi32, _vp, _vp, _i32,
                                  _i32, _vp]),
    "damn_destroy": (C.c_int, [_vp]),
    "damn_mat_info": (C.c_int, [_vp, _pi32, _pi32, _pi64, _pi32, _pi32]),
    "damn_spmv": (C.c_int, [_vp, _vp, _vp, _f64, _f64, _vp]),
    "damn_csr_spmv": (C.c_int, [_vp, _vp, _vp, _f64, _f64, _vp]),
    "damn_spmm": (C.c_int, [_vp, _vp, _vp, _i32, _f64, _f64, _vp]),
    "damn_set_config": (C.c_int, [_vp, _vp]),
    "damn_get_config": (C.c_int, [_vp, _vp]),
    "damn_stream_read": (C.c_int, [_vp, C.c_size_t, _i32, _vp, _i32, _i32, _vp]),
    "damn_stream_copy": (C.c_int, [_vp, _vp, C.c_size_t, _vp]),
    "damn_gather_read": (C.c_int, [_vp, _i64, _i64, _i32, _i32, _vp, _vp, _vp]),
    "damn_cg": (C.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "damn_batch_create": (C.c_int, [C.POINTER(_vp), _i32, _vp, _vp, _vp, _vp, _f64, _f64, _i32,
                                    _vp]),
    "damn_batch_run": (C.c_int, [_vp, _i32, _vp]),
    "damn_batch_info": (C.c_int, [_vp, _pi64, _pi32, _pf64]),
    "damn_batch_destroy": (C.c_int, [_vp]),
    "damn_features": (C.c_int, [_i32, _i32, _pi32, _pi32, _i32, _vp]),
    "damn_class_config": (C.c_int, [_i32, _vp, _pi32]),
    "damn_autotune": (C.c_int, [_vp, _i32, _vp, _vp, _i32, _vp, _vp]),
    "damn_mlp_create": (C.c_int, [C.POINTER(_vp), _vp, C.c_uint64]),
    "damn_mlp_get_params": (C.c_int, [_vp, _vp]),
    "damn_mlp_destroy": (C.c_int, [_vp]),
    "damn_mlp_grad": (C.c_int, [_vp, _i32, _vp, _vp, _vp, _vp, _vp]),
    "damn_mlp_train": (C.c_int, [_vp, _i32, _vp, _vp, _i32, _i32, C.c_float, C.c_float,
                                 C.c_uint64, _vp, _vp]),
    "damn_select": (C.c_int, [_vp, _i32, _vp, _vp, _vp]),
    "damn_select_prob": (C.c_int, [_vp, _i32, _vp, _vp, _vp, _vp]),
    "damn_select_noalloc": (C.c_int, [_vp, _i32, _vp, _vp, _vp, _vp]),
}

class _Lib:
    """libdamn.so, loaded on first use (so the build step can import this
    package before the library exists); raises ImportError if it is missing."""

    def __init__(self):
        self._cdll = None

    def _get(self):
        if self._cdll is None:
            cdll = _load()
            for name, (res, args) in _SIGS.items():
                f = getattr(cdll, name)
                f.restype = res
                f.argtypes = args
            self._cdll = cdll
        return self._cdll

    def __getattr__(self, name):
        return getattr(self._get(), name)


lib = _Lib()
