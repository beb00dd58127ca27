"""Helpers for GPU parity tests: device transfer and the rounding-error bound.

Bound (generalising |y - y_oracle| <= 4 rowlen 2^-53 sum|a_ij x_j| to alpha
and beta):  |y_r - y_r^oracle| <= 4 max(rowlen_r, 1) u (|alpha| S_r + |beta y0_r|)
with S_r = sum_{i in row r} |a_i x_{c_i}|, u = 2^-53 for float64 and 2^-24
for float32 (the oracle then runs on the float32-rounded a and x).
"""

import numpy as np
import pytest

from oracle.spmv import abs_products

U64 = 2.0 ** -53
U32 = 2.0 ** -24


def torch_or_skip():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch


def dev(a, dtype=None):
    import torch

    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to("cuda")


def host(t):
    import torch

    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def error_bound(nrows, rowptr, cols, vals, x, alpha, beta, y0, u):
    S = abs_products(nrows, rowptr, cols, vals, x)
    rl = np.maximum(np.diff(np.asarray(rowptr, dtype=np.int64)), 1)
    b = abs(alpha) * S
    if beta != 0:
        b = b + np.abs(beta * np.asarray(y0, dtype=np.float64))
    return 4.0 * rl * u * b


def assert_within(y, y_ref, bound, what=""):
    y = np.asarray(y, dtype=np.float64)
    err = np.abs(y - y_ref)
    bad = np.flatnonzero(~(err <= bound))
    if bad.size:
        i = bad[0]
        raise AssertionError(
            f"{what}: {bad.size} rows outside the bound; first row {i}: y={y[i]!r} "
            f"oracle={y_ref[i]!r} err={err[i]:.3e} bound={bound[i]:.3e}")
