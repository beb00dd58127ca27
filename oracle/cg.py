"""Conjugate gradients, float64 and mixed precision.

The paper motivates DA storage for iterative solvers (Sec. 3 footnote) and
for multi-precision algorithms (the remark after Fig. 3: halving the scalar
size of a DA-CSR int16 matrix saves 5/3x traffic against 3/2x for CSR int32).
It gives no solver, so the schemes below are the textbook ones:

cg_fp64 -- Hestenes-Stiefel CG from x0 = 0, stopping when the recursively
           updated residual satisfies ||r|| <= tol * ||b||; the true residual
           b - A x is returned beside it.
cg_mixed -- iterative refinement: the outer loop keeps x, b and the residual
           r = b - A x in float64 (float64 matrix); each correction solves
           A d = r approximately with CG on the float32 matrix, the Krylov
           vectors held in float32 and dot products accumulated in float64,
           to a relative residual of max(inner_tol, tol*||b|| / (2 ||r||)):
           a step never solves further than the outer target needs, so the
           last step stops as soon as the outer residual will meet tol.  The
           right-hand side of the inner solve is r scaled to unit norm (and
           the correction scaled back), so small late residuals stay in
           float32 range.

`matvec64(v)` and `matvec32(v)` are caller-supplied products (the oracle's
spmv on the float64 values and on the float32-rounded values).
"""

from __future__ import annotations

import numpy as np


def cg_fp64(matvec64, b, tol=1e-10, max_iter=10000):
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b)
    r = b.copy()
    p = r.copy()
    rho = float(r @ r)
    bnorm = float(np.sqrt(b @ b))
    it = 0
    converged = np.sqrt(rho) <= tol * bnorm
    while not converged and it < max_iter:
        q = matvec64(p)
        pq = float(p @ q)
        if pq <= 0:
            raise ArithmeticError("p.Ap <= 0: matrix is not positive definite")
        a = rho / pq
        x += a * p
        r -= a * q
        rho_new = float(r @ r)
        it += 1
        if np.sqrt(rho_new) <= tol * bnorm:
            converged = True
            break
        p = r + (rho_new / rho) * p
        rho = rho_new
    true_res = float(np.linalg.norm(b - matvec64(x)))
    return {"x": x, "iters": it, "converged": converged,
            "true_rel_res": true_res / bnorm if bnorm > 0 else 0.0}


def _inner_cg32(matvec32, rhs32, inner_tol, max_iter):
    """CG on the float32 matrix; vectors float32, dots float64."""
    f32 = np.float32
    d = np.zeros_like(rhs32)
    r = rhs32.copy()
    p = r.copy()
    rho = float(np.dot(r.astype(np.float64), r.astype(np.float64)))
    stop = inner_tol * np.sqrt(rho)
    it = 0
    while np.sqrt(rho) > stop and it < max_iter:
        q = matvec32(p)
        pq = float(np.dot(p.astype(np.float64), q.astype(np.float64)))
        if pq <= 0:
            raise ArithmeticError("p.Ap <= 0 in the inner solve")
        a = rho / pq
        d = (d + a * p.astype(np.float64)).astype(f32)
        r = (r - a * q.astype(np.float64)).astype(f32)
        rho_new = float(np.dot(r.astype(np.float64), r.astype(np.float64)))
        p = (r + (rho_new / rho) * p.astype(np.float64)).astype(f32)
        rho = rho_new
        it += 1
    return d, it


def cg_mixed(matvec64, matvec32, b, tol=1e-10, inner_tol=1e-5, max_outer=50, max_inner=10000):
    b = np.asarray(b, dtype=np.float64)
    bnorm = float(np.sqrt(b @ b))
    x = np.zeros_like(b)
    r = b.copy()
    outer = inner_total = 0
    rnorm = bnorm
    converged = rnorm <= tol * bnorm
    while not converged and outer < max_outer:
        rhs = (r / rnorm).astype(np.float32)
        target = min(0.5, max(inner_tol, 0.5 * tol * bnorm / rnorm))
        d, k = _inner_cg32(matvec32, rhs, target, max_inner)
        inner_total += k
        x += rnorm * d.astype(np.float64)
        r = b - matvec64(x)
        rnorm = float(np.sqrt(r @ r))
        outer += 1
        converged = rnorm <= tol * bnorm
    return {"x": x, "outer": outer, "inner_iters": inner_total, "converged": converged,
            "true_rel_res": rnorm / bnorm if bnorm > 0 else 0.0}
