"""Pins of the CG oracles against a direct solve on small SPD systems."""

import numpy as np
import pytest

from oracle import cg as CG
from oracle import spmv as S
from workloads import laplace_2d_5pt, poisson_3d_7pt, uniform_vector


def _ops(A):
    v32 = A.vals.astype(np.float32)

    def mv64(v):
        return S.spmv_csr(A.nrows, A.ncols, A.rowptr, A.colids, A.vals, v)

    def mv32(v):
        return S.spmv_csr(A.nrows, A.ncols, A.rowptr, A.colids, v32, v).astype(np.float32)

    return mv64, mv32


@pytest.mark.parametrize("A", [laplace_2d_5pt(12), poisson_3d_7pt(6, 5, 7)],
                         ids=lambda A: A.name)
def test_cg_fp64_matches_direct_solve(A):
    mv64, _ = _ops(A)
    b = uniform_vector(A.nrows, 4)
    r = CG.cg_fp64(mv64, b, tol=1e-10)
    D = S.dense(A.nrows, A.ncols, A.rowptr, A.colids, A.vals)
    xs = np.linalg.solve(D, b)
    assert r["converged"] and r["true_rel_res"] <= 1.01e-10
    cond = np.linalg.cond(D)
    assert np.linalg.norm(r["x"] - xs) <= 10 * cond * 1e-10 * np.linalg.norm(xs)
    # CG on n unknowns converges in at most n steps in exact arithmetic;
    # here well before
    assert r["iters"] < A.nrows


@pytest.mark.parametrize("A", [laplace_2d_5pt(12), poisson_3d_7pt(6, 5, 7)],
                         ids=lambda A: A.name)
def test_cg_mixed_reaches_fp64_tolerance(A):
    mv64, mv32 = _ops(A)
    b = uniform_vector(A.nrows, 5)
    r = CG.cg_mixed(mv64, mv32, b, tol=1e-10, inner_tol=1e-5)
    D = S.dense(A.nrows, A.ncols, A.rowptr, A.colids, A.vals)
    xs = np.linalg.solve(D, b)
    assert r["converged"] and r["true_rel_res"] <= 1e-10
    assert np.linalg.norm(r["x"] - xs) <= 10 * np.linalg.cond(D) * 1e-10 * np.linalg.norm(xs)
    # a 1e-5 inner solve gains about five digits per refinement step
    assert 2 <= r["outer"] <= 4


def test_cg_diagonal_system_one_step():
    # A = 3 I: CG converges in one step with x = b / 3
    n = 10
    rp = np.arange(n + 1)
    c = np.arange(n)
    v = np.full(n, 3.0)

    def mv(u):
        return S.spmv_csr(n, n, rp, c, v, u)

    b = uniform_vector(n, 1)
    r = CG.cg_fp64(mv, b)
    assert r["iters"] == 1 and np.allclose(r["x"], b / 3, rtol=1e-15)


def test_cg_detects_indefinite():
    n = 4
    rp = np.arange(n + 1)
    c = np.arange(n)
    v = np.array([1.0, -1.0, 1.0, -1.0])

    def mv(u):
        return S.spmv_csr(n, n, rp, c, v, u)

    with pytest.raises(ArithmeticError):
        CG.cg_fp64(mv, np.array([0.0, 1.0, 0.0, 0.0]))


def test_cg_mixed_scaled_identity_refines_in_two_steps():
    """A = 3 I: every inner CG converges in one iteration, so the refinement
    is fixed by rounding alone.  The first correction is float32(r/|r|)/3
    scaled back by |r|: its error is float32 rounding, a relative residual
    in (0, 2^-23]; the second correction removes it to float64 level.  Two
    outer steps, one inner iteration each, x = b/3.  (Drop the |r| scaling
    of the correction, or the float64 residual between steps, and this
    fails.)"""
    n = 50
    rp = np.arange(n + 1)
    c = np.arange(n)
    v = np.full(n, 3.0)

    def mv64(u):
        return S.spmv_csr(n, n, rp, c, v, u)

    def mv32(u):
        return S.spmv_csr(n, n, rp, c, v.astype(np.float32), u).astype(np.float32)

    b = uniform_vector(n, 9) * 1e3
    one = CG.cg_mixed(mv64, mv32, b, tol=1e-10, inner_tol=1e-5, max_outer=1)
    assert one["outer"] == 1 and one["inner_iters"] == 1 and not one["converged"]
    assert 0.0 < one["true_rel_res"] <= 2.0 ** -23
    r = CG.cg_mixed(mv64, mv32, b, tol=1e-10, inner_tol=1e-5)
    assert r["converged"] and r["outer"] == 2 and r["inner_iters"] == 2
    np.testing.assert_allclose(r["x"], b / 3, rtol=1e-13)
