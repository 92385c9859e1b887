"""Pins for the oracle's fourth-order 13-point multi-field operator.

* Closed form: with every coefficient 1 the operator is u - kappa L4 u, and L4
  is exact (equals the continuous Laplacian) on polynomials of degree <= 5.
* Textbook matrix: with every coefficient 1 the assembled matrix equals
  I - kappa (T4 (+) T4 (+) T4), T4 the 1D stencil [-1/12, 4/3, -5/2, 4/3, -1/12]
  with zero Dirichlet boundary, built with numpy.kron.
* Independent evaluator for variable coefficients (numpy.pad halos).
* The diagonal equals the assembled matrix's diagonal; the FP64 Jacobi solve
  agrees with numpy.linalg.solve on a tiny grid.
"""
import numpy as np
import pytest

import oracle
from paper_1207_1746_amd import workloads as W

KAPPA = W.VC13_KAPPA


def _ones(shp):
    return [np.ones(shp) for _ in range(10)]


def test_constant_coefficient_closed_form_on_quartic():
    n = 12
    z, y, x = np.meshgrid(*(np.arange(n, dtype=np.float64),) * 3, indexing="ij")
    u = x ** 4 - 2 * y ** 3 * z + x * y * z + 3 * z ** 5 / 64 + 5
    lap = 12 * x ** 2 - 12 * y * z + 3 * 20 * z ** 3 / 64
    out = oracle.vc13_apply(u, _ones(u.shape), KAPPA)
    inner = (slice(2, -2),) * 3
    expect = u - KAPPA * lap
    np.testing.assert_allclose(out[inner], expect[inner], rtol=1e-13, atol=1e-10)


def _T4(n):
    T = np.zeros((n, n))
    for i in range(n):
        for d, w in ((-2, -1 / 12), (-1, 4 / 3), (0, -5 / 2), (1, 4 / 3), (2, -1 / 12)):
            if 0 <= i + d < n:
                T[i, i + d] = w
    return T


def _assemble(apply, shp):
    npts = int(np.prod(shp))
    M = np.zeros((npts, npts))
    for j in range(npts):
        e = np.zeros(npts)
        e[j] = 1.0
        M[:, j] = apply(e.reshape(shp)).ravel()
    return M


def test_constant_coefficient_matrix_is_kronecker_sum():
    n = 5
    shp = (n, n, n)
    M = _assemble(lambda e: oracle.vc13_apply(e, _ones(shp), KAPPA), shp)
    T, I = _T4(n), np.eye(n)
    L = np.kron(np.kron(I, I), T) + np.kron(np.kron(I, T), I) + np.kron(np.kron(T, I), I)
    np.testing.assert_allclose(M, np.eye(n ** 3) - KAPPA * L, rtol=0, atol=1e-14)


def _independent_apply(u, c, kappa):
    p = np.pad(u, 2, mode="constant")
    nz, ny, nx = u.shape
    sh = lambda dx, dy, dz: p[2 + dz:2 + dz + nz, 2 + dy:2 + dy + ny, 2 + dx:2 + dx + nx]
    total = 0.0
    for d, e in enumerate([(1, 0, 0), (0, 1, 0), (0, 0, 1)]):
        e2 = tuple(2 * v for v in e)
        m1 = tuple(-v for v in e)
        m2 = tuple(-v for v in e2)
        near = c[1 + 2 * d] * (sh(*e) - u) + c[2 + 2 * d] * (sh(*m1) - u)
        far = c[7 + d] * (sh(*e2) + sh(*m2) - 2 * u)
        total = total + (4 / 3) * near - far / 12
    return c[0] * u - kappa * total


def test_variable_coefficients_match_padded_evaluator():
    c, _ = W.vc13_grids(9, 7, 6)
    c = [x.astype(np.float64) for x in c]
    u = W.vc13_fields(9, 7, 6, 1)[0].astype(np.float64)
    np.testing.assert_allclose(oracle.vc13_apply(u, c, KAPPA), _independent_apply(u, c, KAPPA),
                               rtol=1e-13, atol=1e-13)


def test_diag_equals_matrix_diagonal():
    shp = (3, 4, 5)
    c, _ = W.vc13_grids(5, 4, 3)
    M = _assemble(lambda e: oracle.vc13_apply(e, c, KAPPA), shp)
    np.testing.assert_allclose(oracle.vc13_diag(c, KAPPA).ravel(), np.diag(M), rtol=1e-15)


def test_jacobi_solve_matches_dense_solve():
    shp = (4, 4, 5)
    c, b = W.vc13_grids(5, 4, 4, nfields=1)
    M = _assemble(lambda e: oracle.vc13_apply(e, c, KAPPA), shp)
    exact = np.linalg.solve(M, b[0].ravel()).reshape(shp)
    x, sweeps, rel = oracle.vc13_jacobi_solve(b[0], c, KAPPA, 6 / 7, 1e-13, 5000)
    assert rel <= 1e-13
    # cond(A) is small for this diagonally dominant operator
    err = np.linalg.norm((x - exact).ravel()) / np.linalg.norm(exact.ravel())
    assert err <= 1e-13 * np.linalg.cond(M)


def test_diagonal_dominance_margin():
    # Jacobi converges: D - sum |off-diagonal| >= c0 - kappa sum_d c_{d2} / 3 > 0
    shp = (5, 5, 5)
    c, _ = W.vc13_grids(5)
    M = _assemble(lambda e: oracle.vc13_apply(e, c, KAPPA), shp)
    off = np.abs(M).sum(axis=1) - np.abs(np.diag(M))
    assert np.all(np.diag(M) - off > 0.1)


def test_residual_is_b_minus_assembled_operator():
    """r = b - A x: against the densely assembled variable-coefficient matrix
    (columns from the independent padded evaluator) on a small grid, and zero
    up to rounding at the dense solution of A x = b."""
    shp = (3, 4, 5)
    c, b = W.vc13_grids(5, 4, 3, nfields=1)
    c = [x.astype(np.float64) for x in c]
    b = b[0]
    M = _assemble(lambda e: _independent_apply(e, c, KAPPA), shp)
    x = np.random.default_rng(90).standard_normal(shp)
    r = oracle.vc13_residual(x, b, c, KAPPA)
    np.testing.assert_allclose(r.ravel(), b.ravel() - M @ x.ravel(), rtol=0, atol=1e-13)
    xs = np.linalg.solve(M, b.ravel()).reshape(shp)
    assert np.abs(oracle.vc13_residual(xs, b, c, KAPPA)).max() <= 1e-13 * np.abs(b).max()
