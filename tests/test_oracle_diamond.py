"""Pins of the oracle's diamond iteration space (Section 3: do_diamond, cells
(i-1, j) and (i, j-1) processed before (i, j); 2D).

* With a = b = 1, c = 0 and seed 1 the recurrence counts lattice paths from
  the boundary: out(i, j) = C(i+j+2, i+1), exactly.
* The transpose of the inputs gives the transposed output with a and b
  swapped (the two predecessors play symmetric roles).
* One lexicographic SOR sweep equals its matrix form, solved independently:
  with A = D - L - U the 5-point matrix in row-major order,
  (D/w - L) u' = ((1/w - 1) D + U) u - h^2 f (+ boundary terms, bcv = 0).
* The exact discrete solution is a fixed point, and the asymptotic rate of
  lexicographic Gauss-Seidel is rho_J^2 with rho_J = cos(pi h) on the square
  (the same as red-black: both orderings are consistent).
"""
import math

import numpy as np
import pytest

import oracle


def test_lattice_path_counts():
    shape = (1, 9, 11)
    out = oracle.diamond_recur(np.ones(shape), np.ones(shape), np.zeros(shape), seed=1.0)
    for j in range(shape[1]):
        for i in range(shape[2]):
            assert out[0, j, i] == math.comb(i + j + 2, i + 1)


def test_transpose_swaps_predecessors():
    g = np.random.default_rng(60)
    shape = (2, 7, 9)
    a, b, c = g.uniform(-0.7, 0.7, shape), g.uniform(-0.7, 0.7, shape), g.standard_normal(shape)
    out = oracle.diamond_recur(a, b, c, seed=0.2)
    t = lambda x: np.ascontiguousarray(x.transpose(0, 2, 1))
    outt = oracle.diamond_recur(t(b), t(a), t(c), seed=0.2)
    np.testing.assert_allclose(t(out), outt, rtol=0, atol=1e-13)


def _five_point(ny, nx):
    n = nx * ny
    A = np.zeros((n, n))
    for j in range(ny):
        for i in range(nx):
            p = j * nx + i
            A[p, p] = 4.0
            if i > 0:
                A[p, p - 1] = -1.0
            if i + 1 < nx:
                A[p, p + 1] = -1.0
            if j > 0:
                A[p, p - nx] = -1.0
            if j + 1 < ny:
                A[p, p + nx] = -1.0
    return A


@pytest.mark.parametrize("shape", [(5, 6), (1, 7), (4, 1), (6, 6)])
@pytest.mark.parametrize("omega", [1.0, 1.45])
def test_sor_sweep_equals_matrix_form(shape, omega):
    g = np.random.default_rng(61)
    ny, nx = shape
    u = g.standard_normal((1, ny, nx))
    f = g.standard_normal((1, ny, nx))
    h2 = 0.2
    A = _five_point(ny, nx)
    D = np.diag(np.diag(A))
    L = -np.tril(A, -1)
    U = -np.triu(A, 1)
    rhs = ((1 / omega - 1) * D + U) @ u.ravel() - h2 * f.ravel()
    ref = np.linalg.solve(D / omega - L, rhs)
    got = oracle.gs2d_sweep(u, f, omega, h2)
    np.testing.assert_allclose(got.ravel(), ref, rtol=0, atol=1e-12)


def test_exact_solution_fixed_point_and_rate():
    n = 16
    h = 1.0 / (n + 1)
    x = np.arange(1, n + 1) * h
    ustar = np.sin(math.pi * x)[None, :, None] * np.sin(2 * math.pi * x)[None, None, :]
    lam = (2 / h ** 2) * (math.cos(math.pi * h) + math.cos(2 * math.pi * h) - 2)
    f = lam * ustar  # the 5-point Laplacian of a sine mode is lam times the mode
    got = oracle.gs2d_sweep(ustar, f, 1.0, h * h)
    np.testing.assert_allclose(got, ustar, rtol=0, atol=1e-13)
    # asymptotic contraction of lexicographic Gauss-Seidel (f = 0)
    u = np.random.default_rng(62).standard_normal((1, n, n))
    norms = []
    for _ in range(400):
        u = oracle.gs2d_sweep(u, None, 1.0, 1.0)
        norms.append(math.sqrt(oracle.sumsq(u)))
    rho_j = math.cos(math.pi * h)
    assert abs(norms[-1] / norms[-2] - rho_j ** 2) <= 3e-3 * rho_j ** 2
