"""Pins for the oracle's Jacobi averaging iteration and Poisson solve (Section 5.2).

* Mode decay: a discrete Dirichlet sine mode is an eigenvector of the sweep,
  so n sweeps multiply it by (1 - omega + omega mu)^n exactly, with
  mu = (cos k pi h + cos l pi h + cos m pi h) / 3; sum of phi^2 = ((N+1)/2)^3.
* Manufactured solution: f built from the closed-form eigenvalues gives a zero
  residual for u*, and the solve reaches u* within the rtol-implied bound.
* Dense linear algebra: on tiny grids the Poisson solve agrees with
  numpy.linalg.solve on the Laplacian assembled as a Kronecker sum.
* Stopping sweep: for a single mode the residual trace is closed form, which
  predicts the first checkpoint that meets rtol.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1207_1746_amd import workloads as W


@pytest.mark.parametrize("klm,omega", [((1, 2, 3), 1.0), ((2, 1, 1), 6 / 7), ((3, 3, 2), 0.8)])
def test_mode_decay_closed_form(klm, omega):
    n = 12
    h = 1.0 / (n + 1)
    phi = W.sine_mode(n, *klm)
    mu = sum(math.cos(q * math.pi * h) for q in klm) / 3.0
    g = 1.0 - omega + omega * mu
    sweeps = 7
    u, l2upd, maxupd = oracle.jacobi_run(phi, sweeps, None, omega, h * h)
    np.testing.assert_allclose(u, g ** sweeps * phi, rtol=0, atol=1e-14)
    norm_phi = math.sqrt(((n + 1) / 2.0) ** 3)
    expect_l2 = abs(g ** sweeps - g ** (sweeps - 1)) * norm_phi
    assert abs(l2upd - expect_l2) <= 1e-12 * expect_l2
    assert abs(maxupd - abs(g ** sweeps - g ** (sweeps - 1)) * np.abs(phi).max()) <= 1e-13


def test_sine_mode_norm_closed_form():
    n = 9
    phi = W.sine_mode(n, 2, 3, 4)
    assert abs(oracle.sumsq(phi) - ((n + 1) / 2.0) ** 3) <= 1e-12 * ((n + 1) / 2.0) ** 3


def test_manufactured_residual_is_zero():
    req = W.poisson_requests(count=1, qps=float("inf"), nmin=20, nmax=20)[0]
    ustar, f = W.poisson_fields(req)
    _, _, res = oracle.wjacobi_sweep(ustar, f, 6 / 7, req.h2)
    assert np.sqrt(oracle.sumsq(res)) <= 1e-9 * np.sqrt(oracle.sumsq(f))


def _lap_matrix(n):
    """Dirichlet 7-point Laplacian (unit spacing) as a Kronecker sum, [z][y][x] order."""
    T = -2 * np.eye(n) + np.eye(n, k=1) + np.eye(n, k=-1)
    I = np.eye(n)
    return np.kron(np.kron(I, I), T) + np.kron(np.kron(I, T), I) + np.kron(np.kron(T, I), I)


def test_poisson_solve_matches_dense_solve():
    n = 5
    h2 = 1.0 / (n + 1) ** 2
    f = np.random.default_rng(5).standard_normal((n, n, n))
    A = _lap_matrix(n) / h2
    exact = np.linalg.solve(A, f.ravel()).reshape(f.shape)
    u, sweeps, rel, conv = oracle.poisson_solve(f, h2, 6 / 7, 1e-12, 4, 20000)
    assert conv
    # ||u - exact|| <= ||A^-1|| ||r|| with ||A^-1||_2 = 1 / |lambda_min|
    lam_min = abs(np.linalg.eigvalsh(A)).min()
    bound = rel * np.linalg.norm(f) / lam_min
    assert np.linalg.norm((u - exact).ravel()) <= bound * 1.01 + 1e-14


def test_jacobi_matches_dense_iteration_matrix():
    # one weighted sweep == u + omega D^-1 (f - A u) with the assembled matrix
    n = 4
    h2 = 0.3
    g = np.random.default_rng(9)
    u = g.standard_normal((n, n, n))
    f = g.standard_normal((n, n, n))
    A = _lap_matrix(n) / h2
    omega = 0.9
    D = -6.0 / h2
    expect = u.ravel() + omega * (f.ravel() - A @ u.ravel()) / D
    unew, upd, res = oracle.wjacobi_sweep(u, f, omega, h2)
    np.testing.assert_allclose(unew.ravel(), expect, rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(res.ravel(), f.ravel() - A @ u.ravel(), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(upd, unew - u, rtol=0, atol=1e-15)


def test_two_dimensional_layers_are_independent():
    g = np.random.default_rng(2)
    u = g.standard_normal((3, 6, 7))
    stacked, _, _ = oracle.wjacobi_sweep(u, None, 1.0, 1.0, ndim=2)
    for l in range(3):
        single, _, _ = oracle.wjacobi_sweep(u[l:l + 1], None, 1.0, 1.0, ndim=2)
        assert np.array_equal(stacked[l], single[0])
    # 5-point Laplacian of x^2 + y^2 is 4 at inner points, so the residual is -4 for f = 0
    y, x = np.meshgrid(np.arange(6.0), np.arange(7.0), indexing="ij")
    q = (x * x + y * y)[None]
    _, _, res = oracle.wjacobi_sweep(q, None, 1.0, 1.0, ndim=2)
    assert np.all(res[0, 1:-1, 1:-1] == -4.0)


def test_stopping_sweep_matches_closed_form_trace():
    # single mode, u0 = 0: r_n = a lambda rho^n phi, rho = 1 - omega + omega mu
    n, klm, a = 10, (1, 1, 2), 1.7
    h = 1.0 / (n + 1)
    omega, rtol, S = 6 / 7, 1e-6, 8
    phi = W.sine_mode(n, *klm)
    lam = W.mode_eigenvalue(n, *klm)
    f = a * lam * phi
    mu = sum(math.cos(q * math.pi * h) for q in klm) / 3.0
    rho = abs(1 - omega + omega * mu)
    # residual checked on u_{m-1} at m = S, 2S, ...: rel = rho^(m-1)
    m = S
    while rho ** (m - 1) > rtol:
        m += S
    u, sweeps, rel, conv = oracle.poisson_solve(f, h * h, omega, rtol, S, 100000)
    assert conv and sweeps == m
    assert abs(rel - rho ** (m - 1)) <= 1e-9 * rel
    np.testing.assert_allclose(u, a * phi * (1 - rho ** m), rtol=0, atol=1e-12)
