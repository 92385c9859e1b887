"""Pins of the oracle's red-black relaxation (Section 3: stateful stencils
query the index of the point they update, e.g. for red-black Gauss-Seidel).

* One sweep equals its matrix form, built independently with numpy: the
  neighbour matrix N of the 7-point stencil is the Kronecker sum of 1D path
  adjacencies, the points are split by the parity of i+j+k, and
  u_r' = (1-w) u_r + w (N_rb u_b - h^2 f_r)/6, then
  u_b' = (1-w) u_b + w (N_br u_r' - h^2 f_b)/6.
* The exact discrete solution and a constant Dirichlet state are fixed points.
* Asymptotic contraction (Young's theory for consistently ordered matrices):
  Gauss-Seidel contracts the slowest error by rho_J^2, rho_J = cos(pi h) the
  Jacobi spectral radius on the cube, and SOR with w below the optimum by the
  largest root lambda of (lambda + w - 1)^2 = lambda w^2 rho_J^2.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1207_1746_amd import workloads as W


def _path(n):
    a = np.zeros((n, n))
    for i in range(n - 1):
        a[i, i + 1] = a[i + 1, i] = 1.0
    return a


def _neighbour_matrix(nz, ny, nx):
    ix, iy, iz = np.eye(nx), np.eye(ny), np.eye(nz)
    return (np.kron(iz, np.kron(iy, _path(nx))) + np.kron(iz, np.kron(_path(ny), ix))
            + np.kron(_path(nz), np.kron(iy, ix)))


@pytest.mark.parametrize("shape", [(3, 4, 5), (4, 4, 4), (1, 3, 7), (2, 1, 6)])
@pytest.mark.parametrize("omega", [1.0, 1.4])
def test_sweep_equals_matrix_form(shape, omega):
    g = np.random.default_rng(hash(shape) % 1000)
    u = g.standard_normal(shape)
    f = g.standard_normal(shape)
    h2 = 0.3
    nz, ny, nx = shape
    N = _neighbour_matrix(nz, ny, nx)
    kk, jj, ii = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    red = ((ii + jj + kk) % 2 == 0).ravel()
    x = u.ravel().copy()
    b = f.ravel()
    for colour in (red, ~red):
        other = ~colour
        x_new = x.copy()
        x_new[colour] = (1 - omega) * x[colour] + omega * (N[np.ix_(colour, other)] @ x[other] - h2 * b[colour]) / 6
        x = x_new
    got = oracle.rbgs_sweep(u, f, omega, h2)
    np.testing.assert_allclose(got.ravel(), x, rtol=0, atol=1e-13)


def test_pass_outputs_update_and_residual():
    g = np.random.default_rng(3)
    shape = (5, 6, 7)
    u = g.standard_normal(shape)
    f = g.standard_normal(shape)
    h2 = 0.5
    for colour in (0, 1):
        un, upd, res = oracle.rbgs_pass(u, f, 1.2, h2, colour)
        kk, jj, ii = np.meshgrid(*[np.arange(n) for n in shape], indexing="ij")
        mine = (ii + jj + kk) % 2 == colour
        np.testing.assert_array_equal(un[~mine], u[~mine])
        np.testing.assert_array_equal(upd[~mine], 0.0)
        np.testing.assert_allclose(upd[mine], (un - u)[mine], rtol=0, atol=1e-14)
        _, _, jres = oracle.wjacobi_sweep(u, f, 1.0, h2)  # residual of the same u
        np.testing.assert_allclose(res[mine], jres[mine], rtol=0, atol=1e-12)
        np.testing.assert_array_equal(res[~mine], 0.0)


def test_exact_solution_and_constant_state_are_fixed_points():
    req = W.poisson_requests(count=1, qps=float("inf"), nmin=14, nmax=14, seed_index=2)[0]
    ustar, f = W.poisson_fields(req)
    for omega in (1.0, 1.7):
        got = oracle.rbgs_sweep(ustar, f, omega, req.h2)
        np.testing.assert_allclose(got, ustar, rtol=0, atol=1e-12 * np.abs(ustar).max())
    c = np.full((4, 5, 6), 0.75)
    np.testing.assert_array_equal(oracle.rbgs_sweep(c, None, 1.3, 1.0, bcv=0.75), c)


def _rate(omega, n=10, sweeps=300):
    u = np.random.default_rng(7).standard_normal((n, n, n))
    norms = []
    for _ in range(sweeps):
        u = oracle.rbgs_sweep(u, None, omega, 1.0)
        norms.append(math.sqrt(oracle.sumsq(u)))
    return norms[-1] / norms[-2]


def test_gauss_seidel_rate_is_jacobi_rate_squared():
    n = 10
    rho_j = math.cos(math.pi / (n + 1))
    assert abs(_rate(1.0, n) - rho_j ** 2) <= 2e-3 * rho_j ** 2
    # and not the Jacobi rate
    assert _rate(1.0, n) < rho_j - 0.02


def test_sor_rate_matches_young():
    n, omega = 10, 1.5
    rho_j = math.cos(math.pi / (n + 1))
    w_opt = 2 / (1 + math.sqrt(1 - rho_j ** 2))
    assert omega < w_opt
    lam = ((omega * rho_j + math.sqrt(omega ** 2 * rho_j ** 2 - 4 * (omega - 1))) / 2) ** 2
    assert abs(_rate(omega, n, 400) - lam) <= 2e-3 * lam


def test_solve_stops_at_first_chunk_meeting_rtol():
    req = W.poisson_requests(count=1, qps=float("inf"), nmin=12, nmax=12, seed_index=4)[0]
    _, f = W.poisson_fields(req)
    u, sweeps, rel, conv = oracle.rbgs_solve(f, req.h2, 1.0, 1e-6, 4, 10 ** 5)
    assert conv and sweeps % 4 == 0 and rel <= 1e-6
    _, _, res = oracle.wjacobi_sweep(u, f, 1.0, req.h2)
    assert abs(math.sqrt(oracle.sumsq(res) / oracle.sumsq(f)) - rel) <= 1e-12
    # one chunk earlier the residual was above rtol
    v = np.zeros_like(f)
    for _ in range(sweeps - 4):
        v = oracle.rbgs_sweep(v, f, 1.0, req.h2)
    _, _, res = oracle.wjacobi_sweep(v, f, 1.0, req.h2)
    assert math.sqrt(oracle.sumsq(res) / oracle.sumsq(f)) > 1e-6
