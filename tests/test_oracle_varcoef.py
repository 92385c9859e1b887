"""Pins for the oracle's variable-coefficient multi-grid sweep (9 inputs, 3 outputs).

* Invariant: r = C (u' - u) for every input (C = sum of the 7 coefficients).
* Fixed point: a constant u with s = 0 gives u' = u, r = 0, |F| = 0.
* Independent evaluator: numpy.roll implements the periodic shifts.
* Conservation: with symmetric fluxes the operator reduces to periodic
  diffusion, which conserves the grid sum.
"""
import numpy as np

import oracle
from paper_1207_1746_amd import workloads as W


def _rolled(u, dx, dy, dz):
    # value at p + (dx, dy, dz) under periodic boundaries
    return np.roll(u, shift=(-dz, -dy, -dx), axis=(0, 1, 2))


def test_matches_roll_evaluator():
    u, c, s = W.varcoef_grids(7, 6, 5)
    u, c, s = u.astype(np.float64), [x.astype(np.float64) for x in c], s.astype(np.float64)
    unew, r, fm = oracle.varcoef7_sweep(u, c, s)
    offs = [(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)]
    nb = [_rolled(u, *o) for o in offs]
    out = sum(ck * v for ck, v in zip(c, nb))
    C = sum(c)
    np.testing.assert_allclose(unew, (out + s) / C, rtol=1e-14, atol=1e-14)
    np.testing.assert_allclose(r, s + out - C * u, rtol=1e-13, atol=1e-13)
    F = [0.5 * (c[1 + 2 * d] * (nb[1 + 2 * d] - u) + c[2 + 2 * d] * (u - nb[2 + 2 * d]))
         for d in range(3)]
    np.testing.assert_allclose(fm, np.sqrt(F[0] ** 2 + F[1] ** 2 + F[2] ** 2), rtol=1e-13,
                               atol=1e-14)


def test_residual_equals_C_times_update():
    u, c, s = W.varcoef_grids(8)
    unew, r, _ = oracle.varcoef7_sweep(u, c, s)
    C = sum(x.astype(np.float64) for x in c)
    np.testing.assert_allclose(r, C * (unew - u.astype(np.float64)), rtol=0,
                               atol=1e-13 * (np.abs(u).max() + 1))


def test_constant_field_is_fixed_point():
    shp = (4, 5, 6)
    g = np.random.default_rng(1)
    # dyadic coefficients k/8 keep every sum exact, so the fixed point is exact
    c = [g.integers(1, 9, shp) / 8.0 for _ in range(7)]
    u = np.full(shp, 0.75)
    unew, r, fm = oracle.varcoef7_sweep(u, c, np.zeros(shp))
    assert np.all(unew == 0.75) and np.all(r == 0.0) and np.all(fm == 0.0)
    # general coefficients: zero up to a few ulps of C u
    c = [g.uniform(0.1, 1, shp) for _ in range(7)]
    unew, r, fm = oracle.varcoef7_sweep(u, c, np.zeros(shp))
    np.testing.assert_allclose(unew, 0.75, rtol=4 * 2.0 ** -52)
    assert np.all(np.abs(r) <= 8 * 2.0 ** -52 * 7 * 0.75) and np.all(fm == 0.0)


def test_symmetric_coefficients_conserve_sum():
    # c_{+d}(p) = c_{-d}(p + e_d) = k_d(p) makes sum_k c_k (u_k - u) a divergence:
    # r sums to sum(s) exactly in exact arithmetic.
    shp = (6, 5, 7)
    g = np.random.default_rng(4)
    kx, ky, kz = (g.uniform(0.1, 1, shp) for _ in range(3))
    c = [g.uniform(0.1, 1, shp), kx, _rolled(kx, -1, 0, 0), ky, _rolled(ky, 0, -1, 0), kz,
         _rolled(kz, 0, 0, -1)]
    u = g.standard_normal(shp)
    s = g.standard_normal(shp)
    _, r, _ = oracle.varcoef7_sweep(u, c, s)
    assert abs(oracle.sum(r) - oracle.sum(s)) <= 1e-12 * (oracle.sum(np.abs(r)) + 1)


def test_run_records_residual_norms():
    u, c, s = W.varcoef_grids(6)
    uf, r, fm, norms = oracle.varcoef7_run(u, c, s, 20, 10)
    assert len(norms) == 2
    # the same sweeps one by one
    x = u.astype(np.float64)
    for n in range(20):
        x, rr, _ = oracle.varcoef7_sweep(x, c, s)
        if n == 9:
            assert norms[0] == np.sqrt(oracle.sumsq(rr))
    assert np.array_equal(x, uf) and norms[1] == np.sqrt(oracle.sumsq(r))
