"""Pins for the oracle's generic linear do_all (Section 3, Fig. 1b).

The oracle is checked against things other than itself: exact closed forms of
the discrete Laplacian on polynomials, the operator printed in Fig. 1b, and an
independent evaluator built on numpy's own padding modes ('constant', 'wrap',
'edge' are the Dirichlet, periodic and clamp boundary rules).
"""
import json
import os

import numpy as np
import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))

LAP7 = [(0, 0, 1, 0, 0, 1.0, -1), (0, 0, -1, 0, 0, 1.0, -1), (0, 0, 0, 1, 0, 1.0, -1),
        (0, 0, 0, -1, 0, 1.0, -1), (0, 0, 0, 0, 1, 1.0, -1), (0, 0, 0, 0, -1, 1.0, -1),
        (0, 0, 0, 0, 0, -6.0, -1)]


def _coords(nz, ny, nx):
    z, y, x = np.meshgrid(np.arange(nz, dtype=np.float64), np.arange(ny, dtype=np.float64),
                          np.arange(nx, dtype=np.float64), indexing="ij")
    return x, y, z


def test_laplacian_of_quadratic_is_exact():
    # 7-point Laplacian of a x^2 + b y^2 + c z^2 + (bilinear/trilinear/linear) = 2(a+b+c),
    # exactly, at integer coordinates with unit spacing.
    nz, ny, nx = 7, 9, 11
    x, y, z = _coords(nz, ny, nx)
    a, b, c = 3.0, -2.0, 5.0
    u = a * x * x + b * y * y + c * z * z + 4 * x * y - 3 * y * z + 2 * x * z + 7 * x * y * z \
        + x - 6 * y + 2 * z + 11
    (out,) = oracle.linear(3, [u], LAP7, 1, [oracle.DIRICHLET], [0.0])
    inner = out[1:-1, 1:-1, 1:-1]
    assert np.all(inner == 2 * (a + b + c))


def test_laplacian_of_trilinear_is_zero():
    nz, ny, nx = 6, 5, 8
    x, y, z = _coords(nz, ny, nx)
    u = 2 * x * y * z - x * y + 3 * y * z + x - 4
    for bc in (oracle.DIRICHLET, oracle.CLAMP):
        (out,) = oracle.linear(3, [u], LAP7, 1, [bc], [0.0])
        assert np.all(out[1:-1, 1:-1, 1:-1] == 0.0)


def test_fig1b_operator_on_quadratic():
    g = json.load(open(os.path.join(HERE, "golden", "fig1b_operator.json")))
    terms = [(0, 0, dx, dy, dz, num / den, -1) for dx, dy, dz, num, den in g["terms"]]
    nz, ny, nx = 6, 7, 8
    x, y, z = _coords(nz, ny, nx)
    a, b, c = 1.0, 2.0, -4.0
    u = a * x * x + b * y * y + c * z * z + x * y * z - 2 * x
    (v,) = oracle.linear(3, [u], terms, 1, [oracle.DIRICHLET], [0.0])
    expect = -(a + b + c) / 18.0
    np.testing.assert_allclose(v[1:-1, 1:-1, 1:-1], expect, rtol=1e-12, atol=1e-12 * np.abs(u).max())


def _pad_mode(bc):
    return {oracle.DIRICHLET: "constant", oracle.PERIODIC: "wrap", oracle.CLAMP: "edge"}[bc]


def _independent_linear(ndim, ins, terms, nout, bc, bcv, R):
    """Evaluate the same operator with numpy.pad halos and shifted slices."""
    padded = []
    for g, a in enumerate(ins):
        if ndim == 3:
            pw = ((R, R), (R, R), (R, R))
        else:
            pw = ((0, 0), (R, R), (R, R))
        kw = {"constant_values": bcv[g]} if bc[g] == oracle.DIRICHLET else {}
        padded.append(np.pad(a, pw, mode=_pad_mode(bc[g]), **kw))
    nz, ny, nx = ins[0].shape
    outs = [np.zeros((nz, ny, nx)) for _ in range(nout)]
    for (o, g, dx, dy, dz, w, coef) in terms:
        zoff = R + dz if ndim == 3 else 0
        sl = padded[g][zoff:zoff + nz, R + dy:R + dy + ny, R + dx:R + dx + nx]
        cf = ins[coef] if coef >= 0 else 1.0
        outs[o] = outs[o] + w * cf * sl
    return outs


@pytest.mark.parametrize("bc", [oracle.DIRICHLET, oracle.PERIODIC, oracle.CLAMP])
@pytest.mark.parametrize("ndim", [2, 3])
def test_linear_matches_padded_evaluator(bc, ndim):
    g = np.random.default_rng(7 + bc + 10 * ndim)
    shp = (5, 6, 7)
    ins = [g.standard_normal(shp) for _ in range(3)]
    R = 2
    terms = []
    for _ in range(12):
        dz = int(g.integers(-R, R + 1)) if ndim == 3 else 0
        terms.append((int(g.integers(0, 2)), int(g.integers(0, 3)), int(g.integers(-R, R + 1)),
                      int(g.integers(-R, R + 1)), dz, float(g.standard_normal()),
                      int(g.integers(-1, 3))))
    bcs = [bc] * 3
    bcv = [0.0, 0.5, -1.25]
    got = oracle.linear(ndim, ins, terms, 2, bcs, bcv)
    exp = _independent_linear(ndim, ins, terms, 2, bcs, bcv, R)
    for a, b in zip(got, exp):
        np.testing.assert_allclose(a, b, rtol=1e-13, atol=1e-13)


def test_mixed_boundaries_per_grid():
    g = np.random.default_rng(3)
    shp = (4, 5, 6)
    ins = [g.standard_normal(shp) for _ in range(3)]
    bcs = [oracle.DIRICHLET, oracle.PERIODIC, oracle.CLAMP]
    bcv = [2.0, 0.0, 0.0]
    terms = [(0, 0, -1, 0, 0, 1.0, -1), (0, 1, 0, 1, -1, 1.0, -1), (0, 2, 1, 1, 1, 1.0, 0)]
    got = oracle.linear(3, ins, terms, 1, bcs, bcv)
    exp = _independent_linear(3, ins, terms, 1, bcs, bcv, 1)
    np.testing.assert_allclose(got[0], exp[0], rtol=1e-14, atol=1e-14)


def test_periodic_diffusion_conserves_sum():
    # u' = u + nu (sum of 6 neighbours - 6u) with periodic boundaries conserves sum(u).
    g = np.random.default_rng(11)
    u = g.uniform(-1, 1, size=(9, 10, 11))
    nu = 0.125
    terms = [(0, 0, dx, dy, dz, nu, -1) for dx, dy, dz in
             [(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)]]
    terms.append((0, 0, 0, 0, 0, 1 - 6 * nu, -1))
    s0 = oracle.sum(u)
    scale = oracle.sum(np.abs(u))
    for _ in range(5):
        (u,) = oracle.linear(3, [u], terms, 1, [oracle.PERIODIC], [0.0])
        assert abs(oracle.sum(u) - s0) <= 1e-12 * scale
    # a constant field is a fixed point
    cst = np.full((4, 4, 4), 0.375)
    (out,) = oracle.linear(3, [cst], terms, 1, [oracle.PERIODIC], [0.0])
    assert np.all(out == 0.375)
