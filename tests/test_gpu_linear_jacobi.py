"""GPU parity: generic LINEAR do_all and the weighted-Jacobi sweep against the
FP64 oracle (Section 3 do_all, Fig. 1b, Section 5.2 averaging + fused check).

Tolerances: F64 sweeps elementwise |g - o| <= 1e-12 * (sum of |terms|) (one
sweep) and ||g - o||_inf <= 1e-12 * ||u0||_inf after k sweeps (the sweep is a
contraction, so per-sweep rounding does not grow); F32 uses 2^-24 in place of
1e-12 with an 8-operation rounding budget.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
import paper_1207_1746_amd as G
from paper_1207_1746_amd import workloads as W

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))

SHAPES = [(29, 53, 37), (9, 70, 130), (8, 8, 8), (1, 1, 1), (3, 5, 300)]


def _rand_terms(g, nin, nout, R, ndim, n=10):
    terms = []
    for _ in range(n):
        dz = int(g.integers(-R, R + 1)) if ndim == 3 else 0
        terms.append((int(g.integers(0, nout)), int(g.integers(0, nin)), int(g.integers(-R, R + 1)),
                      int(g.integers(-R, R + 1)), dz, float(g.standard_normal()),
                      int(g.integers(-1, nin))))
    return terms


@pytest.mark.parametrize("bc", [G.DIRICHLET, G.PERIODIC, G.CLAMP])
@pytest.mark.parametrize("shape", [(29, 53, 37), (6, 17, 70)])
@pytest.mark.parametrize("ndim", [3, 2])
def test_linear_random_terms_f64(ctx, bc, shape, ndim):
    g = np.random.default_rng(hash((bc, shape, ndim)) % 2 ** 32)
    ins_np = [g.standard_normal(shape) for _ in range(3)]
    R = 2
    terms = _rand_terms(g, 3, 2, R, ndim, 14)
    bcv = [0.0, 0.75, -1.5]
    ins = [ctx.grid(shape, G.F64, halo=R, bc=bc, bc_value=bcv[i], ndim=ndim, data=a)
           for i, a in enumerate(ins_np)]
    outs = [ctx.grid(shape, G.F64, halo=0, ndim=ndim) for _ in range(2)]
    ctx.do_all(G.K_LINEAR, ins, outs, terms=terms)
    exp = oracle.linear(ndim, ins_np, terms, 2, [bc] * 3, bcv)
    for o, e in zip(outs, exp):
        got = o.numpy().reshape(e.shape)
        scale = sum(abs(t[5]) for t in terms) * max(np.abs(a).max() for a in ins_np) ** 2
        np.testing.assert_allclose(got, e, rtol=0, atol=1e-12 * scale)


def test_linear_f32_and_fused_reduce(ctx):
    g = np.random.default_rng(3)
    shape = (11, 40, 77)
    u = g.standard_normal(shape).astype(np.float32)
    terms = [(0, 0, dx, dy, dz, w, -1) for (dx, dy, dz, w) in
             [(1, 0, 0, .25), (-1, 0, 0, .25), (0, 1, 0, .125), (0, -1, 0, .125), (0, 0, 1, .5),
              (0, 0, -1, -.5), (0, 0, 0, -.75)]]
    gin = ctx.grid(shape, G.F32, halo=1, data=u)
    gout = ctx.grid(shape, G.F32, halo=0)
    ex = oracle.linear(3, [u], terms, 1, [G.DIRICHLET], [0.0])[0]
    for op in (G.R_SUM, G.R_SUMSQ, G.R_L2, G.R_MAXABS):
        r = ctx.do_all(G.K_LINEAR, [gin], [gout], terms=terms, reduce=(op, G.RV_OUT0))
        got = gout.numpy()
        np.testing.assert_allclose(got, ex, rtol=0, atol=8 * 2 ** -24 * 2.5 * np.abs(u).max())
        # the reduction sees the F32 outputs the kernel computed
        gd = got.astype(np.float64)
        ref = {G.R_SUM: oracle.sum(gd), G.R_SUMSQ: oracle.sumsq(gd), G.R_L2: math.sqrt(oracle.sumsq(gd)),
               G.R_MAXABS: oracle.maxabs(gd)}[op]
        assert abs(r - ref) <= 1e-12 * max(abs(ref), oracle.sum(np.abs(gd)) if op == G.R_SUM else 0)
    # ALL_LE and UPDATE operand
    m = oracle.maxabs(gout.numpy().astype(np.float64) - u.astype(np.float64))
    assert ctx.do_all(G.K_LINEAR, [gin], [gout], terms=terms, reduce=(G.R_ALL_LE, G.RV_UPDATE, m * 1.001)) == 1.0
    assert ctx.do_all(G.K_LINEAR, [gin], [gout], terms=terms, reduce=(G.R_ALL_LE, G.RV_UPDATE, m * 0.999)) == 0.0


def test_fig1b_operator_golden(ctx):
    gold = json.load(open(os.path.join(HERE, "golden", "fig1b_operator.json")))
    terms = [(0, 0, dx, dy, dz, num / den, -1) for dx, dy, dz, num, den in gold["terms"]]
    nz, ny, nx = 10, 12, 14
    z, y, x = np.meshgrid(np.arange(nz, dtype=float), np.arange(ny, dtype=float), np.arange(nx, dtype=float),
                          indexing="ij")
    a, b, c = 1.0, 2.0, -4.0
    u = a * x * x + b * y * y + c * z * z + x * y * z - 2 * x
    gu = ctx.grid(u.shape, G.F64, halo=1, data=u)
    gv = ctx.grid(u.shape, G.F64, halo=0)
    ctx.do_all(G.K_LINEAR, [gu], [gv], terms=terms)
    v = gv.numpy()
    np.testing.assert_allclose(v[1:-1, 1:-1, 1:-1], -(a + b + c) / 18.0, rtol=0, atol=1e-12 * np.abs(u).max())
    np.testing.assert_allclose(v, oracle.linear(3, [u], terms, 1, [0], [0.0])[0], rtol=0,
                               atol=1e-12 * np.abs(u).max())


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("bc", [G.DIRICHLET, G.PERIODIC, G.CLAMP])
@pytest.mark.parametrize("has_f", [False, True])
def test_wjacobi_f64_one_sweep(ctx, shape, bc, has_f):
    g = np.random.default_rng(11)
    u = g.uniform(-1, 1, shape)
    f = g.standard_normal(shape) if has_f else None
    omega, h2 = 6 / 7, 0.37
    gu = ctx.grid(shape, G.F64, halo=1, bc=bc, bc_value=0.25 if bc == G.DIRICHLET else 0.0, data=u)
    ins = [gu] + ([ctx.grid(shape, G.F64, halo=0, data=f)] if has_f else [])
    go = ctx.grid(shape, G.F64, halo=1)
    for operand in (G.RV_UPDATE, G.RV_RESIDUAL):
        l2 = ctx.do_all(G.K_WJACOBI, ins, [go], p=(omega, h2), reduce=(G.R_SUMSQ, operand))
        un, upd, res = oracle.wjacobi_sweep(u, f, omega, h2, bc, 0.25 if bc == G.DIRICHLET else 0.0)
        scale = 6 * max(np.abs(u).max(), 0.25) + (h2 * np.abs(f).max() if has_f else 0)
        np.testing.assert_allclose(go.numpy(), un, rtol=0, atol=1e-12 * scale)
        ref = oracle.sumsq(upd if operand == G.RV_UPDATE else res)
        # relative, plus the rounding floor of each per-point value (scale, /h2 for residuals)
        floor = (1e-13 * scale / (h2 if operand == G.RV_RESIDUAL else 1.0)) ** 2 * u.size
        assert abs(l2 - ref) <= 1e-11 * ref + floor


def test_wjacobi_cube_10_sweeps_l2_update(ctx):
    """64^3 FP64, Dirichlet 0, f = 0, 10 sweeps, then ||u10 - u9||_2 (fused)."""
    u0, h2 = W.jacobi_cube(64)
    a = ctx.grid(u0.shape, G.F64, halo=1, data=u0)
    b = ctx.grid(u0.shape, G.F64, halo=1)
    for k in range(10):
        src, dst = (a, b) if k % 2 == 0 else (b, a)
        red = (G.R_L2, G.RV_UPDATE) if k == 9 else None
        r = ctx.do_all(G.K_WJACOBI, [src], [dst], p=(1.0, h2), reduce=red)
    uo, l2, _ = oracle.jacobi_run(u0, 10, None, 1.0, h2)
    got = a.numpy()
    assert np.abs(got - uo).max() <= 1e-12 * np.abs(u0).max()
    assert abs(r - l2) <= 1e-12 * l2


def test_wjacobi_mode_decay_closed_form(ctx):
    n, klm, omega = 40, (2, 3, 1), 6 / 7
    h = 1.0 / (n + 1)
    phi = W.sine_mode(n, *klm)
    mu = sum(math.cos(q * math.pi * h) for q in klm) / 3
    gfac = 1 - omega + omega * mu
    a = ctx.grid(phi.shape, G.F64, halo=1, data=phi)
    b = ctx.grid(phi.shape, G.F64, halo=1)
    for k in range(6):
        src, dst = (a, b) if k % 2 == 0 else (b, a)
        r = ctx.do_all(G.K_WJACOBI, [src], [dst], p=(omega, h * h), reduce=(G.R_L2, G.RV_UPDATE))
    np.testing.assert_allclose(a.numpy(), gfac ** 6 * phi, rtol=0, atol=1e-14)
    expect = abs(gfac ** 6 - gfac ** 5) * math.sqrt(((n + 1) / 2) ** 3)
    assert abs(r - expect) <= 1e-11 * expect


def test_wjacobi_tiling_invariance(ctx):
    """do_all outputs are bitwise identical for every tile shape."""
    shape = (21, 45, 150)
    u = np.random.default_rng(5).standard_normal(shape)
    gu = ctx.grid(shape, G.F64, halo=1, bc=G.PERIODIC, data=u)
    ref = None
    for V in (1, 2):
        for NW in (4, 8):
            for cz in (1, 4, 7, 32):
                ctx.tile_set(G.K_WJACOBI, gu, (V, NW, cz))
                go = ctx.grid(shape, G.F64, halo=1)
                ctx.do_all(G.K_WJACOBI, [gu], [go], p=(0.9, 1.0))
                out = go.numpy()
                if ref is None:
                    ref = out
                assert np.array_equal(out, ref), (V, NW, cz)
    ctx.tile_clear()
    np.testing.assert_allclose(ref, oracle.wjacobi_sweep(u, None, 0.9, 1.0, G.PERIODIC)[0], rtol=0, atol=1e-14)


def test_wjacobi_f32_and_2d_layers(ctx):
    g = np.random.default_rng(8)
    shape = (13, 66, 260)
    u = g.standard_normal(shape).astype(np.float32)
    f = g.standard_normal(shape).astype(np.float32)
    gu = ctx.grid(shape, G.F32, halo=1, bc=G.CLAMP, data=u)
    gf = ctx.grid(shape, G.F32, halo=0, data=f)
    go = ctx.grid(shape, G.F32, halo=1)
    ctx.do_all(G.K_WJACOBI, [gu, gf], [go], p=(0.8, 0.5))
    un = oracle.wjacobi_sweep(u, f, 0.8, 0.5, G.CLAMP)[0]
    np.testing.assert_allclose(go.numpy(), un, rtol=0, atol=10 * 2 ** -24 * (6 * np.abs(u).max() + 0.5 * np.abs(f).max()))
    # 2D: nz independent layers, 4-neighbour average
    u2 = g.standard_normal((3, 33, 70))
    a = ctx.grid(u2.shape, G.F64, halo=1, ndim=2, bc=G.PERIODIC, data=u2)
    b = ctx.grid(u2.shape, G.F64, halo=1, ndim=2)
    ctx.do_all(G.K_WJACOBI, [a], [b], p=(1.0, 1.0))
    np.testing.assert_allclose(b.numpy(), oracle.wjacobi_sweep(u2, None, 1.0, 1.0, G.PERIODIC, ndim=2)[0],
                               rtol=0, atol=1e-14 * 4 * np.abs(u2).max())


def test_prepared_call_equals_do_all(ctx):
    """Context.prepare_all issues the same gscl_do_all call: ten sweeps with a
    fused update norm give the grids and norms do_all gives, host or device
    result, and a failing call still raises."""
    import torch
    shape = (20, 33, 70)
    u0 = np.random.default_rng(81).standard_normal(shape)
    grids = {}
    for tag in ("a", "b"):
        grids[tag] = (ctx.grid(shape, G.F64, halo=1, data=u0), ctx.grid(shape, G.F64, halo=1))
    res = torch.zeros(1, dtype=torch.float64, device="cuda")
    calls = []
    x, y = grids["b"]
    for k in range(10):
        src, dst = (x, y) if k % 2 == 0 else (y, x)
        calls.append(ctx.prepare_all(G.K_WJACOBI, [src], [dst], p=(0.9, 0.01),
                                     reduce=(G.R_L2, G.RV_UPDATE) if k == 9 else None))
    dev = ctx.prepare_all(G.K_WJACOBI, [x], [y], p=(0.9, 0.01), reduce=(G.R_L2, G.RV_UPDATE), dev_result=res)
    x0, y0 = grids["a"]
    for k in range(10):
        src, dst = (x0, y0) if k % 2 == 0 else (y0, x0)
        r_ref = ctx.do_all(G.K_WJACOBI, [src], [dst], p=(0.9, 0.01),
                           reduce=(G.R_L2, G.RV_UPDATE) if k == 9 else None)
        r_got = calls[k]()
        assert (r_got is None) == (k != 9)
    assert r_got == r_ref
    assert np.array_equal(x.numpy(), x0.numpy()) and np.array_equal(y.numpy(), y0.numpy())
    assert dev() is None
    ref = ctx.do_all(G.K_WJACOBI, [x0], [y0], p=(0.9, 0.01), reduce=(G.R_L2, G.RV_UPDATE))
    torch.cuda.synchronize()
    assert res.item() == ref
    bad = ctx.prepare_all(G.K_WJACOBI, [x], [x], p=(0.9, 0.01))
    with pytest.raises(G.GsclError):
        bad()
