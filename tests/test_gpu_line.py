"""Ordered line iteration spaces on the GPU (Section 3: do_i/j/k_inc and
do_i/j/k_dec): a first-order recurrence and the Thomas algorithm along every
axis in both orders against the oracle (bit for bit in FP64: the same
operations in the same order), on ragged shapes and 2D layered grids, and a
batch of vertical tridiagonal solves checked by their residual."""
import numpy as np
import pytest

import oracle
import paper_1207_1746_amd as G

pytestmark = pytest.mark.gpu


def _grid(ctx, x, dt, ndim=3):
    return ctx.grid(x.shape if ndim == 3 else x.shape[1:], dt, halo=0, ndim=ndim, data=x)


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("direction", [1, -1])
@pytest.mark.parametrize("dt", [G.F64, G.F32])
def test_line_recur_matches_oracle(ctx, axis, direction, dt):
    shape = (9, 7, 131)
    g = np.random.default_rng(40 + axis)
    a = g.uniform(-0.95, 0.95, shape)
    b = g.standard_normal(shape)
    if dt == G.F32:
        a, b = a.astype(np.float32).astype(np.float64), b.astype(np.float32).astype(np.float64)
    ga, gb = _grid(ctx, a, dt), _grid(ctx, b, dt)
    go = ctx.grid(shape, dt, halo=0)
    ctx.do_line(G.K_LINE_RECUR, axis, direction, [ga, gb], [go], p=(0.5,))
    ex = oracle.line_recur(a, b, axis, direction, seed=0.5)
    got = go.numpy().astype(np.float64)
    if dt == G.F64:
        assert np.array_equal(got, ex)
    else:
        # |a| < 1: the recurrence contracts, errors stay within a few roundings of the value scale
        assert np.abs(got - ex).max() <= 64 * 2.0 ** -24 * (np.abs(ex).max() + 1)


@pytest.mark.parametrize("axis", [0, 1])
def test_line_recur_on_2d_layers(ctx, axis):
    shape = (3, 40, 70)  # three independent 2D layers
    g = np.random.default_rng(45)
    a = g.uniform(-0.9, 0.9, shape)
    b = g.standard_normal(shape)
    ga = ctx.grid(shape, G.F64, halo=0, ndim=2, data=a)
    gb = ctx.grid(shape, G.F64, halo=0, ndim=2, data=b)
    go = ctx.grid(shape, G.F64, halo=0, ndim=2)
    ctx.do_line(G.K_LINE_RECUR, axis, 1, [ga, gb], [go], p=(0.0,))
    assert np.array_equal(go.numpy(), oracle.line_recur(a, b, axis, 1, seed=0.0))


@pytest.mark.parametrize("axis,direction", [(2, 1), (2, -1), (1, 1), (0, -1)])
def test_thomas_matches_oracle(ctx, axis, direction):
    shape = (17, 9, 70)
    g = np.random.default_rng(50 + axis)
    lo = g.uniform(-1, 1, shape)
    up = g.uniform(-1, 1, shape)
    di = 2.5 + g.uniform(0, 1, shape)
    rhs = g.standard_normal(shape)
    gs = [_grid(ctx, v, G.F64) for v in (lo, di, up, rhs)]
    cp, dp, x = (ctx.grid(shape, G.F64, halo=0) for _ in range(3))
    ctx.do_line(G.K_TRIDIAG_FWD, axis, direction, gs, [cp, dp])
    ctx.do_line(G.K_TRIDIAG_BACK, axis, -direction, [cp, dp], [x])
    ecp, edp = oracle.tridiag_fwd(lo, di, up, rhs, axis, direction)
    ex = oracle.tridiag_back(ecp, edp, axis, -direction)
    assert np.array_equal(cp.numpy(), ecp) and np.array_equal(dp.numpy(), edp)
    assert np.array_equal(x.numpy(), ex)


@pytest.mark.parametrize("direction", [1, -1])
@pytest.mark.parametrize("dt", [G.F64, G.F32])
def test_lines_along_x_several_blocks(ctx, direction, dt):
    """Lines along x run 128 to a block (256 for the FP32 recurrence and
    substitution) in chunks of 32 cells: 350 lines (full blocks and a partial
    one) of 203 cells (six whole chunks and a ragged last one of 11 cells, in
    either order), recurrence and both Thomas passes against the oracle."""
    shape = (5, 70, 203)
    g = np.random.default_rng(46)
    a = g.uniform(-0.95, 0.95, shape)
    b = g.standard_normal(shape)
    lo, up = g.uniform(-1, 1, shape), g.uniform(-1, 1, shape)
    di = 2.5 + g.uniform(0, 1, shape)
    if dt == G.F32:
        a, b, lo, up, di = (v.astype(np.float32).astype(np.float64) for v in (a, b, lo, up, di))
    go = ctx.grid(shape, dt, halo=0)
    ctx.do_line(G.K_LINE_RECUR, 0, direction, [_grid(ctx, a, dt), _grid(ctx, b, dt)], [go], p=(0.25,))
    ex = oracle.line_recur(a, b, 0, direction, seed=0.25)
    gs = [_grid(ctx, v, dt) for v in (lo, di, up, b)]
    cp, dp, x = (ctx.grid(shape, dt, halo=0) for _ in range(3))
    ctx.do_line(G.K_TRIDIAG_FWD, 0, direction, gs, [cp, dp])
    ctx.do_line(G.K_TRIDIAG_BACK, 0, -direction, [cp, dp], [x])
    ecp, edp = oracle.tridiag_fwd(lo, di, up, b, 0, direction)
    exx = oracle.tridiag_back(ecp, edp, 0, -direction)
    if dt == G.F64:
        assert np.array_equal(go.numpy(), ex)
        assert np.array_equal(cp.numpy(), ecp) and np.array_equal(dp.numpy(), edp)
        assert np.array_equal(x.numpy(), exx)
    else:
        tol = 64 * 2.0 ** -24
        assert np.abs(go.numpy() - ex).max() <= tol * (np.abs(ex).max() + 1)
        # diagonally dominant systems: the F32 solve stays within a few roundings
        assert np.abs(x.numpy() - exx).max() <= 16 * tol * (np.abs(exx).max() + 1)


def test_vertical_tridiagonal_solves_residual(ctx):
    """256 x 256 columns of 128 levels (climate-style implicit vertical
    solves), F64: every column's residual |A x - rhs| is at rounding level."""
    import torch
    nz, ny, nx = 128, 256, 256
    gen = torch.Generator(device="cuda").manual_seed(3)
    shape = (nz, ny, nx)
    lo = torch.rand(shape, dtype=torch.float64, device="cuda", generator=gen) * 2 - 1
    up = torch.rand(shape, dtype=torch.float64, device="cuda", generator=gen) * 2 - 1
    di = torch.rand(shape, dtype=torch.float64, device="cuda", generator=gen) + 2.5
    rhs = torch.randn(shape, dtype=torch.float64, device="cuda", generator=gen)
    grids = []
    for t in (lo, di, up, rhs):
        gg = ctx.grid(shape, G.F64, halo=0)
        gg.view.copy_(t)
        grids.append(gg)
    cp, dp, x = (ctx.grid(shape, G.F64, halo=0) for _ in range(3))
    ctx.do_line(G.K_TRIDIAG_FWD, 2, 1, grids, [cp, dp])
    ctx.do_line(G.K_TRIDIAG_BACK, 2, -1, [cp, dp], [x])
    xv = x.view
    ax = di * xv
    ax[1:] += lo[1:] * xv[:-1]
    ax[:-1] += up[:-1] * xv[1:]
    res = (ax - rhs).abs().max().item()
    assert res <= 1e-13 * rhs.abs().max().item()


def test_line_errors(ctx):
    shape = (4, 5, 6)
    a = ctx.grid(shape, G.F64, halo=0).fill(0.5)
    b = ctx.grid(shape, G.F64, halo=0).fill(1.0)
    o = ctx.grid(shape, G.F64, halo=0)

    def err(fn):
        with pytest.raises(G.GsclError) as e:
            fn()
        return e.value.code

    assert err(lambda: ctx.do_line(G.K_LINE_RECUR, 3, 1, [a, b], [o])) == G.ERR_ARG
    assert err(lambda: ctx.do_line(G.K_LINE_RECUR, 0, 0, [a, b], [o])) == G.ERR_ARG
    assert err(lambda: ctx.do_line(G.K_LINE_RECUR, 0, 1, [a], [o])) == G.ERR_ARG
    assert err(lambda: ctx.do_line(G.K_WJACOBI, 0, 1, [a, b], [o])) == G.ERR_ARG
    assert err(lambda: ctx.do_line(G.K_LINE_RECUR, 2, 1, [a, b], [a])) == G.ERR_ALIAS
    l2 = ctx.grid((2, 5, 6), G.F64, halo=0, ndim=2)
    m2 = ctx.grid((2, 5, 6), G.F64, halo=0, ndim=2)
    n2 = ctx.grid((2, 5, 6), G.F64, halo=0, ndim=2)
    assert err(lambda: ctx.do_line(G.K_LINE_RECUR, 2, 1, [l2, m2], [n2])) == G.ERR_SHAPE
    i8 = ctx.grid(shape, G.U8, halo=0)
    assert err(lambda: ctx.do_line(G.K_LINE_RECUR, 0, 1, [i8, i8], [o])) == G.ERR_DTYPE
