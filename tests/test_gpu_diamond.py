"""The diamond iteration space on the GPU (Section 3: do_diamond, cells
(i-1, j) and (i, j-1) before (i, j), 2D layers): a two-predecessor recurrence
and lexicographic Gauss-Seidel / SOR in place against the oracle (bit for bit
in FP64: the same operations per cell, and the anti-diagonal order respects
the same dependencies as the oracle's row-major order)."""
import numpy as np
import pytest

import oracle
import paper_1207_1746_amd as G

pytestmark = pytest.mark.gpu


def _g(ctx, x, dt, **kw):
    return ctx.grid(x.shape, dt, ndim=2, data=x, **kw)


@pytest.mark.parametrize("shape", [(3, 37, 53), (1, 1, 1), (1, 200, 7), (5, 1, 64), (2, 130, 129)])
@pytest.mark.parametrize("dt", [G.F64, G.F32])
def test_diamond_recur_matches_oracle(ctx, shape, dt):
    g = np.random.default_rng(70)
    a = g.uniform(-0.6, 0.6, shape)
    b = g.uniform(-0.6, 0.6, shape)
    c = g.standard_normal(shape)
    if dt == G.F32:
        a, b, c = (x.astype(np.float32).astype(np.float64) for x in (a, b, c))
    ga, gb, gc = (_g(ctx, x, dt, halo=0) for x in (a, b, c))
    go = ctx.grid(shape, dt, halo=0, ndim=2)
    ctx.do_diamond(G.K_DIAMOND_RECUR, [ga, gb, gc], [go], p=(0.75,))
    ex = oracle.diamond_recur(a, b, c, seed=0.75)
    got = go.numpy().astype(np.float64)
    if dt == G.F64:
        assert np.array_equal(got, ex)
    else:
        assert np.abs(got - ex).max() <= 256 * 2.0 ** -24 * (np.abs(ex).max() + 1)


# shapes: one partial tile; whole 64 x 64 tiles (every row batch of the
# tile's waves full); 2 x 3 tiles with 2-row and 3-column ragged tails
@pytest.mark.parametrize("shape", [(4, 45, 70), (2, 64, 128), (1, 130, 131)])
@pytest.mark.parametrize("dt", [G.F64, G.F32])
def test_gs2d_sweeps_match_oracle(ctx, dt, shape):
    g = np.random.default_rng(71)
    u = g.standard_normal(shape)
    f = g.standard_normal(shape)
    if dt == G.F32:
        u, f = u.astype(np.float32).astype(np.float64), f.astype(np.float32).astype(np.float64)
    omega, h2, bcv = 1.3, 0.05, 0.5
    gu = _g(ctx, u, dt, halo=1, bc_value=bcv)
    gf = _g(ctx, f, dt, halo=0)
    cur = u
    for _ in range(3):
        ctx.do_diamond(G.K_GS2D, [gu, gf], [gu], p=(omega, h2))
        ex = oracle.gs2d_sweep(cur, f, omega, h2, bcv)
        got = gu.numpy().astype(np.float64)
        if dt == G.F64:
            assert np.array_equal(got, ex)
        else:
            assert np.abs(got - ex).max() <= 64 * 2.0 ** -24 * (np.abs(ex).max() + 1)
        cur = got


def test_diamond_errors(ctx):
    shape = (2, 6, 8)
    a = ctx.grid(shape, G.F64, halo=0, ndim=2).fill(0.5)
    b = ctx.grid(shape, G.F64, halo=0, ndim=2).fill(0.5)
    o = ctx.grid(shape, G.F64, halo=0, ndim=2)

    def err(fn):
        with pytest.raises(G.GsclError) as e:
            fn()
        return e.value.code

    assert err(lambda: ctx.do_diamond(G.K_DIAMOND_RECUR, [a, b], [o])) == G.ERR_ARG
    assert err(lambda: ctx.do_diamond(G.K_DIAMOND_RECUR, [a, b, o], [o])) == G.ERR_ALIAS
    assert err(lambda: ctx.do_diamond(G.K_GS2D, [a], [o], p=(1.0, 1.0))) == G.ERR_ARG
    assert err(lambda: ctx.do_diamond(G.K_LINE_RECUR, [a, b], [o])) == G.ERR_ARG
    a3 = ctx.grid(shape, G.F64, halo=0).fill(0.5)
    b3 = ctx.grid(shape, G.F64, halo=0).fill(0.5)
    c3 = ctx.grid(shape, G.F64, halo=0).fill(0.5)
    o3 = ctx.grid(shape, G.F64, halo=0)
    assert err(lambda: ctx.do_diamond(G.K_DIAMOND_RECUR, [a3, b3, c3], [o3])) == G.ERR_SHAPE
    gp = ctx.grid(shape, G.F64, halo=1, ndim=2, bc=G.PERIODIC).fill(1.0)
    assert err(lambda: ctx.do_diamond(G.K_GS2D, [gp], [gp], p=(1.0, 1.0))) == G.ERR_UNSUPPORTED
