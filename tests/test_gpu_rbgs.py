"""Red-black relaxation on the GPU (Section 3: stateful stencils query the
index of the point they update): one colour pass in place against the
oracle's pass (values, update and residual reductions), bitwise invariance
under every tile shape, and Gauss-Seidel / SOR solves against the oracle's
checked solve (same stopping sweep, same iterate)."""
import math

import numpy as np
import pytest

import oracle
import paper_1207_1746_amd as G
from paper_1207_1746_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("shape", [(11, 13, 150), (1, 1, 1), (2, 3, 5), (6, 40, 129)])
@pytest.mark.parametrize("dt", [G.F64, G.F32])
def test_rbgs_pass_matches_oracle(ctx, shape, dt):
    g = np.random.default_rng(31)
    u = g.standard_normal(shape)
    f = g.standard_normal(shape)
    if dt == G.F32:
        u, f = u.astype(np.float32).astype(np.float64), f.astype(np.float32).astype(np.float64)
    omega, h2, bcv = 1.3, 0.4, 0.25
    gu = ctx.grid(shape, dt, halo=1, bc_value=bcv, data=u)
    gf = ctx.grid(shape, dt, halo=0, data=f)
    cur = u
    for colour in (0, 1, 0):
        l2u = ctx.do_all(G.K_RBGS, [gu, gf], [gu], p=(omega, h2, colour), reduce=(G.R_L2, G.RV_UPDATE))
        ex, upd, _ = oracle.rbgs_pass(cur, f, omega, h2, colour, bcv)
        scale = 8 * (np.abs(cur).max() + bcv) + h2 * np.abs(f).max()
        tol = (1e-14 if dt == G.F64 else 16 * 2.0 ** -24) * scale
        got = gu.numpy()
        assert np.abs(got - ex).max() <= tol, colour
        assert abs(l2u - math.sqrt(oracle.sumsq(upd))) <= 1e3 * tol * (1 + math.sqrt(upd.size))
        cur = got.astype(np.float64)
    # residual operand: the residual before the update, at the pass's points
    _, _, res = oracle.rbgs_pass(cur, f, omega, h2, 1, bcv)
    l2r = ctx.do_all(G.K_RBGS, [gu, gf], [gu], p=(omega, h2, 1), reduce=(G.R_SUMSQ, G.RV_RESIDUAL))
    rel = 1e-12 if dt == G.F64 else 1e-5
    assert abs(l2r - oracle.sumsq(res)) <= rel * max(oracle.sumsq(res), 1.0)


@pytest.mark.parametrize("dt", [G.F64, G.F32])
def test_rbgs_tiling_invariance(ctx, dt):
    shape = (13, 37, 203)
    g = np.random.default_rng(32)
    u = g.standard_normal(shape)
    f = g.standard_normal(shape)
    gf = ctx.grid(shape, dt, halo=0, data=f)
    ref = None
    for V in (1, 2):
        for NW in (4, 8):
            for cz in (1, 5, 32):
                gu = ctx.grid(shape, dt, halo=1, data=u)
                ctx.tile_set(G.K_RBGS, gu, (V, NW, cz))
                for colour in (0, 1):
                    ctx.do_all(G.K_RBGS, [gu, gf], [gu], p=(1.6, 0.1, colour))
                got = gu.numpy()
                if ref is None:
                    ref = got
                assert np.array_equal(got, ref), (V, NW, cz)
    ctx.tile_clear()


def test_rbgs_errors(ctx):
    shape = (6, 7, 40)
    gu = ctx.grid(shape, G.F64, halo=1).fill(1.0)
    go = ctx.grid(shape, G.F64, halo=1)

    def err(fn):
        with pytest.raises(G.GsclError) as e:
            fn()
        return e.value.code

    assert err(lambda: ctx.do_all(G.K_RBGS, [gu], [go], p=(1.0, 1.0, 0))) == G.ERR_ARG
    assert err(lambda: ctx.do_all(G.K_RBGS, [gu], [gu], p=(1.0, 1.0, 2))) == G.ERR_ARG
    assert err(lambda: ctx.do_all(G.K_RBGS, [gu, gu], [gu], p=(1.0, 1.0, 0))) == G.ERR_ALIAS
    gp = ctx.grid(shape, G.F64, halo=1, bc=G.PERIODIC).fill(1.0)
    assert err(lambda: ctx.do_all(G.K_RBGS, [gp], [gp], p=(1.0, 1.0, 0))) == G.ERR_UNSUPPORTED
    g0 = ctx.grid(shape, G.F64, halo=0).fill(1.0)
    assert err(lambda: ctx.do_all(G.K_RBGS, [g0], [g0], p=(1.0, 1.0, 0))) == G.ERR_HALO


def _opt_omega(n):
    # the model-problem optimum the solver uses for omega = 0 (a cube here)
    c = math.cos(math.pi / (n + 1))
    rho = (c + c + c) / 3.0
    return 2 / (1 + math.sqrt(1 - rho * rho))


@pytest.mark.parametrize("n,S,omega", [(24, 4, 1.0), (24, 4, 0.0), (31, 6, 1.5)])
def test_rbgs_solve_matches_oracle(ctx, n, S, omega):
    req = W.poisson_requests(count=1, qps=float("inf"), nmin=n, nmax=n, seed_index=n)[0]
    ustar, f = W.poisson_fields(req)
    u = ctx.grid(f.shape, G.F64, halo=1).fill(0.0)
    gf = ctx.grid(f.shape, G.F64, halo=0, data=f)
    st = ctx.solve(G.K_RBGS, [u], [gf], omega=omega, h2=req.h2, rtol=1e-8, check_every=S)
    w = omega if omega != 0.0 else _opt_omega(n)
    uo, so, relo, conv = oracle.rbgs_solve(f, req.h2, w, 1e-8, S, 10 ** 6)
    assert conv and st["sweeps"] == so
    assert abs(st["rel_residual"] - relo) <= 1e-6 * relo
    assert np.abs(u.numpy() - uo).max() <= 1e-11 * np.abs(uo).max()


def test_sor_needs_far_fewer_sweeps_than_jacobi(ctx):
    """Same request, same rtol: optimal SOR (O(N) sweeps) against weighted
    Jacobi (O(N^2) sweeps), both returning answers the oracle accepts."""
    n = 96
    req = W.poisson_requests(count=1, qps=float("inf"), nmin=n, nmax=n, seed_index=9)[0]
    _, f = W.poisson_fields(req)
    gf = ctx.grid(f.shape, G.F64, halo=0, data=f)
    res = {}
    for name, kind, omega in (("jacobi", G.K_WJACOBI, 6 / 7), ("sor", G.K_RBGS, 0.0)):
        u = ctx.grid(f.shape, G.F64, halo=1).fill(0.0)
        st = ctx.solve(kind, [u], [gf], omega=omega, h2=req.h2, rtol=1e-8, check_every=16)
        _, _, r = oracle.wjacobi_sweep(u.numpy(), f, 1.0, req.h2)
        assert math.sqrt(oracle.sumsq(r) / oracle.sumsq(f)) <= 1e-8 * 1.0001
        res[name] = st["sweeps"]
    assert res["sor"] * 10 < res["jacobi"], res


def _inplace_passes(ctx, u, f, dt, omega, h2, c0, k, reduce=None):
    gu = ctx.grid(u.shape, dt, halo=1, data=u)
    gf = ctx.grid(u.shape, dt, halo=0, data=f)
    r = None
    for q in range(k):
        last = q == k - 1
        r = ctx.do_all(G.K_RBGS, [gu, gf], [gu], p=(omega, h2, (c0 + q) % 2),
                       reduce=reduce if last else None)
    return gu.numpy(), r


@pytest.mark.parametrize("shape", [(9, 37, 203), (2, 3, 5), (1, 1, 1), (21, 50, 120)])
@pytest.mark.parametrize("dt", [G.F64, G.F32])
def test_rbgs_blocked_equals_inplace_passes(ctx, shape, dt):
    """k colour passes in one blocked pass (Sections 2 and 3) against k
    in-place colour passes: bit for bit, for every k and first colour; the
    fused update norm of the last pass agrees to reduction-order rounding."""
    g = np.random.default_rng(33)
    u = g.standard_normal(shape)
    f = g.standard_normal(shape)
    if dt == G.F32:
        u, f = u.astype(np.float32).astype(np.float64), f.astype(np.float32).astype(np.float64)
    omega, h2 = 1.7, 0.3
    gu = ctx.grid(shape, dt, halo=1, data=u)
    gf = ctx.grid(shape, dt, halo=0, data=f)
    go = ctx.grid(shape, dt, halo=1)
    for k in (1, 2, 3, 4):
        for c0 in (0, 1):
            ref, l2_ref = _inplace_passes(ctx, u, f, dt, omega, h2, c0, k, reduce=(G.R_L2, G.RV_UPDATE))
            l2 = ctx.do_all(G.K_RBGS_TB, [gu, gf], [go], p=(omega, h2, c0, k), reduce=(G.R_L2, G.RV_UPDATE))
            assert np.array_equal(go.numpy(), ref), (k, c0)
            assert abs(l2 - l2_ref) <= 1e-12 * max(l2_ref, 1e-300) * (1 if dt == G.F64 else 1e3), (k, c0)


def test_rbgs_blocked_matches_oracle(ctx):
    shape = (12, 29, 75)
    g = np.random.default_rng(34)
    u = g.standard_normal(shape)
    f = g.standard_normal(shape)
    omega, h2 = 1.45, 0.2
    gu = ctx.grid(shape, G.F64, halo=1, data=u)
    gf = ctx.grid(shape, G.F64, halo=0, data=f)
    go = ctx.grid(shape, G.F64, halo=1)
    ctx.do_all(G.K_RBGS_TB, [gu, gf], [go], p=(omega, h2, 1, 4))
    cur = u
    for q in range(4):
        cur, _, _ = oracle.rbgs_pass(cur, f, omega, h2, (1 + q) % 2, 0.0)
    scale = 8 * np.abs(u).max() + h2 * np.abs(f).max()
    assert np.abs(go.numpy() - cur).max() <= 4e-14 * scale


def test_rbgs_blocked_errors(ctx):
    shape = (6, 7, 40)
    gu = ctx.grid(shape, G.F64, halo=1).fill(1.0)
    go = ctx.grid(shape, G.F64, halo=1)

    def err(fn):
        with pytest.raises(G.GsclError) as e:
            fn()
        return e.value.code

    assert err(lambda: ctx.do_all(G.K_RBGS_TB, [gu], [go], p=(1.0, 1.0, 2, 2))) == G.ERR_ARG
    assert err(lambda: ctx.do_all(G.K_RBGS_TB, [gu], [go], p=(1.0, 1.0, 0, 5))) == G.ERR_ARG
    assert err(lambda: ctx.do_all(G.K_RBGS_TB, [gu], [go], p=(1.0, 1.0, 0, 1.5))) == G.ERR_ARG
    assert err(lambda: ctx.do_all(G.K_RBGS_TB, [gu], [go], p=(1.0, 0.0, 0, 2))) == G.ERR_ARG
    assert err(lambda: ctx.do_all(G.K_RBGS_TB, [gu], [gu], p=(1.0, 1.0, 0, 2))) == G.ERR_ALIAS
    assert err(lambda: ctx.do_all(G.K_RBGS_TB, [gu, go], [go], p=(1.0, 1.0, 0, 2))) == G.ERR_ALIAS
    gp = ctx.grid(shape, G.F64, halo=1, bc=G.PERIODIC).fill(1.0)
    gq = ctx.grid(shape, G.F64, halo=1, bc=G.PERIODIC)
    assert err(lambda: ctx.do_all(G.K_RBGS_TB, [gp], [gq], p=(1.0, 1.0, 0, 2))) == G.ERR_UNSUPPORTED
    g8 = ctx.grid(shape, G.U8, halo=1)
    h8 = ctx.grid(shape, G.U8, halo=1)
    assert err(lambda: ctx.do_all(G.K_RBGS_TB, [g8], [h8], p=(1.0, 1.0, 0, 2))) == G.ERR_DTYPE


@pytest.mark.parametrize("n,S", [(150, 6), (146, 4), (75, 6)])
def test_blocked_sor_solve_equals_inplace_solve(sctx, n, S):
    """Grids of 72^3 points or more run the SOR chunks as blocked passes
    (2S colour passes: S = 6 -> 4+4+2+2, S = 4 -> 4+4): the same stopping
    sweep and the same iterate, bit for bit, as in-place colour passes with
    the same residual checks, and the oracle accepts the answer."""
    ctx = sctx
    req = W.poisson_requests(count=1, qps=float("inf"), nmin=n, nmax=n, seed_index=n)[0]
    _, f = W.poisson_fields(req)
    gf = ctx.grid(f.shape, G.F64, halo=0, data=f)
    u = ctx.grid(f.shape, G.F64, halo=1).fill(0.0)
    st = ctx.solve(G.K_RBGS, [u], [gf], omega=0.0, h2=req.h2, rtol=1e-8, check_every=S)
    w = _opt_omega(n)
    v = ctx.grid(f.shape, G.F64, halo=1).fill(0.0)
    r = ctx.grid(f.shape, G.F32, halo=0)
    fn2 = oracle.sumsq(f)
    sweeps = 0
    while True:
        for q in range(2 * S):
            ctx.do_all(G.K_RBGS, [v, gf], [v], p=(w, req.h2, q % 2))
        sweeps += S
        res2 = ctx.do_all(G.K_POISSON_RESID, [v, gf], [r], p=(0.0, req.h2), reduce=(G.R_SUMSQ, G.RV_RESIDUAL))
        if math.sqrt(res2 / fn2) <= 1e-8:
            break
        assert sweeps < 20000
    assert st["sweeps"] == sweeps
    got = u.numpy()
    assert np.array_equal(got, v.numpy())
    _, _, res = oracle.wjacobi_sweep(got, f, 1.0, req.h2)
    assert math.sqrt(oracle.sumsq(res) / fn2) <= 1e-8 * 1.0001
