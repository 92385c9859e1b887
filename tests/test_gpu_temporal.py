"""Temporal blocking (k weighted-Jacobi sweeps per pass, Section 2's wide ghost
areas): the result must be the one k separate sweeps give, bit for bit, under
every supported boundary rule, at ragged sizes that leave partial tiles in x,
y and z; it is also checked against k applications of the oracle's sweep,
with the fused reduction of the last sweep."""
import numpy as np
import pytest

import oracle
import paper_1207_1746_amd as G

pytestmark = pytest.mark.gpu


def _plain(ctx, u, f, k, omega, h2, dt, bc, bcv):
    shape = u.shape
    a = ctx.grid(shape, dt, halo=1, bc=bc, bc_value=bcv, data=u)
    b = ctx.grid(shape, dt, halo=1, bc=bc, bc_value=bcv)
    ins_f = [ctx.grid(shape, dt, halo=0, data=f)] if f is not None else []
    for _ in range(k):
        ctx.do_all(G.K_WJACOBI, [a] + ins_f, [b], p=(omega, h2))
        a, b = b, a
    return a.view.clone()


@pytest.mark.parametrize("dt", [G.F64, G.F32])
@pytest.mark.parametrize("bc", [G.DIRICHLET, G.PERIODIC])
@pytest.mark.parametrize("with_f", [False, True])
def test_tb_equals_k_plain_sweeps_bitwise(ctx, dt, bc, with_f):
    import torch
    shape = (13, 37, 75)
    g = np.random.default_rng(21)
    u = g.standard_normal(shape)
    f = g.standard_normal(shape) if with_f else None
    omega, h2 = 0.8, 0.25
    bcv = 0.5 if bc == G.DIRICHLET else 0.0
    gu = ctx.grid(shape, dt, halo=1, bc=bc, bc_value=bcv, data=u)
    gf = [ctx.grid(shape, dt, halo=0, data=f)] if with_f else []
    for k in (1, 2, 3, 4):
        ref = _plain(ctx, u, f, k, omega, h2, dt, bc, bcv)
        for cz in (1, 3, 16):
            ctx.tile_set(G.K_WJACOBI_TB, gu, (1, 16, cz))
            go = ctx.grid(shape, dt, halo=1)
            ctx.do_all(G.K_WJACOBI_TB, [gu] + gf, [go], p=(omega, h2, k))
            assert torch.equal(go.view, ref), (k, cz)
    ctx.tile_clear()


@pytest.mark.parametrize("k", [2, 4])
def test_tb_matches_oracle_with_fused_reduction(ctx, k):
    shape = (20, 30, 90)
    g = np.random.default_rng(22)
    u = g.standard_normal(shape)
    f = g.standard_normal(shape)
    omega, h2 = 6 / 7, 1.0 / 31 ** 2
    gu = ctx.grid(shape, G.F64, halo=1, data=u)
    gf = ctx.grid(shape, G.F64, halo=0, data=f)
    go = ctx.grid(shape, G.F64, halo=1)
    r_upd = ctx.do_all(G.K_WJACOBI_TB, [gu, gf], [go], p=(omega, h2, k), reduce=(G.R_L2, G.RV_UPDATE))
    r_res = ctx.do_all(G.K_WJACOBI_TB, [gu, gf], [go], p=(omega, h2, k), reduce=(G.R_L2, G.RV_RESIDUAL))
    x = u
    for _ in range(k):
        prev = x
        x, upd, res = oracle.wjacobi_sweep(prev, f, omega, h2)
    scale = np.abs(u).max() + h2 * np.abs(f).max()
    np.testing.assert_allclose(go.numpy(), x, rtol=0, atol=1e-13 * scale * k)
    assert abs(r_upd - np.sqrt(oracle.sumsq(upd))) <= 1e-11 * r_upd
    assert abs(r_res - np.sqrt(oracle.sumsq(res))) <= 1e-11 * r_res


def test_tb_errors(ctx):
    shape = (6, 7, 40)
    gu = ctx.grid(shape, G.F64, halo=1).fill(1.0)
    gf = ctx.grid(shape, G.F64, halo=0).fill(0.0)
    go = ctx.grid(shape, G.F64, halo=1)

    def err(fn):
        with pytest.raises(G.GsclError) as e:
            fn()
        return e.value.code

    assert err(lambda: ctx.do_all(G.K_WJACOBI_TB, [gu], [go], p=(1.0, 1.0, 5))) == G.ERR_ARG
    assert err(lambda: ctx.do_all(G.K_WJACOBI_TB, [gu], [go], p=(1.0, 1.0, 0))) == G.ERR_ARG
    assert err(lambda: ctx.do_all(G.K_WJACOBI_TB, [gu, gf], [gf], p=(1.0, 1.0, 2))) == G.ERR_ALIAS
    assert err(lambda: ctx.do_all(G.K_WJACOBI_TB, [gu], [gu], p=(1.0, 1.0, 2))) == G.ERR_ALIAS
    gc = ctx.grid(shape, G.F64, halo=1, bc=G.CLAMP).fill(1.0)
    assert err(lambda: ctx.do_all(G.K_WJACOBI_TB, [gc], [go], p=(1.0, 1.0, 2))) == G.ERR_UNSUPPORTED
    g2 = ctx.grid((3, 7, 40), G.F64, halo=1, ndim=2)
    h2 = ctx.grid((3, 7, 40), G.F64, halo=1, ndim=2)
    assert err(lambda: ctx.do_all(G.K_WJACOBI_TB, [g2], [h2], p=(1.0, 1.0, 2))) == G.ERR_SHAPE


@pytest.mark.parametrize("dt,k", [(G.F64, 4), (G.F64, 3), (G.F32, 4), (G.F32, 2)])
def test_tb_full_size_512_bitwise(ctx, dt, k):
    """512^3 with a right-hand side, default tile, k levels against k sweeps
    (FP64 k = 3 and FP32 k = 4 march in two-step groups)."""
    import torch
    n = 512
    shape = (n, n, n)
    tt = torch.float64 if dt == G.F64 else torch.float32
    gu = ctx.grid(shape, dt, halo=1)
    gf = ctx.grid(shape, dt, halo=0)
    gen = torch.Generator(device="cuda").manual_seed(5)
    gu.view.copy_(torch.randn(shape, dtype=tt, device="cuda", generator=gen))
    gf.view.copy_(torch.randn(shape, dtype=tt, device="cuda", generator=gen))
    a = ctx.grid(shape, dt, halo=1)
    b = ctx.grid(shape, dt, halo=1)
    a.view.copy_(gu.view)
    h2 = 1.0 / (n + 1) ** 2
    for _ in range(k):
        ctx.do_all(G.K_WJACOBI, [a, gf], [b], p=(6 / 7, h2))
        a, b = b, a
    go = ctx.grid(shape, dt, halo=1)
    ctx.do_all(G.K_WJACOBI_TB, [gu, gf], [go], p=(6 / 7, h2, k))
    assert torch.equal(go.view, a.view)


def test_tb_refuses_planes_of_4_gib(ctx):
    """The blocked kernels address a point within its plane by a 32-bit byte
    offset: an FP64 plane of 23200 x 23200 points (4.3 GB) is refused before
    any launch.  (The grids, one plane each, are allocated, never written.)"""
    import torch
    shape = (1, 23200, 23200)
    gu = ctx.grid(shape, G.F64, halo=1)
    go = ctx.grid(shape, G.F64, halo=1)
    for kind, p in ((G.K_WJACOBI_TB, (1.0, 1.0, 2)), (G.K_RBGS_TB, (1.0, 1.0, 0, 2))):
        with pytest.raises(G.GsclError) as e:
            ctx.do_all(kind, [gu], [go], p=p)
        assert e.value.code == G.ERR_SHAPE
    del gu, go
    torch.cuda.empty_cache()


@pytest.mark.parametrize("bc", [G.DIRICHLET, G.PERIODIC])
def test_tb_64bit_plane_offsets_bitwise(ctx, bc):
    """Plane offsets that do not fit 32 bits take the kernel with 64-bit
    offsets: an FP32 grid of 9 planes 2^29 elements apart (the last plane at
    element 2^32) against k plain sweeps, bit for bit; under the periodic rule
    the wrapped plane below the first is that last plane.  (Four 18 GB
    allocations; only each plane's first rows are written.)"""
    import torch
    shape = (9, 8, 64)
    pitch = (64, 1 << 29)
    g = np.random.default_rng(29)
    u = g.standard_normal(shape)
    omega, h2 = 0.8, 0.25
    bcv = 0.5 if bc == G.DIRICHLET else 0.0
    grids = [ctx.grid(shape, G.F32, halo=1, bc=bc, bc_value=bcv, pitch=pitch) for _ in range(4)]
    gu, go, a, b = grids
    gu.upload(u)
    for k in (3, 4):
        a.upload(u)
        for _ in range(k):
            ctx.do_all(G.K_WJACOBI, [a], [b], p=(omega, h2))
            a, b = b, a
        ctx.do_all(G.K_WJACOBI_TB, [gu], [go], p=(omega, h2, k))
        assert torch.equal(go.view, a.view), k
    del grids, gu, go, a, b
    torch.cuda.empty_cache()


def test_solve_keeps_plain_sweeps_for_planes_of_4_gib(ctx):
    """A Poisson solve on a grid whose planes span 4 GiB (3 rows of 124416
    points, 2^28 + 64 elements apart) runs plain sweeps instead of blocked
    passes: it stops on the sweep limit (not on a shape error) with the
    iterate of 4 plain sweeps, bit for bit.  (About 40 GB allocated.)"""
    import torch
    shape = (1, 3, 124416)
    py = (1 << 28) + 64
    pitch = (py, 3 * py)
    g = np.random.default_rng(31)
    f = g.standard_normal(shape)
    h2 = 1e-4
    gf = ctx.grid(shape, G.F64, halo=0, pitch=pitch)
    gf.upload(f)
    gu = ctx.grid(shape, G.F64, halo=1, pitch=pitch).fill(0.0)
    with pytest.raises(G.GsclError) as e:
        ctx.solve(G.K_WJACOBI, [gu], [gf], omega=6 / 7, h2=h2, rtol=1e-30, check_every=2, max_sweeps=4)
    assert e.value.code == G.ERR_NOCONV
    a = ctx.grid(shape, G.F64, halo=1, pitch=pitch).fill(0.0)
    b = ctx.grid(shape, G.F64, halo=1, pitch=pitch)
    for _ in range(4):
        ctx.do_all(G.K_WJACOBI, [a, gf], [b], p=(6 / 7, h2))
        a, b = b, a
    assert torch.equal(gu.view, a.view)
    del gf, gu, a, b
    torch.cuda.empty_cache()


def test_tb_default_chunk_rule(ctx):
    """Default z chunk of the blocked kinds: the largest power of two up to
    (output tiles per plane) * nz / 160 in FP64 and / 320 in FP32, within
    1..64 (512^3: 10 x 22 tiles per plane at k = 4 geometry)."""
    for n, dt, cz in ((512, G.F64, 64), (512, G.F32, 64), (256, G.F64, 64), (256, G.F32, 32),
                      (192, G.F64, 32), (192, G.F32, 16), (144, G.F64, 16), (96, G.F64, 4)):
        tiles = -(-n // 56) * -(-n // 24)
        want = max(1, tiles * n // (320 if dt == G.F32 else 160))
        expect = 1
        while expect * 2 <= want and expect < 64:
            expect *= 2
        assert expect == cz, (n, dt)
        g = ctx.grid((n, n, n), dt, halo=1)
        assert ctx.tile_get(G.K_WJACOBI_TB, g) == (1, 16, cz), (n, dt)
        assert ctx.tile_get(G.K_RBGS_TB, g) == (1, 16, cz), (n, dt)
        del g
