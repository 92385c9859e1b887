"""GPU parity: the 9-in / 3-out variable-coefficient sweep and the fourth-order
13-point multi-field operators against the FP64 oracle.

FP32 bound (derived from the arithmetic): one sweep computes u' with at most 16
roundings of relative size 2^-24 on terms bounded by (sum |c_k u_k| + |s|)/C;
the sweep map is a convex combination (infinity-norm 1), so after n sweeps
||u_gpu - u_oracle||_inf <= sum_n 16 * 2^-24 * (||u_n||_inf + ||s/C||_inf).
Low-precision storage (cfg: 13-point): a single apply is within
4 * u_s * (sum of |terms|) of FP64, u_s = 2^-8 (BF16), 2^-11 (F16), 2^-24 (F32).
"""
import numpy as np
import pytest

import oracle
import paper_1207_1746_amd as G
from paper_1207_1746_amd import workloads as W

pytestmark = pytest.mark.gpu
U32 = 2.0 ** -24


def _vc_grids(ctx, shape, dt, u, c, s, bc=G.PERIODIC):
    gu = ctx.grid(shape, dt, halo=1, bc=bc, data=u)
    gc = [ctx.grid(shape, dt, halo=0, data=x) for x in c]
    gs = ctx.grid(shape, dt, halo=0, data=s)
    outs = [ctx.grid(shape, dt, halo=1, bc=bc) for _ in range(3)]
    return gu, gc, gs, outs


@pytest.mark.parametrize("shape", [(8, 8, 8), (21, 37, 53), (5, 9, 300), (33, 17, 256)])
def test_varcoef_one_sweep_f64(ctx, shape):
    u, c, s = W.varcoef_grids(shape[2], shape[1], shape[0])
    u, c, s = u.astype(np.float64), [x.astype(np.float64) for x in c], s.astype(np.float64)
    gu, gc, gs, outs = _vc_grids(ctx, shape, G.F64, u, c, s)
    l2 = ctx.do_all(G.K_VARCOEF7, [gu] + gc + [gs], outs, reduce=(G.R_L2, G.RV_RESIDUAL))
    ex = oracle.varcoef7_sweep(u, c, s)
    scale = np.abs(u).max() * 7 + 1
    for o, e in zip(outs, ex):
        np.testing.assert_allclose(o.numpy(), e, rtol=0, atol=1e-12 * scale)
    assert abs(l2 - np.sqrt(oracle.sumsq(ex[1]))) <= 1e-12 * l2


@pytest.mark.parametrize("shape", [(21, 37, 53), (16, 32, 256)])
def test_varcoef_one_sweep_f32(ctx, shape):
    u, c, s = W.varcoef_grids(shape[2], shape[1], shape[0])
    gu, gc, gs, outs = _vc_grids(ctx, shape, G.F32, u, c, s)
    ctx.do_all(G.K_VARCOEF7, [gu] + gc + [gs], outs)
    un, r, fm = oracle.varcoef7_sweep(u, c, s)
    C = sum(x.astype(np.float64) for x in c)
    T = sum(np.abs(ck.astype(np.float64)) for ck in c) * np.abs(u).max() + np.abs(s)
    np.testing.assert_array_less(np.abs(un - outs[0].numpy()), 16 * U32 * T / C + 1e-30)
    np.testing.assert_array_less(np.abs(r - outs[1].numpy()), 16 * U32 * (T + C * np.abs(u).max()) + 1e-30)
    np.testing.assert_array_less(np.abs(fm - outs[2].numpy()), 16 * U32 * (T + C * np.abs(u).max()) + 1e-30)


def _run_gpu(ctx, shape, u, c, s, nsweeps, every):
    gu, gc, gs, outs = _vc_grids(ctx, shape, G.F32, u, c, s)
    ping = [gu, outs[0]]
    norms = []
    for n in range(1, nsweeps + 1):
        src, dst = ping[(n - 1) % 2], ping[n % 2]
        red = (G.R_L2, G.RV_RESIDUAL) if n % every == 0 else None
        r = ctx.do_all(G.K_VARCOEF7, [src] + gc + [gs], [dst, outs[1], outs[2]], reduce=red)
        if red:
            norms.append(r)
    return ping[nsweeps % 2], outs, norms


@pytest.mark.parametrize("shape,nsweeps", [((64, 64, 64), 100), ((256, 256, 256), 20)])
def test_varcoef_multi_sweep_f32_bound(ctx, shape, nsweeps):
    u, c, s = W.varcoef_grids(shape[2], shape[1], shape[0])
    res_u, outs, norms = _run_gpu(ctx, shape, u, c, s, nsweeps, 10)
    # oracle trajectory and the a-priori bound built from it
    x = u.astype(np.float64)
    cp = np.ascontiguousarray(np.stack([ci.astype(np.float64) for ci in c]))
    sd = s.astype(np.float64)
    sC = np.abs(sd / cp.sum(axis=0)).max()
    bound = 0.0
    onorms = []
    r = None
    for n in range(1, nsweeps + 1):
        bound += 16 * U32 * (np.abs(x).max() + sC)
        x, r, _ = oracle.varcoef7_sweep(x, cp, sd)
        if n % 10 == 0:
            onorms.append(np.sqrt(oracle.sumsq(r)))
    err = np.abs(res_u.numpy() - x).max()
    assert err <= bound, (err, bound)
    # residual grids: r = s + out - C u, so |dr| <= 2 C_max |du| + rounding
    rb = 2 * 7 * bound + 16 * U32 * (7 * np.abs(x).max() + 1)
    assert np.abs(outs[1].numpy() - r).max() <= rb
    npts = np.prod(shape)
    for a, b in zip(norms, onorms):
        assert abs(a - b) <= np.sqrt(npts) * rb


@pytest.mark.parametrize("dt,us", [(G.F64, 1e-16), (G.F32, U32), (G.F16, 2.0 ** -11), (G.BF16, 2.0 ** -8)])
@pytest.mark.parametrize("nf", [1, 5])
def test_vc13_apply_per_dtype(ctx, dt, us, nf):
    shape = (11, 19, 150)
    c, _ = W.vc13_grids(shape[2], shape[1], shape[0])
    fields = W.vc13_fields(shape[2], shape[1], shape[0], nf)
    gf = [ctx.grid(shape, dt, halo=2, data=f) for f in fields]
    gc = [ctx.grid(shape, dt, halo=0, data=x) for x in c]
    go = [ctx.grid(shape, dt, halo=0) for _ in range(nf)]
    ctx.do_all(G.K_VC13_APPLY, gf + gc, go, p=(W.VC13_KAPPA, 0.0, nf))
    for f in range(nf):
        stored = gf[f].view.double().cpu().numpy()
        ex = oracle.vc13_apply(stored, c, W.VC13_KAPPA)
        terms = 1.5 * np.abs(stored).max() * (1 + W.VC13_KAPPA * 3 * (4 / 3 * 2 * 2 + 4 / 12))
        tol = 4 * us * max(np.abs(ex).max(), 1.0) + 64 * (U32 if dt != G.F64 else 1e-16) * terms
        got = go[f].view.double().cpu().numpy()
        assert np.abs(got - ex).max() <= tol, (dt, f)


@pytest.mark.parametrize("dt", [G.F64, G.F32, G.BF16])
def test_vc13_jacobi_and_resid(ctx, dt):
    shape = (9, 13, 70)
    nf = 5
    c, b = W.vc13_grids(shape[2], shape[1], shape[0], nf)
    d0 = W.vc13_fields(shape[2], shape[1], shape[0], nf)
    gd = [ctx.grid(shape, dt, halo=2, data=x) for x in d0]
    gg = [ctx.grid(shape, dt, halo=0, data=x) for x in b]
    gc = [ctx.grid(shape, dt, halo=0, data=x) for x in c]
    go = [ctx.grid(shape, dt, halo=2) for _ in range(nf)]
    omega = 6 / 7
    ctx.do_all(G.K_VC13_JACOBI, gd + gg + gc, go, p=(W.VC13_KAPPA, omega, nf))
    D = oracle.vc13_diag(c, W.VC13_KAPPA)
    us = {G.F64: 1e-15, G.F32: U32, G.BF16: 2.0 ** -8}[dt]
    for f in range(nf):
        ds = gd[f].view.double().cpu().numpy()
        gs = gg[f].view.double().cpu().numpy()
        ex = ds + omega * (gs - oracle.vc13_apply(ds, c, W.VC13_KAPPA)) / D
        tol = 4 * us * np.abs(ex).max() + 256 * (U32 if dt != G.F64 else 1e-16) * (np.abs(ds).max() + np.abs(gs).max())
        assert np.abs(go[f].view.double().cpu().numpy() - ex).max() <= tol
    # F64 residual with coefficients in dt storage, fused ||r||^2 over all fields
    gx = [ctx.grid(shape, G.F64, halo=2, data=x.astype(np.float64)) for x in d0]
    gb = [ctx.grid(shape, G.F64, halo=0, data=x) for x in b]
    gr = [ctx.grid(shape, G.F32, halo=0) for _ in range(nf)]
    ss = ctx.do_all(G.K_VC13_RESID, gx + gb + gc, gr, p=(W.VC13_KAPPA, 0.0, nf), reduce=(G.R_SUMSQ, G.RV_RESIDUAL))
    tot = 0.0
    for f in range(nf):
        r = oracle.vc13_residual(d0[f].astype(np.float64), b[f], c, W.VC13_KAPPA)
        tot += oracle.sumsq(r)
        np.testing.assert_allclose(gr[f].numpy(), r, rtol=U32 * 2, atol=1e-12 * np.abs(r).max())
    assert abs(ss - tot) <= 1e-12 * tot


@pytest.mark.parametrize("dt", [G.BF16, G.F32, G.F64])
@pytest.mark.parametrize("bc", [G.DIRICHLET, G.PERIODIC, G.CLAMP])
def test_vc13_five_field_tiling_invariance(ctx, dt, bc):
    """do_all outputs of the five-field 13-point kinds are bitwise identical
    for every tile shape (ragged in x, y and z), under every boundary rule;
    the Dirichlet case with a non-zero boundary value also matches the oracle."""
    shape = (11, 13, 150)
    nf = 5
    c, b = W.vc13_grids(shape[2], shape[1], shape[0], nf)
    fields = W.vc13_fields(shape[2], shape[1], shape[0], nf)
    bcv = 0.5 if bc == G.DIRICHLET else 0.0
    gf = [ctx.grid(shape, dt, halo=2, bc=bc, bc_value=bcv, data=f) for f in fields]
    gc = [ctx.grid(shape, dt, halo=0, data=x) for x in c]
    gg = [ctx.grid(shape, dt, halo=0, data=x) for x in b]
    shapes = [(1, 4, 16), (1, 6, 3), (1, 8, 1)]
    if dt != G.F64:
        shapes += [(2, 4, 3), (2, 6, 16), (2, 8, 1)]
    for kind, ins, p in ((G.K_VC13_APPLY, gf + gc, (W.VC13_KAPPA, 0.0, nf)),
                         (G.K_VC13_JACOBI, gf + gg + gc, (W.VC13_KAPPA, 6 / 7, nf))):
        ref = None
        for t in shapes:
            ctx.tile_set(kind, gf[0], t)
            go = [ctx.grid(shape, dt, halo=2) for _ in range(nf)]
            ctx.do_all(kind, ins, go, p=p)
            got = np.stack([o.view.double().cpu().numpy() for o in go])
            if ref is None:
                ref = got
            assert np.array_equal(got, ref), (kind, t)
        ctx.tile_clear()
        if bc == G.DIRICHLET and kind == G.K_VC13_APPLY:
            us = {G.F64: 1e-16, G.F32: U32, G.BF16: 2.0 ** -8}[dt]
            for f in range(nf):
                stored = gf[f].view.double().cpu().numpy()
                ex = oracle.vc13_apply(stored, c, W.VC13_KAPPA, bcv=bcv)
                terms = 1.5 * max(np.abs(stored).max(), bcv) * (1 + W.VC13_KAPPA * 3 * (4 / 3 * 2 * 2 + 4 / 12))
                tol = 4 * us * max(np.abs(ex).max(), 1.0) + 64 * (U32 if dt != G.F64 else 1e-16) * terms
                assert np.abs(ref[f] - ex).max() <= tol, f


def _bits(grid):
    import torch
    v = grid.view.contiguous()
    return v.view(torch.int16 if v.element_size() == 2 else torch.int32).cpu().numpy()


@pytest.mark.parametrize("dt", [G.BF16, G.F16, G.F32])
@pytest.mark.parametrize("nf,scale", [(5, 1.0), (5, 0.37), (1, 3.0)])
def test_vc13_jacobi0_equals_sweep_of_zero(ctx, dt, nf, scale):
    """The fused first sweep of a zero correction: g is the scaled residual
    rounded to the storage type (as the host rounds FP64 -> FP32 -> storage),
    and d equals a VC13_JACOBI sweep of a zero d with right-hand side g bit
    for bit (ragged row: nx = 70)."""
    import torch
    shape = (9, 13, 70)
    c, _ = W.vc13_grids(shape[2], shape[1], shape[0], nf)
    rng = np.random.default_rng(11)
    r = [rng.standard_normal(shape).astype(np.float32) for _ in range(nf)]
    gr = [ctx.grid(shape, G.F32, halo=0, data=x) for x in r]
    gc = [ctx.grid(shape, dt, halo=0, data=x) for x in c]
    gg = [ctx.grid(shape, dt, halo=0) for _ in range(nf)]
    gd = [ctx.grid(shape, dt, halo=0) for _ in range(nf)]
    omega = 6 / 7
    ctx.do_all(G.K_VC13_JACOBI0, gr + gc, gg + gd, p=(W.VC13_KAPPA, omega, nf, scale))
    tdt = {G.BF16: torch.bfloat16, G.F16: torch.float16, G.F32: torch.float32}[dt]
    for f in range(nf):
        host = torch.from_numpy((scale * r[f].astype(np.float64)).astype(np.float32)).to(tdt)
        assert torch.equal(gg[f].view.cpu(), host), f
    z = [ctx.grid(shape, dt, halo=2).fill(0.0) for _ in range(nf)]
    o = [ctx.grid(shape, dt, halo=0) for _ in range(nf)]
    ctx.do_all(G.K_VC13_JACOBI, z + gg + gc, o, p=(W.VC13_KAPPA, omega, nf))
    for f in range(nf):
        assert np.array_equal(_bits(gd[f]), _bits(o[f])), f
    # d = omega g / D against the oracle's diagonal: FP32 forms D from ten
    # rounded terms, omega / D and the product (<= 16 roundings of 2^-24),
    # then d is rounded once to the storage type
    D = oracle.vc13_diag(c, W.VC13_KAPPA)
    us = {G.F32: U32, G.F16: 2.0 ** -11, G.BF16: 2.0 ** -8}[dt]
    for f in range(nf):
        g64 = gg[f].view.double().cpu().numpy()
        ex = omega * g64 / D
        assert np.abs(gd[f].view.double().cpu().numpy() - ex).max() <= (us + 16 * U32) * np.abs(ex).max()


def test_vc13_jacobi0_errors(ctx):
    shape = (4, 5, 6)
    c, _ = W.vc13_grids(6, 5, 4, 1)
    gr = [ctx.grid(shape, G.F32, halo=0)]
    gc = [ctx.grid(shape, G.BF16, halo=0, data=x) for x in c]
    gg = ctx.grid(shape, G.BF16, halo=0)
    gd = ctx.grid(shape, G.BF16, halo=0)
    p = (W.VC13_KAPPA, 6 / 7, 1, 1.0)
    for ins, outs, code in ((gr + gc, [gg], G.ERR_ARG),                   # one output missing
                            (gc[:1] + gc, [gg, gd], G.ERR_DTYPE),          # residual not F32
                            (gr + gc, [gg, gc[0]], G.ERR_ALIAS)):          # output is an input
        with pytest.raises(G.GsclError) as e:
            ctx.do_all(G.K_VC13_JACOBI0, ins, outs, p=p)
        assert e.value.code == code
