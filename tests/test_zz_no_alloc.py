"""GPU check of the allocation-free do_all (gscl_do_all_noalloc) against
gscl_do_all: same kernels, so outputs and fused reductions must agree bit for
bit; both are also held to the oracle's bars.  Two calls in a row, the second
on a smaller grid, so the fixed scratch keeps the first call's partials when
the second one runs."""
import math

import numpy as np
import pytest

import oracle
import paper_1207_1746_amd as G
from paper_1207_1746_amd import workloads as W

pytestmark = pytest.mark.gpu


def _varcoef_pair(ctx, n):
    u, c, s = W.varcoef_grids(*n)
    shp = u.shape
    gu = ctx.grid(shp, G.F32, halo=1, bc=G.PERIODIC, data=u)
    gc = [ctx.grid(shp, G.F32, halo=0, data=x) for x in c]
    gs = ctx.grid(shp, G.F32, halo=0, data=s)
    ins = [gu] + gc + [gs]
    out_a = [ctx.grid(shp, G.F32, halo=1) for _ in range(3)]
    out_b = [ctx.grid(shp, G.F32, halo=1) for _ in range(3)]
    ra = ctx.do_all(G.K_VARCOEF7, ins, out_a, reduce=(G.R_L2, G.RV_RESIDUAL))
    rb = ctx.do_all(G.K_VARCOEF7, ins, out_b, reduce=(G.R_L2, G.RV_RESIDUAL), noalloc=True)
    return (u, c, s), out_a, out_b, ra, rb


@pytest.mark.parametrize("sizes", [((96, 80, 72), (40, 24, 12))])
def test_noalloc_varcoef_matches_do_all_twice(ctx, sizes):
    for n in sizes:  # second call smaller than the first
        (u, c, s), out_a, out_b, ra, rb = _varcoef_pair(ctx, n)
        for x, y in zip(out_a, out_b):
            assert np.array_equal(x.numpy(), y.numpy()), f"outputs differ at {n}"
        assert ra == rb, f"fused norms differ at {n}: {ra!r} vs {rb!r}"
        un, ro, fo = oracle.varcoef7_sweep(u, c, s)
        tol = 16 * 2.0 ** -24 * (7 * np.abs(u).max() + 1)
        for o, e in zip(out_b, (un, ro, fo)):
            assert np.abs(o.numpy() - e).max() <= tol
        rref = math.sqrt(oracle.sumsq(ro))
        assert abs(rb - rref) <= math.sqrt(ro.size) * tol


def test_noalloc_wjacobi_f64_update_norm_twice(ctx):
    for n in ((70, 66, 64), (21, 17, 13)):
        u0, h2 = W.jacobi_cube(*n)
        src = ctx.grid(u0.shape, G.F64, halo=1, data=u0)
        a = ctx.grid(u0.shape, G.F64, halo=1)
        b = ctx.grid(u0.shape, G.F64, halo=1)
        ra = ctx.do_all(G.K_WJACOBI, [src], [a], p=(1.0, h2), reduce=(G.R_L2, G.RV_UPDATE))
        rb = ctx.do_all(G.K_WJACOBI, [src], [b], p=(1.0, h2), reduce=(G.R_L2, G.RV_UPDATE), noalloc=True)
        assert np.array_equal(a.numpy(), b.numpy())
        assert ra == rb
        uo, l2, _ = oracle.jacobi_run(u0, 1, None, 1.0, h2)
        assert np.abs(b.numpy() - uo).max() <= 1e-12 * np.abs(u0).max()
        assert abs(rb - l2) <= 1e-12 * l2


def test_noalloc_device_result_and_plain_sweep(ctx):
    import torch
    u0, h2 = W.jacobi_cube(33, 31, 29)
    src = ctx.grid(u0.shape, G.F64, halo=1, data=u0)
    a = ctx.grid(u0.shape, G.F64, halo=1)
    b = ctx.grid(u0.shape, G.F64, halo=1)
    dres = torch.zeros(2, dtype=torch.float64, device="cuda")
    ctx.do_all(G.K_WJACOBI, [src], [a], p=(0.8, h2), reduce=(G.R_MAXABS, G.RV_UPDATE), dev_result=dres[0:1])
    ctx.do_all(G.K_WJACOBI, [src], [b], p=(0.8, h2), reduce=(G.R_MAXABS, G.RV_UPDATE), dev_result=dres[1:2],
               noalloc=True)
    torch.cuda.synchronize()
    assert np.array_equal(a.numpy(), b.numpy())
    assert dres[0].item() == dres[1].item() and dres[0].item() > 0
    # no reduction: nothing touches the scratch, outputs still equal
    ctx.do_all(G.K_WJACOBI, [src], [a], p=(0.8, h2))
    ctx.do_all(G.K_WJACOBI, [src], [b], p=(0.8, h2), noalloc=True)
    assert np.array_equal(a.numpy(), b.numpy())


def test_noalloc_rejects_reduction_beyond_fixed_scratch(ctx):
    # LINEAR with a fused reduction uses one block per 64 x 4 x 1 tile:
    # 1 x 64 x 1100 = 70400 blocks > GSCL_NOALLOC_PARTIALS
    shape = (1100, 256, 64)
    u = ctx.grid(shape, G.F32, halo=0).fill(1.0)
    o = ctx.grid(shape, G.F32, halo=0)
    terms = [(0, 0, 0, 0, 0, 2.0, -1)]
    with pytest.raises(G.GsclError) as ei:
        ctx.do_all(G.K_LINEAR, [u], [o], terms=terms, reduce=(G.R_SUM, G.RV_OUT0), noalloc=True)
    assert ei.value.code == G.ERR_NOMEM
    # the same call through gscl_do_all grows its own scratch and succeeds
    r = ctx.do_all(G.K_LINEAR, [u], [o], terms=terms, reduce=(G.R_SUM, G.RV_OUT0))
    assert r == 2.0 * 1100 * 256 * 64
