"""C-ABI behaviour on the GPU: host-side validation (Section 3 semantics: an
operator reads fixed offsets within the halo and writes the core element, so
an output may not alias a grid read at offsets), the context phases of
Section 4 / Fig. 2b, and HIP-graph capture of library launches replayed
several times with eager work in between.
"""
import numpy as np
import pytest

import oracle
import paper_1207_1746_amd as G

pytestmark = pytest.mark.gpu


def _err(fn):
    with pytest.raises(G.GsclError) as e:
        fn()
    return e.value.code


def test_validation_errors(ctx):
    shp = (6, 7, 40)
    u = ctx.grid(shp, G.F64, halo=1).fill(1.0)
    v = ctx.grid(shp, G.F64, halo=1)
    # output aliasing a grid read at offsets
    assert _err(lambda: ctx.do_all(G.K_WJACOBI, [u], [u], p=(1.0, 1.0))) == G.ERR_ALIAS
    # halo too small for the operator's offsets
    u0 = ctx.grid(shp, G.F64, halo=0).fill(1.0)
    assert _err(lambda: ctx.do_all(G.K_WJACOBI, [u0], [v], p=(1.0, 1.0))) == G.ERR_HALO
    # dtype not accepted / mixed
    w32 = ctx.grid(shp, G.F32, halo=1)
    assert _err(lambda: ctx.do_all(G.K_WJACOBI, [u], [w32], p=(1.0, 1.0))) == G.ERR_DTYPE
    # extents differ
    other = ctx.grid((6, 7, 41), G.F64, halo=1)
    assert _err(lambda: ctx.do_all(G.K_WJACOBI, [u], [other], p=(1.0, 1.0))) == G.ERR_SHAPE
    # LINEAR: pointwise in-place update is allowed, offset read in place is not
    ctx.do_all(G.K_LINEAR, [u], [u], terms=[(0, 0, 0, 0, 0, 2.0, -1)])
    assert np.all(u.numpy() == 2.0)
    assert _err(lambda: ctx.do_all(G.K_LINEAR, [u], [u], terms=[(0, 0, 1, 0, 0, 1.0, -1)])) == G.ERR_ALIAS
    # term referring to a missing grid, dz in 2D
    assert _err(lambda: ctx.do_all(G.K_LINEAR, [u], [v], terms=[(0, 3, 0, 0, 0, 1.0, -1)])) == G.ERR_ARG
    g2 = ctx.grid((3, 7, 40), G.F64, halo=1, ndim=2)
    h2 = ctx.grid((3, 7, 40), G.F64, halo=1, ndim=2)
    assert _err(lambda: ctx.do_all(G.K_LINEAR, [g2], [h2], terms=[(0, 0, 0, 0, 1, 1.0, -1)])) == G.ERR_ARG
    # image kernel needs the clamp rule and U8 -> U8, I16
    img = ctx.grid((1, 8, 16), G.U8, halo=2, ndim=2)
    b8 = ctx.grid((1, 8, 16), G.U8, halo=0, ndim=2)
    l16 = ctx.grid((1, 8, 16), G.I16, halo=0, ndim=2)
    assert _err(lambda: ctx.do_all(G.K_IMG_BOX5_LAP, [img], [b8, l16], p=(4,))) == G.ERR_ARG
    # unsupported field count for the 13-point kinds
    outs3 = [ctx.grid(shp, G.F64, halo=0) for _ in range(3)]
    assert _err(lambda: ctx.do_all(G.K_VC13_APPLY, [u] * 13, outs3, p=(0.25, 0, 3))) == G.ERR_UNSUPPORTED
    # outputs may not overlap each other
    assert _err(lambda: ctx.do_all(G.K_LINEAR, [u], [v, v], terms=[(0, 0, 0, 0, 0, 1.0, -1)])) == G.ERR_ALIAS


def test_context_phases():
    import torch
    c = G.Context(0)
    g = c.grid((4, 4, 16), G.F64, halo=1).fill(1.0)
    o = c.grid((4, 4, 16), G.F64, halo=1)
    c.do_all(G.K_WJACOBI, [g], [o], p=(1.0, 1.0))
    c.end()
    # after end the host may read the grids; iteration spaces are an error
    assert o.numpy()[2, 2, 8] == 1.0
    assert _err(lambda: c.do_all(G.K_WJACOBI, [g], [o], p=(1.0, 1.0))) == G.ERR_STATE
    assert _err(lambda: c.do_reduce(G.R_SUM, g)) == G.ERR_STATE
    c.begin()  # a context may be re-entered
    assert c.do_reduce(G.R_SUM, g) == 4 * 4 * 16
    c.end()
    c.finalize()
    torch.cuda.synchronize()


def test_graph_capture_replays_match_eager(sctx):
    ctx = sctx
    import torch
    shp = (12, 20, 70)
    u0 = np.random.default_rng(1).standard_normal(shp)
    a = ctx.grid(shp, G.F64, halo=1, data=u0)
    b = ctx.grid(shp, G.F64, halo=1)
    res = torch.zeros(4, dtype=torch.float64, device="cuda")
    ctx.reserve(int(np.prod(shp)))
    ctx.graph_begin()
    for k in range(4):
        src, dst = (a, b) if k % 2 == 0 else (b, a)
        ctx.do_all(G.K_WJACOBI, [src], [dst], p=(0.9, 1.0), reduce=(G.R_L2, G.RV_UPDATE), dev_result=res[k])
    graph = ctx.graph_end()
    u = u0
    for rep in range(3):
        graph.launch()
        got = a.numpy()
        norms = res.cpu().numpy()
        for k in range(4):
            u, upd, _ = oracle.wjacobi_sweep(u, None, 0.9, 1.0)
            assert abs(norms[k] - np.sqrt(oracle.sumsq(upd))) <= 1e-12 * norms[k]
        np.testing.assert_allclose(got, u, rtol=0, atol=1e-13 * np.abs(u0).max())
        # eager work between replays: one sweep forward and back through a scratch grid
        tmp = ctx.grid(shp, G.F64, halo=1)
        ctx.do_all(G.K_LINEAR, [a], [tmp], terms=[(0, 0, 0, 0, 0, 1.0, -1)])
        torch.cuda.synchronize()
    graph.close()


def test_vc13_five_fields_refuse_grids_of_4_gib(ctx):
    """The five-field 13-point kernels address grids with 32-bit byte offsets:
    a grid of 4 GiB or more is refused on the host, before any launch.  The
    FP64 residual kind has the smallest footprint for a 4 GiB grid (FP64 x and
    b, BF16 coefficients, F32 outputs: about 65 GB, left uninitialized)."""
    import torch
    shape = (513, 1024, 1024)  # 4.3 GB per FP64 grid
    x = [ctx.grid(shape, G.F64, halo=2) for _ in range(5)]
    b = [ctx.grid(shape, G.F64, halo=0) for _ in range(5)]
    c = [ctx.grid(shape, G.BF16, halo=0) for _ in range(10)]
    r = [ctx.grid(shape, G.F32, halo=0) for _ in range(5)]
    assert x[0].storage.numel() * 8 >= 1 << 32
    assert _err(lambda: ctx.do_all(G.K_VC13_RESID, x + b + c, r, p=(0.25, 0.0, 5))) == G.ERR_UNSUPPORTED
    del x, b, c, r
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
