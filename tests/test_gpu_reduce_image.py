"""GPU parity: do_reduce (Section 3) and the integer image filters (Section 1).

Reductions: exact on integer-valued data (index sums below 2^53), within
1e-12 relative of the pairwise FP64 oracle otherwise; NaN propagates through
MAXABS.  Image filters: bit-exact against the oracle.
"""
import math

import numpy as np
import pytest

import oracle
import paper_1207_1746_amd as G
from paper_1207_1746_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("shape", [(1, 1, 1), (7, 9, 37), (64, 64, 64), (3, 300, 260)])
def test_index_sum_exact(ctx, shape):
    n = int(np.prod(shape))
    idx = np.arange(n, dtype=np.float64).reshape(shape)
    g = ctx.grid(shape, G.F64, halo=0, data=idx)
    assert ctx.do_reduce(G.R_SUM, g) == n * (n - 1) / 2
    assert ctx.do_reduce(G.R_MAXABS, g) == n - 1


@pytest.mark.parametrize("dt", [G.F64, G.F32, G.F16, G.BF16])
def test_float_reductions_vs_oracle(ctx, dt):
    import torch
    shape = (17, 45, 131)
    a = np.random.default_rng(dt).standard_normal(shape)
    b = np.random.default_rng(dt + 10).standard_normal(shape)
    ga = ctx.grid(shape, dt, halo=0, data=a)
    gb = ctx.grid(shape, dt, halo=0, data=b)
    av = ga.view.double().cpu().numpy()  # the stored (rounded) values
    bv = gb.view.double().cpu().numpy()
    for op, f in ((G.R_SUM, oracle.sum), (G.R_SUMSQ, oracle.sumsq), (G.R_MAXABS, oracle.maxabs)):
        got = ctx.do_reduce(op, ga)
        ref = f(av)
        tol = 1e-12 * (oracle.sum(np.abs(av)) if op == G.R_SUM else abs(ref))
        assert abs(got - ref) <= tol
        gotd = ctx.do_reduce(op, ga, gb)
        refd = f(av - bv)
        told = 1e-12 * (oracle.sum(np.abs(av - bv)) if op == G.R_SUM else abs(refd))
        assert abs(gotd - refd) <= told
    assert abs(ctx.do_reduce(G.R_L2, ga) - math.sqrt(oracle.sumsq(av))) <= 1e-12 * math.sqrt(oracle.sumsq(av))
    m = oracle.maxabs(av)
    assert ctx.do_reduce(G.R_ALL_LE, ga, eps=m) == 1.0
    assert ctx.do_reduce(G.R_ALL_LE, ga, eps=m * 0.999) == 0.0
    del torch


def test_nan_propagates_and_integer_grids(ctx):
    shape = (4, 5, 33)
    a = np.ones(shape)
    a[2, 3, 17] = np.nan
    g = ctx.grid(shape, G.F64, halo=0, data=a)
    assert math.isnan(ctx.do_reduce(G.R_MAXABS, g))
    assert ctx.do_reduce(G.R_ALL_LE, g, eps=10.0) == 0.0
    img = W.image_planes(48, 40, 3)
    gi = ctx.grid(img.shape, G.U8, halo=0, ndim=2, data=img)
    assert ctx.do_reduce(G.R_SUM, gi) == int(img.astype(np.int64).sum())
    assert ctx.do_reduce(G.R_SUMSQ, gi) == int((img.astype(np.int64) ** 2).sum())


def test_empty_grid_reduces_to_identity(ctx):
    g = ctx.grid((0, 4, 4), G.F64, halo=0)
    assert ctx.do_reduce(G.R_SUM, g) == 0.0
    assert ctx.do_reduce(G.R_ALL_LE, g, eps=0.0) == 1.0


@pytest.mark.parametrize("shape", [(1, 37, 53), (2, 48, 64), (3, 70, 1040), (1, 5, 16), (1, 1, 1)])
@pytest.mark.parametrize("lap_kind", [4, 8])
def test_image_filters_bit_exact(ctx, shape, lap_kind):
    img = W.rng(3, 5).integers(0, 256, size=shape, dtype=np.uint8)
    gi = ctx.grid(shape, G.U8, halo=2, bc=G.CLAMP, ndim=2, data=img)
    gb = ctx.grid(shape, G.U8, halo=0, ndim=2)
    gl = ctx.grid(shape, G.I16, halo=0, ndim=2)
    ctx.do_all(G.K_IMG_BOX5_LAP, [gi], [gb, gl], p=(lap_kind,))
    box, lap = oracle.img(img, lap_kind)
    assert np.array_equal(gb.numpy(), box)
    assert np.array_equal(gl.numpy(), lap)


def test_image_full_size_four_planes(ctx):
    """4 x 8192^2 uint8, 5x5 box + 3x3 Laplacian, clamp: bit-exact."""
    img = W.image_planes(8192)
    gi = ctx.grid(img.shape, G.U8, halo=2, bc=G.CLAMP, ndim=2, data=img)
    gb = ctx.grid(img.shape, G.U8, halo=0, ndim=2)
    gl = ctx.grid(img.shape, G.I16, halo=0, ndim=2)
    ctx.do_all(G.K_IMG_BOX5_LAP, [gi], [gb, gl], p=(4,))
    box, lap = oracle.img(img, 4)
    assert np.array_equal(gb.numpy(), box)
    assert np.array_equal(gl.numpy(), lap)


def test_image_special_cases(ctx):
    img = np.zeros((1, 32, 48), np.uint8)
    img[0, 9, 20] = 255
    gi = ctx.grid(img.shape, G.U8, halo=2, bc=G.CLAMP, ndim=2, data=img)
    gb = ctx.grid(img.shape, G.U8, halo=0, ndim=2)
    gl = ctx.grid(img.shape, G.I16, halo=0, ndim=2)
    ctx.do_all(G.K_IMG_BOX5_LAP, [gi], [gb, gl], p=(4,))
    b, l = gb.numpy()[0], gl.numpy()[0]
    assert np.all(b[7:12, 18:23] == 10) and b.sum() == 250
    assert l[9, 20] == -1020 and np.count_nonzero(l) == 5


def test_reduce_512_full_size(ctx):
    """The reduction benchmark's size (512^3 FP64): the index sum is exact
    (n(n-1)/2 = 2^53 - 2^26, every partial sum an integer below 2^53), and
    the L2 norm of uniform data agrees with the pairwise oracle to 1e-12."""
    import torch
    n = 512
    shape = (n, n, n)
    g = ctx.grid(shape, G.F64, halo=0)
    g.view.copy_(torch.arange(n ** 3, dtype=torch.float64, device="cuda").reshape(shape))
    assert ctx.do_reduce(G.R_SUM, g) == float(2 ** 53 - 2 ** 26)
    assert ctx.do_reduce(G.R_MAXABS, g) == float(n ** 3 - 1)
    gen = torch.Generator(device="cuda").manual_seed(9)
    g.view.copy_(torch.rand(shape, dtype=torch.float64, device="cuda", generator=gen))
    ref = math.sqrt(oracle.sumsq(g.view.cpu().numpy()))
    assert abs(ctx.do_reduce(G.R_L2, g) - ref) <= 1e-12 * ref
