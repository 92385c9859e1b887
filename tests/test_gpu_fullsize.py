"""GPU parity at the workloads' full sizes, in the launch configuration the
benchmark uses, via checks the oracle can afford at any size.

* 13-point operator on 5 fields at 512^3: the first and last fields of the
  BF16 apply against the full FP64 oracle apply; iterative refinement with
  BF16, FP16 and FP32 storage to 1e-10 with the FP64 residual of every field
  recomputed by the oracle.
* Poisson solves at N = 192 (the largest request size): the residual trace of
  weighted Jacobi on a sum of distinct sine modes is closed form,
  ||r_n||^2 = sum_m a_m^2 lambda_m^2 rho_m^(2n) ||phi||^2, which predicts the
  stopping sweep exactly; the oracle recomputes the FP64 residual of the answer.
"""
import math

import numpy as np
import pytest

import oracle
import paper_1207_1746_amd as G
from paper_1207_1746_amd import workloads as W

pytestmark = pytest.mark.gpu


def test_vc13_512_apply_bf16(ctx):
    n, nf = 512, 5
    c, _ = W.vc13_grids(n, nfields=nf)
    fields = W.vc13_fields(n, nfields=nf)
    shp = (n, n, n)
    gf = [ctx.grid(shp, G.BF16, halo=2, data=x) for x in fields]
    gc = [ctx.grid(shp, G.BF16, halo=0, data=x) for x in c]
    go = [ctx.grid(shp, G.BF16, halo=0) for _ in range(nf)]
    ctx.do_all(G.K_VC13_APPLY, gf + gc, go, p=(W.VC13_KAPPA, 0.0, nf))
    for f in (0, nf - 1):
        stored = gf[f].view.double().cpu().numpy()
        ex = oracle.vc13_apply(stored, c, W.VC13_KAPPA)
        got = go[f].view.double().cpu().numpy()
        terms = 1.5 * np.abs(stored).max() * (1 + W.VC13_KAPPA * 3 * (4 / 3 * 2 * 2 + 4 / 12))
        tol = 4 * 2.0 ** -8 * np.abs(ex).max() + 64 * 2.0 ** -24 * terms
        assert np.abs(got - ex).max() <= tol, f


@pytest.mark.parametrize("prec,dt", [(G.PREC_BF16_IR, G.BF16), (G.PREC_F16_IR, G.F16),
                                     (G.PREC_F32_IR, G.F32)])
def test_vc13_512_refinement_reaches_1e10(sctx, prec, dt):
    """Refinement with the correction grids stored in BF16, FP16 or FP32 (FP32
    math) to 1e-10: the oracle recomputes every field's FP64 residual."""
    ctx = sctx
    n, nf = 512, 5
    c, b = W.vc13_grids(n, nfields=nf)
    shp = (n, n, n)
    gx = [ctx.grid(shp, G.F64, halo=2).fill(0.0) for _ in range(nf)]
    gb = [ctx.grid(shp, G.F64, halo=0, data=x) for x in b]
    gc = [ctx.grid(shp, dt, halo=0, data=x) for x in c]
    st = ctx.solve(G.K_VC13_APPLY, gx, gb, gc, kappa=W.VC13_KAPPA, rtol=1e-10, check_every=8,
                   precision=prec, inner_sweeps=16)
    del gc
    bn2 = sum(oracle.sumsq(x) for x in b)
    per_field = []
    for f in range(nf):
        per_field.append(oracle.sumsq(oracle.vc13_residual(gx[f].numpy(), b[f], c, W.VC13_KAPPA)))
        gx[f].close()
    rel = math.sqrt(sum(per_field) / bn2)
    assert rel <= 1e-10 * 1.001, (st, [math.sqrt(r / oracle.sumsq(x)) for r, x in zip(per_field, b)])
    assert abs(rel - st["rel_residual"]) <= 1e-3 * st["rel_residual"]


def _predicted_stop(req, S, rtol, omega=6 / 7):
    """First multiple of S whose checked residual (of u_{n-1}) meets rtol."""
    n = req.n
    h = 1.0 / (n + 1)
    terms = []
    for k, l, m, a in req.modes:
        lam = W.mode_eigenvalue(n, k, l, m)
        mu = (math.cos(k * math.pi * h) + math.cos(l * math.pi * h) + math.cos(m * math.pi * h)) / 3
        rho = 1 - omega + omega * mu
        terms.append((a * a * lam * lam, rho))
    f2 = sum(t for t, _ in terms)
    sweep = S
    while True:
        r2 = sum(t * rho ** (2 * (sweep - 1)) for t, rho in terms)
        if r2 <= rtol * rtol * f2:
            return sweep
        sweep += S


@pytest.mark.parametrize("seed", [0, 3])
def test_poisson_192_solve_matches_closed_form_trace(sctx, seed):
    ctx = sctx
    req = W.poisson_requests(count=1, qps=float("inf"), nmin=192, nmax=192, seed_index=seed)[0]
    _, f = W.poisson_fields(req)
    S = 64
    expect = _predicted_stop(req, S, 1e-8)
    u = ctx.grid(f.shape, G.F64, halo=1).fill(0.0)
    gf = ctx.grid(f.shape, G.F64, halo=0, data=f)
    st = ctx.solve(G.K_WJACOBI, [u], [gf], h2=req.h2, rtol=1e-8, check_every=S)
    assert st["sweeps"] == expect
    _, _, res = oracle.wjacobi_sweep(u.numpy(), f, 6 / 7, req.h2)
    # the returned grid is one sweep past the checked one: its residual is smaller still
    assert math.sqrt(oracle.sumsq(res) / oracle.sumsq(f)) <= 1e-8


def test_batch_mixed_sizes_up_to_192(sctx):
    ctx = sctx
    reqs = W.poisson_requests(count=6, qps=float("inf"), nmin=32, nmax=192, seed_index=11)
    reqs[0] = W.poisson_requests(count=1, qps=float("inf"), nmin=192, nmax=192, seed_index=5)[0]
    S = 64
    b = G.Batch(ctx, max_slots=8, precision=G.PREC_F64, sweeps_per_step=S, rtol=1e-8, hbm_budget=4 << 30)
    grids = []
    for r in reqs:
        _, f = W.poisson_fields(r)
        u = ctx.grid(f.shape, G.F64, halo=1).fill(0.0)
        gf = ctx.grid(f.shape, G.F64, halo=0, data=f)
        grids.append((u, gf, f))
        assert b.admit(u, gf, r.h2) is not None
    done = {}
    steps = 0
    while len(done) < len(reqs):
        b.step()
        steps += 1
        for s in b.poll():
            done[s] = b.retire(s)
        assert steps < 20000
    b.close()
    for i, r in enumerate(reqs):
        assert done[i]["sweeps"] == _predicted_stop(r, S, 1e-8), i
        u, _, f = grids[i]
        _, _, res = oracle.wjacobi_sweep(u.numpy(), f, 6 / 7, r.h2)
        assert math.sqrt(oracle.sumsq(res) / oracle.sumsq(f)) <= 1e-8


@pytest.mark.parametrize("n,S", [(150, 10), (150, 6), (160, 4), (90, 10)])
def test_poisson_temporal_chunks_match_closed_form_trace(sctx, n, S):
    """Grids of 72^3 points or more run their chunks as temporally blocked
    passes (S = 10 -> 4+4+1+1, 6 -> 4+2, 4 -> 2+2): same stopping sweep as
    the closed-form residual trace, and the oracle's residual of the answer."""
    ctx = sctx
    req = W.poisson_requests(count=1, qps=float("inf"), nmin=n, nmax=n, seed_index=n)[0]
    _, f = W.poisson_fields(req)
    expect = _predicted_stop(req, S, 1e-8)
    u = ctx.grid(f.shape, G.F64, halo=1).fill(0.0)
    gf = ctx.grid(f.shape, G.F64, halo=0, data=f)
    st = ctx.solve(G.K_WJACOBI, [u], [gf], h2=req.h2, rtol=1e-8, check_every=S)
    assert st["sweeps"] == expect
    _, _, res = oracle.wjacobi_sweep(u.numpy(), f, 6 / 7, req.h2)
    assert math.sqrt(oracle.sumsq(res) / oracle.sumsq(f)) <= 1e-8


def test_rbgs_512_blocked_bitwise_and_sampled_oracle(ctx):
    """The red-black benchmark workload at its size (512^3 FP64 with a
    right-hand side, omega 1.9): four colour passes as one blocked pass equal
    four in-place passes bit for bit, and sampled points of one in-place pass
    match the oracle's pass on each point's 3^3 neighbourhood (zero outside
    the domain, the Dirichlet value)."""
    import torch
    n = 512
    shape = (n, n, n)
    u0, h2 = W.jacobi_cube(n)
    f = W.jacobi_rhs(n)
    omega = 1.9
    gu = ctx.grid(shape, G.F64, halo=1, data=u0)
    gf = ctx.grid(shape, G.F64, halo=0, data=f)
    a = ctx.grid(shape, G.F64, halo=1)
    a.view.copy_(gu.view)
    ctx.do_all(G.K_RBGS, [a, gf], [a], p=(omega, h2, 0))
    # sampled points of the pass's colour (0): the oracle on the neighbourhood
    g = np.random.default_rng(70)
    pts = g.integers(0, n, size=(1200, 3))
    pts = pts[(pts.sum(axis=1) % 2) == 0][:500]  # (k + j + i) even: the pass's colour
    pts = np.vstack([pts, [[0, 0, 0], [n - 1, n - 1, 0], [n - 2, 0, n - 2]]])
    got = a.view[torch.as_tensor(pts[:, 0]), torch.as_tensor(pts[:, 1]), torch.as_tensor(pts[:, 2])].cpu().numpy()
    up = np.pad(u0, 1)
    fp = np.pad(f, 1)
    for (k, j, i), gv in zip(pts, got):
        box = up[k:k + 3, j:j + 3, i:i + 3]
        fbox = fp[k:k + 3, j:j + 3, i:i + 3]
        ex = oracle.rbgs_pass(box, fbox, omega, h2, 1, 0.0)[0][1, 1, 1]  # centre (1,1,1) has odd parity
        assert abs(gv - ex) <= 1e-14 * (8 * np.abs(box).max() + h2 * abs(fbox[1, 1, 1])), (k, j, i)
    # the other colour is untouched
    assert torch.equal(a.view[0, 0, 1], gu.view[0, 0, 1])
    for c in (1, 0, 1):
        ctx.do_all(G.K_RBGS, [a, gf], [a], p=(omega, h2, c))
    go = ctx.grid(shape, G.F64, halo=1)
    ctx.do_all(G.K_RBGS_TB, [gu, gf], [go], p=(omega, h2, 0, 4))
    assert torch.equal(go.view, a.view)


def test_tridiag_512_sampled_columns(ctx):
    """The line benchmark workload at its size: tridiagonal solves along k for
    every column of a 512^3 FP64 grid (elimination do_k_inc, substitution
    do_k_dec); sampled columns equal the oracle's Thomas solve bit for bit."""
    import torch
    n = 512
    shape = (n, n, n)
    gen = torch.Generator(device="cuda").manual_seed(12071746)
    grids = []
    for lo, hi in ((-1.0, 1.0), (2.5, 3.5), (-1.0, 1.0), (-1.0, 1.0)):
        gg = ctx.grid(shape, G.F64, halo=0)
        gg.view.copy_(torch.rand(shape, dtype=torch.float64, device="cuda", generator=gen) * (hi - lo) + lo)
        grids.append(gg)
    cp, dp, x = (ctx.grid(shape, G.F64, halo=0) for _ in range(3))
    ctx.do_line(G.K_TRIDIAG_FWD, 2, 1, grids, [cp, dp])
    ctx.do_line(G.K_TRIDIAG_BACK, 2, -1, [cp, dp], [x])
    g = np.random.default_rng(71)
    cols = [(0, 0), (n - 1, n - 1), (0, n - 1)] + [tuple(c) for c in g.integers(0, n, size=(13, 2))]
    for j, i in cols:
        col = [gg.view[:, j, i].cpu().numpy().reshape(n, 1, 1) for gg in grids]
        ecp, edp = oracle.tridiag_fwd(*col, 2, 1)
        ex = oracle.tridiag_back(ecp, edp, 2, -1)
        assert np.array_equal(x.view[:, j, i].cpu().numpy(), ex.reshape(n)), (j, i)
