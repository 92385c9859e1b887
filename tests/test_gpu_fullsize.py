"""GPU parity at the workloads' full sizes, in the launch configuration the
benchmark uses, via checks the oracle can afford at any size.

* 13-point operator on 5 fields at 512^3: the first and last fields of the
  BF16 apply against the full FP64 oracle apply; iterative refinement in BF16 storage to 1e-10
  with the FP64 residual of every field recomputed by the oracle.
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


def test_vc13_512_refinement_bf16_reaches_1e10(sctx):
    ctx = sctx
    n, nf = 512, 5
    c, b = W.vc13_grids(n, nfields=nf)
    shp = (n, n, n)
    gx = [ctx.grid(shp, G.F64, halo=2).fill(0.0) for _ in range(nf)]
    gb = [ctx.grid(shp, G.F64, halo=0, data=x) for x in b]
    gc = [ctx.grid(shp, G.BF16, halo=0, data=x) for x in c]
    st = ctx.solve(G.K_VC13_APPLY, gx, gb, gc, kappa=W.VC13_KAPPA, rtol=1e-10, check_every=8,
                   precision=G.PREC_BF16_IR, inner_sweeps=16)
    bn2 = sum(oracle.sumsq(x) for x in b)
    rn2 = 0.0
    for f in range(nf):
        rn2 += oracle.sumsq(oracle.vc13_residual(gx[f].numpy(), b[f], c, W.VC13_KAPPA))
    assert math.sqrt(rn2 / bn2) <= 1e-10 * 1.001, st
    assert abs(math.sqrt(rn2 / bn2) - st["rel_residual"]) <= 1e-3 * st["rel_residual"]


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


@pytest.mark.parametrize("n,S", [(150, 10), (150, 6), (160, 4)])
def test_poisson_temporal_chunks_match_closed_form_trace(sctx, n, S):
    """Grids of 144^3 points or more run their chunks as temporally blocked
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
