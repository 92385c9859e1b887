"""GPU parity for the solver, the batched executor and the serving loop.

* gscl_solve F64 (Section 5.2: sweep + fused check until done) takes exactly
  the oracle's number of sweeps (the check is fused into the last sweep of
  each chunk on both sides) and returns the same iterate to 1e-11 relative.
* Mixed-precision refinement: the oracle recomputes the FP64 residual of the
  GPU's answer; it must meet rtol (1e-10), and the answer must agree with the
  oracle's tight FP64 solution within cond(A) * rtol.
* Batched executor: every request's answer is bit-identical alone and in a
  mix (per-slot arithmetic and reduction order do not depend on the mix), and
  matches the one-at-a-time solver.
"""
import math

import numpy as np
import pytest

import oracle
import paper_1207_1746_amd as G
from paper_1207_1746_amd import serve as SV
from paper_1207_1746_amd import workloads as W

pytestmark = pytest.mark.gpu


def _req(n, seed=0, rid=0):
    r = W.poisson_requests(count=1, qps=float("inf"), nmin=n, nmax=n, seed_index=seed)[0]
    r.rid = rid
    return r


def _oracle_rel_residual(u, f, h2):
    _, _, res = oracle.wjacobi_sweep(u, f, 6 / 7, h2)
    return math.sqrt(oracle.sumsq(res) / oracle.sumsq(f))


@pytest.mark.parametrize("n,S", [(20, 32), (33, 16)])
def test_poisson_f64_matches_oracle(ctx, n, S):
    req = _req(n, seed=n)
    ustar, f = W.poisson_fields(req)
    u = ctx.grid(f.shape, G.F64, halo=1).fill(0.0)
    gf = ctx.grid(f.shape, G.F64, halo=0, data=f)
    st = ctx.solve(G.K_WJACOBI, [u], [gf], h2=req.h2, rtol=1e-8, check_every=S)
    uo, so, relo, conv = oracle.poisson_solve(f, req.h2, 6 / 7, 1e-8, S, 10 ** 6)
    assert conv and st["sweeps"] == so
    assert abs(st["rel_residual"] - relo) <= 1e-6 * relo  # cancellation at 1e-8
    got = u.numpy()
    assert np.abs(got - uo).max() <= 1e-11 * np.abs(uo).max()
    # manufactured solution: ||u - u*||_2 <= ||r||_2 / |lambda_min|
    lam_min = abs(W.mode_eigenvalue(n, 1, 1, 1))
    r_now = _oracle_rel_residual(got, f, req.h2) * math.sqrt(oracle.sumsq(f))
    assert math.sqrt(oracle.sumsq(got - ustar)) <= r_now / lam_min * 1.0001


def test_poisson_f32_refinement_reaches_1e10(sctx):
    ctx = sctx
    n = 28
    req = _req(n, seed=3)
    ustar, f = W.poisson_fields(req)
    u = ctx.grid(f.shape, G.F64, halo=1).fill(0.0)
    gf = ctx.grid(f.shape, G.F64, halo=0, data=f)
    st = ctx.solve(G.K_WJACOBI, [u], [gf], h2=req.h2, rtol=1e-10, check_every=2,
                   precision=G.PREC_F32_IR, inner_sweeps=128)
    got = u.numpy()
    rel = _oracle_rel_residual(got, f, req.h2)
    assert rel <= 1e-10 * 1.001 and st["outer"] >= 1
    assert abs(rel - st["rel_residual"]) <= 1e-4 * rel  # cancellation at 1e-10
    # matches the FP64 solve to the accuracy rtol allows
    uo, _, _, _ = oracle.poisson_solve(f, req.h2, 6 / 7, 1e-12, 32, 10 ** 6)
    lam_min = abs(W.mode_eigenvalue(n, 1, 1, 1))
    lam_max = abs(W.mode_eigenvalue(n, n, n, n))
    assert np.abs(got - uo).max() <= 2e-10 * lam_max / lam_min * np.abs(uo).max()


def test_poisson_solver_errors(ctx):
    req = _req(12)
    _, f = W.poisson_fields(req)
    u = ctx.grid(f.shape, G.F64, halo=1).fill(0.0)
    gf = ctx.grid(f.shape, G.F64, halo=0, data=f)
    with pytest.raises(G.GsclError) as e:
        ctx.solve(G.K_WJACOBI, [u], [gf], h2=req.h2, rtol=1e-12, check_every=4, max_sweeps=8)
    assert e.value.code == G.ERR_NOCONV
    bad = f.copy()
    bad[3, 4, 5] = np.nan
    gb = ctx.grid(f.shape, G.F64, halo=0, data=bad)
    u.fill(0.0)
    with pytest.raises(G.GsclError) as e:
        ctx.solve(G.K_WJACOBI, [u], [gb], h2=req.h2, rtol=1e-8, check_every=4)
    assert e.value.code == G.ERR_NUMERIC
    z = ctx.grid(f.shape, G.F64, halo=0).fill(0.0)
    u.fill(1.0)
    st = ctx.solve(G.K_WJACOBI, [u], [z], h2=req.h2, rtol=1e-8, check_every=4)
    assert st["sweeps"] == 0 and np.all(u.numpy() == 0.0)
    # pitches whose narrow-type workspace rows or planes would not start on
    # 16-byte boundaries are refused before any launch
    for pitch in ((18, 18 * 12), (16, 16 * 12 + 2)):
        d = G.make_desc(f.shape, G.F64, halo=1, pitch=pitch)
        up = G.Grid(ctx, d).fill(0.0)
        fp = G.Grid(ctx, G.make_desc(f.shape, G.F64, halo=0, pitch=pitch)).upload(f)
        with pytest.raises(G.GsclError) as e:
            ctx.solve(G.K_WJACOBI, [up], [fp], h2=req.h2, rtol=1e-8, check_every=4, precision=G.PREC_F32_IR)
        assert e.value.code == G.ERR_SHAPE, pitch


@pytest.mark.parametrize("prec,dt", [(G.PREC_F64, G.BF16), (G.PREC_F32_IR, G.F32),
                                     (G.PREC_BF16_IR, G.BF16), (G.PREC_F16_IR, G.F16)])
def test_vc13_solve_per_precision(ctx, prec, dt):
    shape = (10, 12, 20)
    nf = 5
    c, b = W.vc13_grids(shape[2], shape[1], shape[0], nf)
    gx = [ctx.grid(shape, G.F64, halo=2).fill(0.0) for _ in range(nf)]
    gb = [ctx.grid(shape, G.F64, halo=0, data=x) for x in b]
    gc = [ctx.grid(shape, dt, halo=0, data=x) for x in c]
    st = ctx.solve(G.K_VC13_APPLY, gx, gb, gc, kappa=W.VC13_KAPPA, rtol=1e-10, check_every=8,
                   precision=prec, inner_sweeps=16)
    bn = math.sqrt(sum(oracle.sumsq(x) for x in b))
    rn = math.sqrt(sum(oracle.sumsq(oracle.vc13_residual(gx[f].numpy(), b[f], c, W.VC13_KAPPA))
                       for f in range(nf)))
    assert rn / bn <= 1e-10 * 1.001, (prec, rn / bn, st)
    for f in range(nf):
        xo, _, _ = oracle.vc13_jacobi_solve(b[f], c, W.VC13_KAPPA, 6 / 7, 1e-14, 10000)
        # A is diagonally dominant with cond(A) < 10 for these coefficients
        assert np.abs(gx[f].numpy() - xo).max() <= 1e-9 * 10 * np.abs(xo).max()


def _batch_solve(ctx, reqs, prec, S, admit_at=None, use_graph=True, rtol=1e-8, method=G.BATCH_JACOBI,
                 omega=6 / 7, sweeps_per_pass=1, hbm_budget=1 << 30, rule=None):
    """Run requests through one batch; admit_at[i] = step index to admit request i."""
    b = G.Batch(ctx, max_slots=8, precision=prec, sweeps_per_step=S, use_graph=use_graph, rtol=rtol,
                hbm_budget=hbm_budget, method=method, omega=omega, sweeps_per_pass=sweeps_per_pass)
    if rule:
        b.set_tile_rule(rule)
    admit_at = admit_at or [0] * len(reqs)
    grids = {}
    out = {}
    slots = {}
    step = 0
    while len(out) < len(reqs):
        for i, r in enumerate(reqs):
            if admit_at[i] == step and i not in slots:
                _, f = W.poisson_fields(r)
                u = ctx.grid(f.shape, G.F64, halo=1).fill(0.0)
                gf = ctx.grid(f.shape, G.F64, halo=0, data=f)
                grids[i] = (u, gf)
                s = b.admit(u, gf, r.h2)
                assert s is not None
                slots[i] = s
        b.step()
        step += 1
        for s in b.poll():
            i = [k for k, v in slots.items() if v == s and k not in out][0]
            st = b.retire(s)
            out[i] = (grids[i][0].numpy(), st)
        assert step < 100000
    b.close()
    return out


@pytest.mark.parametrize("prec", [G.PREC_F64, G.PREC_F32_IR])
def test_batch_alone_equals_mix(ctx, prec):
    reqs = [_req(n, seed=n, rid=i) for i, n in enumerate((24, 37, 17, 45))]
    S = 16
    mix = _batch_solve(ctx, reqs, prec, S, admit_at=[0, 0, 3, 5])
    for i, r in enumerate(reqs):
        alone = _batch_solve(ctx, [r], prec, S)[0]
        assert np.array_equal(alone[0], mix[i][0]), i
        assert alone[1]["sweeps"] == mix[i][1]["sweeps"] and alone[1]["state"] == 2
        _, f = W.poisson_fields(r)
        assert _oracle_rel_residual(mix[i][0], f, r.h2) <= 1e-8 * 1.01


def test_batch_f64_matches_solver_and_oracle(sctx):
    ctx = sctx
    reqs = [_req(n, seed=n + 1, rid=i) for i, n in enumerate((19, 30))]
    S = 16
    res = _batch_solve(ctx, reqs, G.PREC_F64, S, use_graph=False)
    resg = _batch_solve(ctx, reqs, G.PREC_F64, S, use_graph=True)
    for i, r in enumerate(reqs):
        _, f = W.poisson_fields(r)
        uo, so, _, _ = oracle.poisson_solve(f, r.h2, 6 / 7, 1e-8, S, 10 ** 6)
        assert res[i][1]["sweeps"] == so
        assert np.abs(res[i][0] - uo).max() <= 1e-11 * np.abs(uo).max()
        assert np.array_equal(res[i][0], resg[i][0])
        u = ctx.grid(f.shape, G.F64, halo=1).fill(0.0)
        gf = ctx.grid(f.shape, G.F64, halo=0, data=f)
        st = ctx.solve(G.K_WJACOBI, [u], [gf], h2=r.h2, rtol=1e-8, check_every=S)
        assert st["sweeps"] == so and np.array_equal(u.numpy(), res[i][0])


@pytest.mark.parametrize("omega", [0.0, 1.0, 1.7])
def test_batch_rbgs_matches_solver_and_oracle(sctx, omega):
    """Red-black SOR slots: alone == among others (bitwise), and the same
    stopping sweep and iterate as the plain checked solve and the oracle."""
    ctx = sctx
    reqs = [_req(n, seed=n + 2, rid=i) for i, n in enumerate((21, 34, 16))]
    S = 4
    mix = _batch_solve(ctx, reqs, G.PREC_F64, S, admit_at=[0, 1, 2], method=G.BATCH_RBGS, omega=omega)
    for i, r in enumerate(reqs):
        _, f = W.poisson_fields(r)
        alone = _batch_solve(ctx, [r], G.PREC_F64, S, use_graph=False, method=G.BATCH_RBGS, omega=omega)[0]
        assert np.array_equal(alone[0], mix[i][0]), i
        assert alone[1]["sweeps"] == mix[i][1]["sweeps"] and mix[i][1]["state"] == 2
        u = ctx.grid(f.shape, G.F64, halo=1).fill(0.0)
        gf = ctx.grid(f.shape, G.F64, halo=0, data=f)
        st = ctx.solve(G.K_RBGS, [u], [gf], omega=omega, h2=r.h2, rtol=1e-8, check_every=S)
        assert st["sweeps"] == mix[i][1]["sweeps"] and np.array_equal(u.numpy(), mix[i][0])
        w = omega
        if w == 0.0:
            c = math.cos(math.pi / (r.n + 1))
            rho = (c + c + c) / 3.0
            w = 2 / (1 + math.sqrt(1 - rho * rho))
        uo, so, _, conv = oracle.rbgs_solve(f, r.h2, w, 1e-8, S, 10 ** 6)
        assert conv and mix[i][1]["sweeps"] == so
        assert np.abs(mix[i][0] - uo).max() <= 1e-11 * np.abs(uo).max()
        assert _oracle_rel_residual(mix[i][0], f, r.h2) <= 1e-8 * 1.01


def test_batch_rbgs_errors_and_footprint(ctx):
    with pytest.raises(G.GsclError) as e:
        G.Batch(ctx, precision=G.PREC_F32_IR, method=G.BATCH_RBGS)
    assert e.value.code == G.ERR_UNSUPPORTED
    for kw in ({"omega": 2.0}, {"omega": -0.5}, {"method": 2}):
        with pytest.raises(G.GsclError) as e:
            G.Batch(ctx, **{"method": G.BATCH_RBGS, **kw})
        assert e.value.code == G.ERR_ARG
    jb = G.Batch(ctx, max_slots=1, hbm_budget=1 << 20)
    rb = G.Batch(ctx, max_slots=1, hbm_budget=1 << 20, method=G.BATCH_RBGS, omega=0.0)
    # in-place sweeps: the work grid is one F32 residual instead of an F64 ping-pong grid
    assert rb.footprint((40, 40, 40)) < jb.footprint((40, 40, 40))
    jb.close()
    rb.close()


@pytest.mark.parametrize("prec,k", [(G.PREC_F64, 4), (G.PREC_F64, 2), (G.PREC_F32_IR, 4)])
def test_batch_blocked_passes_equal_plain_sweeps(ctx, prec, k):
    """Jacobi slots swept as temporally blocked passes of k sweeps: the same
    iterates bit for bit as one-sweep passes (same stopping step), and alone
    equals among others."""
    reqs = [_req(n, seed=n + 3, rid=i) for i, n in enumerate((17, 37, 45, 24, 7))]
    S = 16
    plain = _batch_solve(ctx, reqs, prec, S, admit_at=[0, 0, 2, 3, 1])
    blocked = _batch_solve(ctx, reqs, prec, S, admit_at=[0, 0, 2, 3, 1], sweeps_per_pass=k)
    for i, r in enumerate(reqs):
        assert blocked[i][1]["state"] == 2
        assert blocked[i][1]["sweeps"] == plain[i][1]["sweeps"], i
        assert np.array_equal(blocked[i][0], plain[i][0]), i
        alone = _batch_solve(ctx, [r], prec, S, sweeps_per_pass=k, use_graph=False)[0]
        assert np.array_equal(alone[0], blocked[i][0]) and alone[1]["sweeps"] == blocked[i][1]["sweeps"], i
        _, f = W.poisson_fields(r)
        assert _oracle_rel_residual(blocked[i][0], f, r.h2) <= 1e-8 * 1.01


def test_batch_f32_refinement_large_slots_1e10(ctx):
    """The served configuration at the large end of the request sizes: F32
    refinement with blocked passes of 4 sweeps, steps of 64 sweeps, three
    slots of N in [150, 192] among small ones, to 1e-10.  Every answer's FP64
    residual is recomputed by the oracle, and each request alone gives the
    same answer bit for bit as in the mix."""
    sizes = (150, 24, 171, 37, 192, 61)
    reqs = [_req(n, seed=n + 7, rid=i) for i, n in enumerate(sizes)]
    S, k, rtol = 64, 4, 1e-10
    mix = _batch_solve(ctx, reqs, G.PREC_F32_IR, S, admit_at=[0, 0, 1, 2, 3, 5], rtol=rtol,
                       sweeps_per_pass=k, hbm_budget=4 << 30)
    for i, r in enumerate(reqs):
        assert mix[i][1]["state"] == 2, (r.n, mix[i][1])
        _, f = W.poisson_fields(r)
        rel = _oracle_rel_residual(mix[i][0], f, r.h2)
        assert rel <= rtol * 1.01, (r.n, rel, mix[i][1])
        if r.n >= 150:
            alone = _batch_solve(ctx, [r], G.PREC_F32_IR, S, rtol=rtol, sweeps_per_pass=k,
                                 hbm_budget=4 << 30)[0]
            assert np.array_equal(alone[0], mix[i][0]), r.n
            assert alone[1]["sweeps"] == mix[i][1]["sweeps"], r.n


def test_batch_tile_rule(ctx):
    """Tuned tile rules of the batched kernels.  Refinement with blocked
    passes: a rule that changes only the blocked-pass chunks gives the untuned
    answers bit for bit (those passes carry no reduction).  A rule that
    changes the one-sweep chunks (which fold the residual) keeps every answer
    the same alone and in the mix, and within rtol by the oracle."""
    reqs = [_req(n, seed=n + 11, rid=i) for i, n in enumerate((17, 37, 45, 24, 9))]
    at = [0, 0, 2, 3, 1]
    base = _batch_solve(ctx, reqs, G.PREC_F32_IR, 16, admit_at=at, sweeps_per_pass=4)
    tb_only = _batch_solve(ctx, reqs, G.PREC_F32_IR, 16, admit_at=at, sweeps_per_pass=4,
                           rule=[(24, 0, 2), (40, 0, 32), (64, 0, 1)])
    for i in range(len(reqs)):
        assert np.array_equal(base[i][0], tb_only[i][0]) and base[i][1]["sweeps"] == tb_only[i][1]["sweeps"], i
    rule = [(20, 2, 0), (40, 16, 0), (64, 4, 8)]
    for prec, k in ((G.PREC_F64, 1), (G.PREC_F32_IR, 4)):
        mix = _batch_solve(ctx, reqs, prec, 16, admit_at=at, sweeps_per_pass=k, rule=rule)
        for i, r in enumerate(reqs):
            assert mix[i][1]["state"] == 2
            alone = _batch_solve(ctx, [r], prec, 16, sweeps_per_pass=k, rule=rule, use_graph=False)[0]
            assert np.array_equal(alone[0], mix[i][0]) and alone[1]["sweeps"] == mix[i][1]["sweeps"], (prec, i)
            _, f = W.poisson_fields(r)
            assert _oracle_rel_residual(mix[i][0], f, r.h2) <= 1e-8 * 1.01
    b = G.Batch(ctx, max_slots=2)
    for bad in ([(40, 4, 4), (20, 4, 4)], [(0, 4, 4)], [(40, -1, 4)], [(40, 4, 2000)]):
        with pytest.raises(G.GsclError) as e:
            b.set_tile_rule(bad)
        assert e.value.code == G.ERR_ARG
    b.set_tile_rule([])
    b.close()


def test_autotuner_batch_rule(ctx, tmp_path):
    """The tuner times candidate chunks per request-size bucket on a filled
    batch, returns a rule the executor accepts, and caches it."""
    from paper_1207_1746_amd import autotune
    path = str(tmp_path / "tiles.json")
    t = autotune.Tuner(ctx, cache_path=path)
    rule = t.tune_batch(buckets=((24, 20), (40, 36)), slots=3, reps=1, sweeps_per_step=16)
    assert [r[0] for r in rule] == [24, 40]
    assert all(r[1] in (4, 8, 16) and r[2] in (4, 8, 16, 32) for r in rule)
    t.save()
    again = autotune.Tuner(ctx, cache_path=path).tune_batch(buckets=((24, 20), (40, 36)), slots=3, reps=1,
                                                           sweeps_per_step=16)
    assert again == rule
    reqs = [_req(n, seed=n + 13, rid=i) for i, n in enumerate((21, 33))]
    res = _batch_solve(ctx, reqs, G.PREC_F32_IR, 16, sweeps_per_pass=4, rule=rule)
    for i, r in enumerate(reqs):
        _, f = W.poisson_fields(r)
        assert res[i][1]["state"] == 2 and _oracle_rel_residual(res[i][0], f, r.h2) <= 1e-8 * 1.01


@pytest.mark.parametrize("k,S", [(4, 4), (2, 6)])
def test_batch_rbgs_blocked_equals_inplace(ctx, k, S):
    """Red-black slots swept as blocked passes of k colour passes through a
    second grid: the same iterates bit for bit and the same stopping sweep as
    in-place colour passes, alone equal to among others."""
    reqs = [_req(n, seed=n + 4, rid=i) for i, n in enumerate((21, 40, 9, 33))]
    plain = _batch_solve(ctx, reqs, G.PREC_F64, S, admit_at=[0, 1, 1, 2], method=G.BATCH_RBGS, omega=0.0)
    blocked = _batch_solve(ctx, reqs, G.PREC_F64, S, admit_at=[0, 1, 1, 2], method=G.BATCH_RBGS, omega=0.0,
                           sweeps_per_pass=k)
    for i, r in enumerate(reqs):
        assert blocked[i][1]["state"] == 2
        assert blocked[i][1]["sweeps"] == plain[i][1]["sweeps"], i
        assert np.array_equal(blocked[i][0], plain[i][0]), i
        alone = _batch_solve(ctx, [r], G.PREC_F64, S, method=G.BATCH_RBGS, omega=0.0, sweeps_per_pass=k,
                             use_graph=False)[0]
        assert np.array_equal(alone[0], blocked[i][0]) and alone[1]["sweeps"] == blocked[i][1]["sweeps"], i


def test_batch_blocked_pass_errors(ctx):
    for kw, code in (({"sweeps_per_pass": 5}, G.ERR_ARG), ({"sweeps_per_pass": -1}, G.ERR_ARG),
                     ({"sweeps_per_pass": 4, "sweeps_per_step": 12}, G.ERR_ARG),
                     ({"sweeps_per_pass": 3, "method": G.BATCH_RBGS}, G.ERR_UNSUPPORTED),
                     ({"sweeps_per_pass": 4, "sweeps_per_step": 6, "method": G.BATCH_RBGS}, G.ERR_ARG)):
        with pytest.raises(G.GsclError) as e:
            G.Batch(ctx, **{"sweeps_per_step": 16, **kw})
        assert e.value.code == code, kw


def test_batch_budget_admission(ctx):
    r = _req(40)
    _, f = W.poisson_fields(r)
    probe = G.Batch(ctx, max_slots=1, precision=G.PREC_F64, sweeps_per_step=8, hbm_budget=1 << 20)
    fp = probe.footprint((40, 40, 40))
    probe.close()
    assert fp >= 3 * 40 ** 3 * 8  # u, f and the ping-pong grid (rows padded to 16 elements)
    b = G.Batch(ctx, max_slots=4, precision=G.PREC_F64, sweeps_per_step=8, hbm_budget=2 * fp + fp // 2)
    grids = [(ctx.grid(f.shape, G.F64, halo=1).fill(0.0), ctx.grid(f.shape, G.F64, halo=0, data=f))
             for _ in range(3)]
    assert b.admit(*grids[0], r.h2) is not None
    assert b.admit(*grids[1], r.h2) is not None
    assert b.admit(*grids[2], r.h2) is None  # over budget: caller queues
    b.close()


def test_serving_loop_continuous_batching(sctx):
    ctx = sctx
    reqs = W.poisson_requests(count=12, qps=200.0, nmin=16, nmax=40, seed_index=7)
    jobs = []
    for r in reqs:
        _, f = W.poisson_fields(r)
        jobs.append(SV.Job(r.rid, r.n, r.h2, r.arrival, f))
    srv = SV.SolveServer(ctx, precision=G.PREC_F32_IR, sweeps_per_step=32, rtol=1e-8, max_slots=8)
    rep = srv.run(jobs)
    srv.close()
    s = rep.summary()
    assert s["converged"] == len(jobs) and s["p99_s"] >= s["p50_s"] > 0
    assert rep.max_running > 1  # requests overlapped on the device
    for j, r in zip(jobs, reqs):
        _, f = W.poisson_fields(r)
        got = j.u.numpy()
        assert _oracle_rel_residual(got, f, r.h2) <= 1e-8 * 1.01
        alone = _batch_solve(ctx, [r], G.PREC_F32_IR, 32)[0]
        assert np.array_equal(alone[0], got)


def test_autotuner_blocked_kind(ctx, tmp_path):
    """The blocked sweep's only tunable is its z chunk: the tuner tries those,
    installs the fastest, and the result is the one the default tile gives."""
    from paper_1207_1746_amd import autotune as AT
    shape = (40, 50, 90)
    u = np.random.default_rng(3).standard_normal(shape)
    gu = ctx.grid(shape, G.F64, halo=1, data=u)
    go = ctx.grid(shape, G.F64, halo=1)
    ctx.do_all(G.K_WJACOBI_TB, [gu], [go], p=(0.9, 1.0, 4))
    ref = go.numpy()
    t = AT.Tuner(ctx, str(tmp_path / "tiles.json"))
    rec = t.tune(G.K_WJACOBI_TB, [gu], [go], p=(0.9, 1.0, 4), reps=2)
    assert len(rec["tried"]) == len(AT.candidates(G.K_WJACOBI_TB, G.F64, shape[0]))
    assert tuple(rec["tile"]) == ctx.tile_get(G.K_WJACOBI_TB, gu) and rec["tile"][:2] == [1, 16]
    ctx.do_all(G.K_WJACOBI_TB, [gu], [go], p=(0.9, 1.0, 4))
    assert np.array_equal(go.numpy(), ref)
    ctx.tile_clear()


def test_autotuner_picks_installs_and_caches(ctx, tmp_path):
    from paper_1207_1746_amd import autotune as AT
    shape = (24, 40, 200)
    u = np.random.default_rng(2).standard_normal(shape)
    gu = ctx.grid(shape, G.F64, halo=1, data=u)
    go = ctx.grid(shape, G.F64, halo=1)
    path = str(tmp_path / "tiles.json")
    t = AT.Tuner(ctx, path)
    rec = t.tune(G.K_WJACOBI, [gu], [go], p=(0.9, 1.0), reps=3)
    assert tuple(rec["tile"]) == ctx.tile_get(G.K_WJACOBI, gu)
    assert len(rec["tried"]) >= 8
    t.save()
    ctx.do_all(G.K_WJACOBI, [gu], [go], p=(0.9, 1.0))
    tuned = go.numpy()
    ctx.tile_clear()
    ctx.do_all(G.K_WJACOBI, [gu], [go], p=(0.9, 1.0))
    assert np.array_equal(go.numpy(), tuned)  # the tile never changes a do_all result
    t2 = AT.Tuner(ctx, path)
    assert t2.apply(G.K_WJACOBI, gu) and ctx.tile_get(G.K_WJACOBI, gu) == tuple(rec["tile"])
    ctx.tile_clear()


@pytest.mark.timeout(60)
def test_serving_rejects_request_that_never_fits(sctx):
    """A request whose footprint exceeds the whole budget is reported as
    rejected instead of waiting in the queue for ever; the loop returns and
    serves the others."""
    ctx = sctx
    reqs = W.poisson_requests(count=4, qps=float("inf"), nmin=12, nmax=20, seed_index=9)
    big = _req(48, seed=5, rid=99)
    jobs = []
    for r in reqs[:2] + [big] + reqs[2:]:
        _, f = W.poisson_fields(r)
        jobs.append(SV.Job(r.rid, r.n, r.h2, 0.0, f))
    probe = G.Batch(ctx, max_slots=1, precision=G.PREC_F64, sweeps_per_step=8, hbm_budget=1 << 30)
    fp_small = max(probe.footprint((r.n,) * 3) for r in reqs)
    fp_big = probe.footprint((48,) * 3)
    probe.close()
    assert fp_big > 2 * fp_small
    srv = SV.SolveServer(ctx, precision=G.PREC_F64, sweeps_per_step=16, rtol=1e-8, max_slots=4,
                         hbm_budget=2 * fp_small, sweeps_per_pass=1)
    rep = srv.run(jobs, realtime=False)
    srv.close()
    s = rep.summary()
    assert s["rejected"] == 1 and s["converged"] == len(reqs)
    rej = [j for j in jobs if j.state == 3]
    assert rej[0].rid == 99 and "budget" in rej[0].error and rej[0].u is None
    for j, r in zip([j for j in jobs if j.state == 2], reqs):
        _, f = W.poisson_fields(r)
        assert _oracle_rel_residual(j.u.numpy(), f, r.h2) <= 1e-8 * 1.01
