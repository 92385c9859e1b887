"""Tile autotuner for the tiled do_all kernels (autotuning is the paper's
stated future work, Section 2 and Section 6).

For one operator kind and one set of grid extents it times every candidate
tile shape (V elements per lane, NW waves per block, cz planes per block) with
HIP events, keeps the fastest, installs it in the context with
``gscl_tile_set`` and records it in a JSON cache keyed by
(gfx arch, kind, dtype, extents).  Outputs do not depend on the tile shape
(only the fused-reduction rounding order does), so tuning never changes a
do_all result.

For the batched executor it picks, per request-size bucket, the z chunks of
the one-sweep and blocked-pass tiles (``gscl_batch_tile_rule``) by timing
steps of a batch filled with requests of the bucket's size, and caches the
rule under (gfx arch, precision, method, step and pass lengths, bucket).
"""
from __future__ import annotations

import itertools
import json
import os
from typing import Callable, Iterable, Sequence

import paper_1207_1746_amd as G

DEFAULT_CACHE = os.environ.get("GSCL_TILE_CACHE",
                               os.path.join(os.path.expanduser("~"), ".cache", "gscl", "tiles.json"))

RADIUS2 = (G.K_VC13_APPLY, G.K_VC13_JACOBI, G.K_VC13_RESID)


BLOCKED = (G.K_WJACOBI_TB, G.K_RBGS_TB)

# request-size buckets of the batched executor: (largest extent, cube side
# timed for the bucket)
BATCH_BUCKETS = ((48, 40), (96, 80), (144, 128), (192, 176))


def candidates(kind: int, dtype: int, nz: int) -> list[tuple[int, int, int]]:
    """Tile shapes that have an instantiated kernel for this kind and dtype."""
    if kind == G.K_IMG_BOX5_LAP:
        return [(4, 4, cy) for cy in (4, 8, 16, 32, 64)]
    if kind in BLOCKED:
        # fixed 16-wave block shape: only the z chunk (output planes) varies
        return [(1, 16, cz) for cz in (1, 2, 4, 8, 16, 32, 64) if cz <= max(nz, 1)]
    if kind in RADIUS2:
        # one-field operators run NW = 4 only; shapes without a kernel are
        # skipped by the tuner (the launch reports them as unsupported)
        vs, nws = ((1,) if dtype == G.F64 else (1, 2)), (4, 6, 8)
    elif dtype == G.F64:
        vs, nws = (1, 2), (4, 8)
    else:
        vs, nws = (1, 2, 4), (4, 8)
    czs = [c for c in (1, 2, 4, 8, 16, 32, 64) if c <= max(nz, 1)]
    return [(v, nw, cz) for v, nw, cz in itertools.product(vs, nws, czs)]


def _key(arch: str, kind: int, g: "G.Grid") -> str:
    d = g.desc
    return f"{arch}|{kind}|{d.dtype}|{d.n[0]}x{d.n[1]}x{d.n[2]}"


def _arch() -> str:
    import torch
    try:
        return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    except Exception:
        return "gfx950"


def time_call(fn: Callable[[], None], reps: int = 10, warmup: int = 2, stream=None) -> float:
    """Mean milliseconds of fn() with HIP events on `stream` (the stream fn
    launches on; default the current stream)."""
    import torch
    for _ in range(warmup):
        fn()
    s = torch.cuda.Event(enable_timing=True)
    e = torch.cuda.Event(enable_timing=True)
    s.record(stream)
    for _ in range(reps):
        fn()
    e.record(stream)
    e.synchronize()
    return s.elapsed_time(e) / reps


class Tuner:
    def __init__(self, ctx: "G.Context", cache_path: str | None = DEFAULT_CACHE):
        self.ctx = ctx
        self.cache_path = cache_path
        self.arch = _arch()
        self.table: dict[str, dict] = {}
        if cache_path and os.path.exists(cache_path):
            with open(cache_path) as f:
                self.table = json.load(f)

    def tune(self, kind: int, ins: Sequence["G.Grid"], outs: Sequence["G.Grid"], p: Iterable[float] = (),
             terms=None, cands: list | None = None, reps: int = 10, force: bool = False) -> dict:
        """Pick the fastest tile for do_all(kind, ins, outs, p) and install it."""
        ref = ins[0]
        key = _key(self.arch, kind, ref)
        if not force and key in self.table:
            rec = self.table[key]
            self.ctx.tile_set(kind, ref, tuple(rec["tile"]))
            return rec
        p = tuple(p)
        cands = cands or candidates(kind, ref.desc.dtype, ref.desc.n[2])
        results = []
        for tile in cands:
            self.ctx.tile_set(kind, ref, tile)
            try:
                ms = time_call(lambda: self.ctx.do_all(kind, ins, outs, p=p, terms=terms), reps=reps,
                               stream=self.ctx.stream)
            except G.GsclError:
                continue
            results.append((ms, tile))
        if not results:
            raise RuntimeError("no tile candidate ran")
        results.sort()
        ms, tile = results[0]
        self.ctx.tile_set(kind, ref, tile)
        rec = {"tile": list(tile), "us": ms * 1e3,
               "tried": [[list(t), round(m * 1e3, 2)] for m, t in results]}
        self.table[key] = rec
        return rec

    def apply(self, kind: int, grid: "G.Grid") -> bool:
        """Install a cached tile for (kind, grid extents) if there is one."""
        rec = self.table.get(_key(self.arch, kind, grid))
        if rec:
            self.ctx.tile_set(kind, grid, tuple(rec["tile"]))
            return True
        return False

    def tune_batch(self, precision: int = G.PREC_F32_IR, method: int = G.BATCH_JACOBI,
                   sweeps_per_step: int = 64, sweeps_per_pass: int = 4, buckets=BATCH_BUCKETS,
                   slots: int = 8, reps: int = 3, force: bool = False) -> list[tuple]:
        """Tile rule [(edge, cz, tb_cz), ...] for a batch of this
        configuration: per bucket, the (cz, tb_cz) whose step is fastest on a
        batch of `slots` requests of the bucket's size (never converging
        during the timing)."""
        import numpy as np
        import torch
        ctx = self.ctx
        rules = []
        for edge, n in buckets:
            key = f"batch|{self.arch}|p{precision}|m{method}|S{sweeps_per_step}|k{sweeps_per_pass}|{edge}"
            if not force and key in self.table:
                rules.append((edge, *self.table[key]["rule"]))
                continue
            shape = (n, n, n)
            f = ctx.grid(shape, G.F64, halo=0, data=np.random.default_rng(n).standard_normal(shape))
            us = [ctx.grid(shape, G.F64, halo=1) for _ in range(slots)]
            czs = (4, 8, 16)
            tbs = (4, 8, 16, 32) if sweeps_per_pass > 1 else (0,)
            results = []
            for cz in czs:
                for tb in tbs:
                    probe = G.Batch(ctx, max_slots=slots, precision=precision, hbm_budget=1 << 20, method=method,
                                    sweeps_per_step=sweeps_per_step, sweeps_per_pass=sweeps_per_pass)
                    budget = int(slots * probe.footprint(shape) * 1.25) + (64 << 20)
                    probe.close()
                    b = G.Batch(ctx, max_slots=slots, precision=precision, sweeps_per_step=sweeps_per_step,
                                rtol=1e-300, hbm_budget=budget, method=method, omega=6 / 7 if method == G.BATCH_JACOBI
                                else 0.0, sweeps_per_pass=sweeps_per_pass, max_sweeps=10 ** 9)
                    b.set_tile_rule([(edge, cz, tb)])
                    for u in us:
                        u.fill(0.0)
                        assert b.admit(u, f, 1.0 / (n + 1) ** 2) is not None
                    ms = time_call(b.step, reps=reps, warmup=1, stream=ctx.stream)
                    b.close()
                    results.append((ms, (cz, tb)))
            del us, f
            torch.cuda.empty_cache()
            results.sort()
            ms, best = results[0]
            self.table[key] = {"rule": list(best), "ms_per_step": round(ms, 4),
                               "tried": [[list(t), round(m, 4)] for m, t in results]}
            rules.append((edge, *best))
        return rules

    def save(self, path: str | None = None):
        path = path or self.cache_path
        if not path:
            return
        os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(self.table, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
