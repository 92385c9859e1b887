"""Tile autotuner for the tiled do_all kernels (autotuning is the paper's
stated future work, Section 2 and Section 6).

For one operator kind and one set of grid extents it times every candidate
tile shape (V elements per lane, NW waves per block, cz planes per block) with
HIP events, keeps the fastest, installs it in the context with
``gscl_tile_set`` and records it in a JSON cache keyed by
(gfx arch, kind, dtype, extents).  Outputs do not depend on the tile shape
(only the fused-reduction rounding order does), so tuning never changes a
do_all result.
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

    def save(self, path: str | None = None):
        path = path or self.cache_path
        if not path:
            return
        os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(self.table, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
