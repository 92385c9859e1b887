#!/usr/bin/env python3
"""Benchmark of the stencil hot path on one MI355X.

Default workload: the multi-grid variable-coefficient sweep -- 256^3 FP32,
7-point operator with 7 coefficient grids, a source grid and the field (9
input grids), writing 3 output grids (new u, residual, flux magnitude),
periodic boundaries, 100 sweeps with the L2 norm of the residual fused into
every 10th sweep.  One step = those 100 sweeps (and 10 reductions, whose
results stay on the device).  Inputs are resident in HBM before timing.

Prints one JSON line with Gpts/s (value), algorithmic HBM GB/s and its
fraction of the 8 TB/s peak for the dominant kernel (HIP events around every
sweep of the timed region), and a CPU baseline: the FP64 oracle on the host
cores over a bounded sample of the same workload.

Other workloads (--config) print the same fields for development use.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "stencil Gpts/s + HBM GB/s vs peak; batched solves/s with p50/p99 latency"
HBM_PEAK_GBS = 8000.0
_CS = "paper_1207_1746_amd/csrc/"
KERNEL_SOURCES = {
    "varcoef7_256_f32": [_CS + f for f in ("kcommon.h", "tiled.h", "ops.h", "sweeps_common.h",
                                          "k_sweep_varcoef.hip")],
    "wjacobi_f64": [_CS + f for f in ("kcommon.h", "tiled.h", "ops.h", "sweeps_common.h",
                                     "k_sweep_wjacobi.hip")],
    "image_8192_u8": [_CS + f for f in ("kcommon.h", "k_image.hip")],
    "reduce_f64": [_CS + f for f in ("kcommon.h", "k_reduce.hip")],
    "wjacobi_tb_512": [_CS + f for f in ("kcommon.h", "tiled.h", "ops.h", "tb7.h", "k_sweep_tb.hip")],
    "rbgs_512": [_CS + f for f in ("kcommon.h", "tiled.h", "ops.h", "sweeps_common.h", "k_sweep_wjacobi.hip")],
    "rbgs_tb_512": [_CS + f for f in ("kcommon.h", "tiled.h", "ops.h", "tb7.h", "k_sweep_tb.hip")],
    "tridiag_512": [_CS + f for f in ("kcommon.h", "launch.h", "k_line.hip")],
    "vc13_512": [_CS + f for f in ("kcommon.h", "tiled.h", "zq13.h", "ops.h", "sweeps_common.h",
                                  "k_sweep_vc13a.hip")],
}


def kernel_hash(workload_key: str = "varcoef7_256_f32") -> str:
    """Hash of the sources the workload's dominant kernel is built from."""
    h = hashlib.sha256()
    for p in KERNEL_SOURCES[workload_key]:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(workload_key: str):
    """HBM bytes per launch of the dominant kernel from the committed
    rocprofv3 counter summary (profiles/<key>_traffic.md), if the counters were
    taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", f"{workload_key}_traffic.md")
    if not os.path.exists(path):
        return None
    rec = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            rec[k.strip("- *`").strip()] = v.strip().strip("`")
    if rec.get("kernel_hash") != kernel_hash(workload_key):
        return None
    try:
        return float(rec["bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def sync():
    import torch
    torch.cuda.synchronize()


# --------------------------------------------------------------------------- #
# workloads
# --------------------------------------------------------------------------- #
class VarCoef:
    key = "varcoef7_256_f32"
    bytes_per_point = 48  # read u, c0..c6, s (9 x 4 B), write u', r, |F| (3 x 4 B)
    event_stride = 1      # one window per run of 9 plain sweeps between fused reductions

    def __init__(self, ctx, n=256, sweeps=100, every=10):
        import torch
        import paper_1207_1746_amd as G
        from paper_1207_1746_amd import workloads as W
        self.G = G
        self.n, self.sweeps, self.every = n, sweeps, every
        u, c, s = W.varcoef_grids(n)
        self.host = (u, c, s)
        shp = (n, n, n)
        self.gu = ctx.grid(shp, G.F32, halo=1, bc=G.PERIODIC, data=u)
        self.gu2 = ctx.grid(shp, G.F32, halo=1, bc=G.PERIODIC)
        self.gc = [ctx.grid(shp, G.F32, halo=0, data=x) for x in c]
        self.gs = ctx.grid(shp, G.F32, halo=0, data=s)
        self.gr = ctx.grid(shp, G.F32, halo=0)
        self.gf = ctx.grid(shp, G.F32, halo=0)
        self.norms = torch.zeros(sweeps // every, dtype=torch.float64, device="cuda")
        self.ctx = ctx
        self.points = n ** 3
        self.units_per_step = self.points * sweeps
        self.unit = "Gpts/s"

    def step(self, ev=None):
        G = self.G
        ping = (self.gu, self.gu2)
        run = 0  # plain sweeps in the open event window
        for k in range(1, self.sweeps + 1):
            src, dst = ping[(k - 1) % 2], ping[k % 2]
            red = k % self.every == 0
            if ev is not None and not red and run == 0:
                ev.begin()
            self.ctx.do_all(G.K_VARCOEF7, [src] + self.gc + [self.gs], [dst, self.gr, self.gf],
                            reduce=(G.R_L2, G.RV_RESIDUAL) if red else None,
                            dev_result=self.norms[k // self.every - 1] if red else None)
            if not red:
                run += 1
            # close the window after the last plain sweep before a fused one
            if ev is not None and run and ((k + 1) % self.every == 0 or k == self.sweeps):
                ev.end(run)
                run = 0

    def config(self):
        return {"workload": f"multi-grid variable-coefficient 7-point sweep, {self.n}^3 FP32, "
                            "9 input grids (u, c0..c6, s) -> 3 outputs (u', r, |F|), periodic, "
                            f"{self.sweeps} sweeps, fused L2(r) every {self.every}",
                "grid": [self.n] * 3, "sweeps_per_step": self.sweeps, "reduce_every": self.every,
                "launch": "tiled z-march, tile " + str(self.ctx.tile_get(self.G.K_VARCOEF7, self.gu))}

    def cpu_baseline(self, budget_s=10.0):
        """The oracle on the same inputs: whole 100-sweep passes (restarting
        from u0) until about budget_s of CPU work has been done."""
        import numpy as np
        import oracle
        u, c, s = self.host
        cp = np.ascontiguousarray(np.stack([ci.astype(np.float64) for ci in c]))
        sd = s.astype(np.float64)
        t0 = time.perf_counter()
        done = 0
        while True:
            x = u.astype(np.float64)
            for k in range(1, self.sweeps + 1):
                x, r, _ = oracle.varcoef7_sweep(x, cp, sd)
                done += 1
                if k % self.every == 0:
                    oracle.sumsq(r)
                if time.perf_counter() - t0 >= 3 * budget_s:
                    break
            if time.perf_counter() - t0 >= budget_s:
                break
        dt = time.perf_counter() - t0
        return {"value": round(self.points * done / dt / 1e9, 4), "unit": self.unit,
                "cores": oracle.num_threads(), "kind": "oracle",
                "sample": f"FP64 oracle, {done} sweeps ({done / self.sweeps:g} passes of the "
                          f"{self.sweeps}-sweep workload) on the same {self.n}^3 inputs in {dt:.1f} s, "
                          f"residual norms every {self.every}"}


class Jacobi:
    key = "wjacobi_f64"
    bytes_per_point = 16
    event_stride = 3      # time every 3rd of the 9 plain sweeps (30 per 10-step run)

    def __init__(self, ctx, n=64, sweeps=10):
        import torch
        import paper_1207_1746_amd as G
        from paper_1207_1746_amd import workloads as W
        self.G = G
        self.n, self.sweeps = n, sweeps
        u0, self.h2 = W.jacobi_cube(n)
        self.host = u0
        self.a = ctx.grid(u0.shape, G.F64, halo=1, data=u0)
        self.b = ctx.grid(u0.shape, G.F64, halo=1)
        self.res = torch.zeros(1, dtype=torch.float64, device="cuda")
        self.ctx = ctx
        self.points = n ** 3
        self.units_per_step = self.points * sweeps
        self.unit = "Gpts/s"
        # the ten launches of a step, with their arguments built once
        self.calls = []
        for k in range(sweeps):
            src, dst = (self.a, self.b) if k % 2 == 0 else (self.b, self.a)
            last = k == sweeps - 1
            self.calls.append(ctx.prepare_all(G.K_WJACOBI, [src], [dst], p=(1.0, self.h2),
                                              reduce=(G.R_L2, G.RV_UPDATE) if last else None,
                                              dev_result=self.res if last else None))

    def step(self, ev=None):
        last = len(self.calls) - 1
        for k, call in enumerate(self.calls):
            if ev is not None and k != last:
                ev.begin()
            call()
            if ev is not None and k != last:
                ev.end()

    def config(self):
        return {"workload": f"Jacobi 7-point {self.n}^3 FP64, Dirichlet 0, {self.sweeps} sweeps + L2 of update",
                "grid": [self.n] * 3}

    def cpu_baseline(self, budget_s=10.0):
        import oracle
        t0 = time.perf_counter()
        reps = 0
        while True:
            oracle.jacobi_run(self.host, self.sweeps, None, 1.0, self.h2)
            reps += 1
            if time.perf_counter() - t0 > budget_s:
                break
        dt = time.perf_counter() - t0
        return {"value": round(self.units_per_step * reps / dt / 1e9, 4), "unit": self.unit,
                "cores": oracle.num_threads(), "kind": "oracle",
                "sample": f"{reps} full runs of the workload in {dt:.1f} s"}


class JacobiTB:
    """Weighted Jacobi with a right-hand side on a 512^3 FP64 cube, Dirichlet
    0: 16 sweeps per step as four temporally blocked passes of 4 sweeps (the
    last with the fused L2 norm of its update).  The same 16 sweeps as plain
    one-sweep passes are timed beside it; both give the same grid bit for bit."""
    key = "wjacobi_tb_512"
    bytes_per_point = 24  # per pass: u and f read once, the 4-sweep result written once

    def __init__(self, ctx, n=512, sweeps=16, k=4):
        import torch
        import paper_1207_1746_amd as G
        from paper_1207_1746_amd import workloads as W
        self.G = G
        self.n, self.sweeps, self.k = n, sweeps, k
        u0, self.h2 = W.jacobi_cube(n)
        f = W.jacobi_rhs(n)
        self.host = (u0, f)
        self.a = ctx.grid(u0.shape, G.F64, halo=1, data=u0)
        self.b = ctx.grid(u0.shape, G.F64, halo=1)
        self.f = ctx.grid(u0.shape, G.F64, halo=0, data=f)
        self.res = torch.zeros(1, dtype=torch.float64, device="cuda")
        self.ctx = ctx
        self.points = n ** 3
        self.units_per_step = self.points * sweeps
        self.unit = "Gpts/s"
        self.extra = {}

    def _run(self, kind, k, ev=None):
        G = self.G
        passes = self.sweeps // k
        for q in range(passes):
            src, dst = (self.a, self.b) if q % 2 == 0 else (self.b, self.a)
            last = q == passes - 1
            if ev is not None and not last:
                ev.begin()
            self.ctx.do_all(kind, [src, self.f], [dst], p=(6 / 7, self.h2, k),
                            reduce=(G.R_L2, G.RV_UPDATE) if last else None,
                            dev_result=self.res if last else None)
            if ev is not None and not last:
                ev.end()

    def step(self, ev=None):
        self._run(self.G.K_WJACOBI_TB, self.k, ev)

    def after(self):
        """The same sweeps as plain passes, and the per-sweep comparison."""
        import torch
        self._run(self.G.K_WJACOBI, 1)
        sync()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 3
        a.record()
        for _ in range(reps):
            self._run(self.G.K_WJACOBI, 1)
        b.record()
        sync()
        ms = a.elapsed_time(b) / reps
        self.extra = {"plain_sweeps": {"ms_per_step": round(ms, 3),
                                       "Gpts_s": round(self.units_per_step / ms / 1e6, 2),
                                       "GBs": round(24 * self.units_per_step / ms / 1e6, 1)},
                      "sweeps_per_pass": self.k,
                      "note": "a pass reads u and f once and writes once for 4 sweeps"}

    def config(self):
        return {"workload": f"weighted Jacobi 7-point {self.n}^3 FP64 with right-hand side, Dirichlet 0, "
                            f"{self.sweeps} sweeps per step as temporally blocked passes of {self.k} "
                            f"+ L2 of the last update", "grid": [self.n] * 3}

    def cpu_baseline(self, budget_s=10.0):
        import oracle
        u0, f = self.host
        t0 = time.perf_counter()
        reps = 0
        u = u0
        while True:
            u, _, _ = oracle.wjacobi_sweep(u, f, 6 / 7, self.h2)
            reps += 1
            if time.perf_counter() - t0 > budget_s:
                break
        dt = time.perf_counter() - t0
        return {"value": round(self.points * reps / dt / 1e9, 4), "unit": self.unit,
                "cores": oracle.num_threads(), "kind": "oracle",
                "sample": f"{reps} single FP64 sweeps of the 512^3 workload in {dt:.1f} s"}


class RBGS:
    """Red-black relaxation on a 512^3 FP64 cube with a right-hand side,
    Dirichlet 0: a step is 8 sweeps (16 in-place colour passes).  Beside it,
    one Poisson request at N = 192 is solved to 1e-8 by weighted Jacobi
    (omega 6/7) and by optimal red-black SOR (reported as extras)."""
    key = "rbgs_512"
    bytes_per_point = 24  # per colour pass: u and f read, u written

    def __init__(self, ctx, n=512, sweeps=8):
        import torch
        import paper_1207_1746_amd as G
        from paper_1207_1746_amd import workloads as W
        self.G, self.W = G, W
        self.n, self.sweeps = n, sweeps
        u0, self.h2 = W.jacobi_cube(n)
        f = W.jacobi_rhs(n)
        self.host = (u0, f)
        self.u = ctx.grid(u0.shape, G.F64, halo=1, data=u0)
        self.f = ctx.grid(u0.shape, G.F64, halo=0, data=f)
        self.res = torch.zeros(1, dtype=torch.float64, device="cuda")
        self.ctx = ctx
        self.points = n ** 3
        self.units_per_step = self.points * sweeps
        self.unit = "Gpts/s"
        self.omega = 1.9
        self.extra = {}

    def step(self, ev=None):
        G = self.G
        for q in range(2 * self.sweeps):
            last = q == 2 * self.sweeps - 1
            if ev is not None and not last:
                ev.begin()
            self.ctx.do_all(G.K_RBGS, [self.u, self.f], [self.u], p=(self.omega, self.h2, q % 2),
                            reduce=(G.R_L2, G.RV_UPDATE) if last else None,
                            dev_result=self.res if last else None)
            if ev is not None and not last:
                ev.end()

    def after(self):
        G, W = self.G, self.W
        req = W.poisson_requests(count=1, qps=float("inf"), nmin=192, nmax=192, seed_index=7)[0]
        _, f = W.poisson_fields(req)
        gf = self.ctx.grid(f.shape, G.F64, halo=0, data=f)
        out = {}
        for name, kind, omega in (("weighted_jacobi", G.K_WJACOBI, 6 / 7), ("rb_gauss_seidel", G.K_RBGS, 1.0),
                                  ("rb_sor_optimal", G.K_RBGS, 0.0)):
            u = self.ctx.grid(f.shape, G.F64, halo=1).fill(0.0)
            t0 = time.perf_counter()
            st = self.ctx.solve(kind, [u], [gf], omega=omega, h2=req.h2, rtol=1e-8, check_every=16)
            sec = time.perf_counter() - t0
            out[name] = {"sweeps": st["sweeps"], "seconds": round(sec, 4),
                         "rel_residual": st["rel_residual"]}
        self.extra = {"poisson_192_to_1e-8": out}

    def config(self):
        return {"workload": f"red-black SOR (omega {self.omega}) 7-point {self.n}^3 FP64 with right-hand side, "
                            f"Dirichlet 0, {self.sweeps} sweeps = {2 * self.sweeps} in-place colour passes "
                            f"+ L2 of the last update", "grid": [self.n] * 3}

    def cpu_baseline(self, budget_s=10.0):
        import oracle
        u0, f = self.host
        t0 = time.perf_counter()
        reps = 0
        u = u0
        while True:
            u = oracle.rbgs_sweep(u, f, self.omega, self.h2)
            reps += 1
            if time.perf_counter() - t0 > budget_s:
                break
        dt = time.perf_counter() - t0
        return {"value": round(self.points * reps / dt / 1e9, 4), "unit": self.unit,
                "cores": oracle.num_threads(), "kind": "oracle",
                "sample": f"{reps} red-black FP64 sweeps of the 512^3 workload in {dt:.1f} s"}


class RBGSTB:
    """Red-black SOR (omega 1.9) on a 512^3 FP64 cube with a right-hand side,
    Dirichlet 0: 8 sweeps per step as four blocked passes of 4 colour passes
    (2 sweeps each, the last with the fused L2 norm of its update).  The same
    sweeps as in-place colour passes are timed beside it (the same grid, bit
    for bit), and one N = 192 Poisson request is solved by optimal SOR (its
    chunks run as blocked passes)."""
    key = "rbgs_tb_512"
    bytes_per_point = 24  # per blocked pass: u and f read once, the 4-pass result written once

    def __init__(self, ctx, n=512, sweeps=8, k=4):
        import torch
        import paper_1207_1746_amd as G
        from paper_1207_1746_amd import workloads as W
        self.G, self.W = G, W
        self.n, self.sweeps, self.k = n, sweeps, k
        u0, self.h2 = W.jacobi_cube(n)
        f = W.jacobi_rhs(n)
        self.host = (u0, f)
        self.a = ctx.grid(u0.shape, G.F64, halo=1, data=u0)
        self.b = ctx.grid(u0.shape, G.F64, halo=1)
        self.f = ctx.grid(u0.shape, G.F64, halo=0, data=f)
        self.res = torch.zeros(1, dtype=torch.float64, device="cuda")
        self.ctx = ctx
        self.points = n ** 3
        self.units_per_step = self.points * sweeps
        self.unit = "Gpts/s"
        self.omega = 1.9
        self.extra = {}

    def step(self, ev=None):
        G = self.G
        passes = 2 * self.sweeps // self.k
        for q in range(passes):
            src, dst = (self.a, self.b) if q % 2 == 0 else (self.b, self.a)
            last = q == passes - 1
            if ev is not None and not last:
                ev.begin()
            self.ctx.do_all(G.K_RBGS_TB, [src, self.f], [dst], p=(self.omega, self.h2, (q * self.k) % 2, self.k),
                            reduce=(G.R_L2, G.RV_UPDATE) if last else None,
                            dev_result=self.res if last else None)
            if ev is not None and not last:
                ev.end()

    def _inplace(self):
        G = self.G
        for q in range(2 * self.sweeps):
            self.ctx.do_all(G.K_RBGS, [self.a, self.f], [self.a], p=(self.omega, self.h2, q % 2))

    def after(self):
        import torch
        G, W = self.G, self.W
        self._inplace()
        sync()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 3
        a.record()
        for _ in range(reps):
            self._inplace()
        b.record()
        sync()
        ms = a.elapsed_time(b) / reps
        req = W.poisson_requests(count=1, qps=float("inf"), nmin=192, nmax=192, seed_index=7)[0]
        _, f = W.poisson_fields(req)
        gf = self.ctx.grid(f.shape, G.F64, halo=0, data=f)
        u = self.ctx.grid(f.shape, G.F64, halo=1).fill(0.0)
        t0 = time.perf_counter()
        st = self.ctx.solve(G.K_RBGS, [u], [gf], omega=0.0, h2=req.h2, rtol=1e-8, check_every=16)
        sec = time.perf_counter() - t0
        self.extra = {"inplace_colour_passes": {"ms_per_step": round(ms, 3),
                                                "Gpts_s": round(self.units_per_step / ms / 1e6, 2)},
                      "colour_passes_per_blocked_pass": self.k,
                      "poisson_192_sor_to_1e-8": {"sweeps": st["sweeps"], "seconds": round(sec, 4),
                                                  "rel_residual": st["rel_residual"]}}

    def config(self):
        return {"workload": f"red-black SOR (omega {self.omega}) 7-point {self.n}^3 FP64 with right-hand side, "
                            f"Dirichlet 0, {self.sweeps} sweeps per step as blocked passes of {self.k} colour "
                            f"passes + L2 of the last update", "grid": [self.n] * 3}

    def cpu_baseline(self, budget_s=10.0):
        import oracle
        u0, f = self.host
        t0 = time.perf_counter()
        reps = 0
        u = u0
        while True:
            u = oracle.rbgs_sweep(u, f, self.omega, self.h2)
            reps += 1
            if time.perf_counter() - t0 > budget_s:
                break
        dt = time.perf_counter() - t0
        return {"value": round(self.points * reps / dt / 1e9, 4), "unit": self.unit,
                "cores": oracle.num_threads(), "kind": "oracle",
                "sample": f"{reps} red-black FP64 sweeps of the 512^3 workload in {dt:.1f} s"}


class Tridiag:
    """Ordered line iteration spaces: tridiagonal solves along k (do_k_inc
    elimination, do_k_dec substitution) for every column of a 512^3 FP64
    grid (diagonally dominant systems)."""
    key = "tridiag_512"
    bytes_per_point = 48  # elimination: lo, di, up, rhs read; cp, dp written

    def __init__(self, ctx, n=512):
        import torch
        import paper_1207_1746_amd as G
        self.G = G
        shape = (n, n, n)
        gen = torch.Generator(device="cuda").manual_seed(12071746)
        self.grids = []
        for lo, hi in ((-1.0, 1.0), (2.5, 3.5), (-1.0, 1.0), (-1.0, 1.0)):
            g = ctx.grid(shape, G.F64, halo=0)
            g.view.copy_(torch.rand(shape, dtype=torch.float64, device="cuda", generator=gen) * (hi - lo) + lo)
            self.grids.append(g)
        self.cp, self.dp, self.x = (ctx.grid(shape, G.F64, halo=0) for _ in range(3))
        self.ctx, self.n = ctx, n
        self.points = n ** 3
        self.units_per_step = self.points
        self.unit = "Gpts/s"

    def step(self, ev=None):
        G = self.G
        if ev is not None:
            ev.begin()
        self.ctx.do_line(G.K_TRIDIAG_FWD, 2, 1, self.grids, [self.cp, self.dp])
        if ev is not None:
            ev.end()
        self.ctx.do_line(G.K_TRIDIAG_BACK, 2, -1, [self.cp, self.dp], [self.x])

    def config(self):
        return {"workload": f"tridiagonal solves along k for {self.n}^2 columns of {self.n} levels, FP64 "
                            f"(do_k_inc elimination + do_k_dec substitution)", "grid": [self.n] * 3}

    def cpu_baseline(self, budget_s=10.0):
        import numpy as np
        import oracle
        m = 64  # a bounded sample: 64 x 64 columns of the full depth
        arrs = [g.view[:, :m, :m].cpu().numpy() for g in self.grids]
        t0 = time.perf_counter()
        reps = 0
        while True:
            oracle.tridiag_solve(*arrs, 2, 1)
            reps += 1
            if time.perf_counter() - t0 > budget_s:
                break
        dt = time.perf_counter() - t0
        return {"value": round(self.n * m * m * reps / dt / 1e9, 4), "unit": self.unit,
                "cores": oracle.num_threads(), "kind": "oracle",
                "sample": f"{reps} solves of 64 x 64 columns x {self.n} levels in {dt:.1f} s"}


class Image:
    key = "image_8192_u8"
    bytes_per_point = 4  # read 1 B, write 1 B box + 2 B Laplacian

    def __init__(self, ctx, n=8192, planes=4):
        import paper_1207_1746_amd as G
        from paper_1207_1746_amd import workloads as W
        self.G = G
        img = W.image_planes(n, n, planes)
        self.host = img
        self.gi = ctx.grid(img.shape, G.U8, halo=2, bc=G.CLAMP, ndim=2, data=img)
        self.gb = ctx.grid(img.shape, G.U8, halo=0, ndim=2)
        self.gl = ctx.grid(img.shape, G.I16, halo=0, ndim=2)
        self.ctx = ctx
        self.points = n * n * planes
        self.units_per_step = self.points
        self.unit = "Gpx/s"
        self.n, self.planes = n, planes

    def step(self, ev=None):
        if ev is not None:
            ev.begin()
        self.ctx.do_all(self.G.K_IMG_BOX5_LAP, [self.gi], [self.gb, self.gl], p=(4,))
        if ev is not None:
            ev.end()

    def config(self):
        return {"workload": f"5x5 box + 3x3 Laplacian, {self.planes} x {self.n}^2 uint8, clamp"}

    def cpu_baseline(self, budget_s=10.0):
        import oracle
        t0 = time.perf_counter()
        reps = 0
        while True:
            oracle.img(self.host[:1], 4)
            reps += 1
            if time.perf_counter() - t0 > budget_s:
                break
        dt = time.perf_counter() - t0
        return {"value": round(self.n * self.n * reps / dt / 1e9, 4), "unit": self.unit,
                "cores": oracle.num_threads(), "kind": "oracle",
                "sample": f"{reps} single planes in {dt:.1f} s"}


class Serve:
    """Stream of Poisson solve requests with cube sides log-uniform in
    [32, 192]: batched mixed-precision serving (continuous batching, F32
    correction sweeps as temporally blocked passes of 4, F64 residual) against
    one solve at a time with the plain F64 solver, both to the same relative
    residual.

    The requests are the first `count` of the seeded 2000-request stream (its
    size mix, modes and arrival order).  The sequential F64 path, run closed
    loop, gives the service rate mu; the batched path runs closed loop (every
    request queued at t = 0, its capacity is the value) and with Poisson
    arrivals offered at 0.5, 1 and 2 x mu (the stream's exponential gaps
    rescaled), for latency.  The oracle recomputes the FP64 relative residual
    of every returned answer of every run."""
    key = "serve"
    bytes_per_point = 12  # F32 correction sweep: read d, rhs; write d'

    # sweeps between residual checks, the same for the batched and the
    # one-at-a-time paths and the oracle (measured on MI355X: 64 -> 256 made
    # the batched path 18% and the one-at-a-time path 4% faster; 512 was
    # slower for both)
    CHECK = 256

    def __init__(self, ctx, count=100, nmin=32, nmax=192, rtol=1e-10, stream=2000, sor=False):
        import paper_1207_1746_amd as G
        from paper_1207_1746_amd import serve as SV
        from paper_1207_1746_amd import workloads as W
        self.G, self.SV, self.W = G, SV, W
        self.ctx = ctx
        # unit-rate arrivals; rescaled per run
        self.reqs = W.poisson_requests(count=stream, qps=1.0, nmin=nmin, nmax=nmax, seed_index=1)[:count]
        self.fields = {r.rid: W.poisson_fields(r)[1] for r in self.reqs}
        self.rtol = rtol
        self.count, self.nmin, self.nmax, self.stream = count, nmin, nmax, stream
        self.with_sor = sor
        # z chunks of the batched kernels per request-size bucket, picked by
        # the tuner on this GPU before any request is served
        from paper_1207_1746_amd import autotune
        t0 = time.perf_counter()
        self.tuner = autotune.Tuner(ctx, cache_path=None)
        self.tile_rule = self.tuner.tune_batch(precision=G.PREC_F32_IR, sweeps_per_step=self.CHECK,
                                               sweeps_per_pass=4)
        self.tune_seconds = time.perf_counter() - t0
        self.unit = "solves/s"
        self.points = 1
        self.units_per_step = count
        self.last = {}
        self.mu = None

    @staticmethod
    def _progress(what):
        """Completion callback: one stderr line per 10 finished requests."""
        count = [0]

        def done(job):
            count[0] += 1
            if count[0] % 10 == 0:
                print(f"[serve] {what}: {count[0]} requests done (last N = {job.n})", file=sys.stderr, flush=True)
        return done

    def _jobs(self, qps=None):
        return [self.SV.Job(r.rid, r.n, r.h2, 0.0 if qps is None else r.arrival / qps,
                            self.ctx.grid((r.n,) * 3, self.G.F64, halo=0, data=self.fields[r.rid]))
                for r in self.reqs]

    def _check(self, jobs, summary):
        """The oracle's FP64 relative residual of every returned answer."""
        import math
        import oracle
        ok, worst = 0, 0.0
        h2 = {r.rid: r.h2 for r in self.reqs}
        for j in jobs:
            if j.state != 2 or j.u is None:
                continue
            f = self.fields[j.rid]
            _, _, res = oracle.wjacobi_sweep(j.u.numpy(), f, 6 / 7, h2[j.rid])
            rel = math.sqrt(oracle.sumsq(res) / oracle.sumsq(f))
            worst = max(worst, rel)
            ok += rel <= self.rtol * 1.01
            j.u = None
        summary["oracle_checked"] = sum(1 for j in jobs if j.state == 2)
        summary["oracle_within_rtol"] = ok
        summary["oracle_worst_rel_residual"] = "%.3e" % worst
        return summary

    def _batched(self, qps=None):
        jobs = self._jobs(qps)
        srv = self.SV.SolveServer(self.ctx, precision=self.G.PREC_F32_IR, sweeps_per_step=self.CHECK,
                                  rtol=self.rtol, max_slots=64, tile_rule=self.tile_rule)
        rep = srv.run(jobs, realtime=qps is not None,
                      on_done=self._progress("batched" + ("" if qps is None else f" at {qps:.3g}/s")))
        srv.close()
        out = rep.summary()
        if qps is not None:
            out["offered_qps"] = round(qps, 3)
        return self._check(jobs, out)

    def step(self, ev=None):
        self.last["batched"] = self._batched()

    def sequential(self):
        jobs = self._jobs()
        rep = self.SV.serve_sequential(self.ctx, jobs, rtol=self.rtol, check_every=self.CHECK, realtime=False,
                                       on_done=self._progress("sequential f64"))
        out = self._check(jobs, rep.summary())
        self.mu = out["solves_per_s"]
        return out

    def loaded(self, factor):
        """Poisson arrivals offered at `factor` x the sequential service rate."""
        return self._batched(factor * self.mu)

    def sor(self):
        """The same requests solved by optimal red-black SOR in F64 (O(N)
        sweeps instead of O(N^2)): batched (continuous batching, a residual
        check every 8 sweeps) and one solve at a time, both closed-loop."""
        jobs = self._jobs()
        srv = self.SV.SolveServer(self.ctx, precision=self.G.PREC_F64, sweeps_per_step=8, rtol=self.rtol,
                                  omega=0.0, max_slots=64, method=self.G.BATCH_RBGS)
        bat = self._check(jobs, srv.run(jobs, realtime=False).summary())
        srv.close()
        jobs = self._jobs()
        seq = self._check(jobs, self.SV.serve_sequential(self.ctx, jobs, rtol=self.rtol, omega=0.0, check_every=8,
                                                         realtime=False, kind=self.G.K_RBGS).summary())
        return bat, seq

    def cpu_baseline(self, budget_s=20.0):
        """The oracle's checked weighted-Jacobi solve (FP64, same omega, rtol
        and check period as the sequential GPU path) on the sample's requests
        in increasing size, until about budget_s of CPU work: solves/s on
        that subsample of the smallest requests, an upper bound on the
        oracle's rate over the whole sample."""
        import oracle
        done, sizes = 0, []
        t0 = time.perf_counter()
        for r in sorted(self.reqs, key=lambda r: r.n):
            _, _, _, conv = oracle.poisson_solve(self.fields[r.rid], r.h2, 6 / 7, self.rtol, self.CHECK, 10 ** 7)
            assert conv
            done += 1
            sizes.append(r.n)
            if time.perf_counter() - t0 > budget_s:
                break
        dt = time.perf_counter() - t0
        return {"value": round(done / dt, 4), "unit": "solves/s", "cores": oracle.num_threads(), "kind": "oracle",
                "sample": f"the {done} smallest of the {self.count} requests (N = {min(sizes)}..{max(sizes)}) "
                          f"solved to {self.rtol} in {dt:.1f} s"}

    def config(self):
        ns = sorted(r.n for r in self.reqs)
        return {"workload": f"Poisson solve requests, cube sides log-uniform in [{self.nmin},{self.nmax}]: the first "
                            f"{self.count} of the seeded {self.stream}-request stream (N = {ns[0]}..{ns[-1]}, "
                            f"{sum(1 for n in ns if n >= 144)} with N >= 144), 3 sine modes, weighted Jacobi "
                            f"omega=6/7 to relative residual {self.rtol:g}, residual checked every {self.CHECK} "
                            "sweeps; value = batched closed-loop capacity; "
                            "latency with Poisson arrivals at 0.5, 1 and 2 x the sequential F64 rate",
                "rtol": self.rtol, "requests": self.count, "n_range": [self.nmin, self.nmax],
                "serving": "continuous batching, F32 correction sweeps (temporally blocked passes of 4) + "
                           "F64 residual (refinement)",
                "batch_tile_rule": {"rule (largest extent <=, one-sweep cz, blocked-pass cz)": self.tile_rule,
                                    "tuned_in_s": round(self.tune_seconds, 1)}}


class Reduce:
    """Standalone do_reduce: L2 norm of a 512^3 FP64 grid (8 B per point)."""
    key = "reduce_f64"
    bytes_per_point = 8

    def __init__(self, ctx, n=512):
        import torch
        import paper_1207_1746_amd as G
        self.G = G
        self.g = ctx.grid((n, n, n), G.F64, halo=0)
        self.g.view.copy_(torch.rand(n, n, n, dtype=torch.float64, device="cuda"))
        self.res = torch.zeros(1, dtype=torch.float64, device="cuda")
        self.ctx, self.n = ctx, n
        self.points = n ** 3
        self.units_per_step = self.points
        self.unit = "Gpts/s"

    def step(self, ev=None):
        if ev is not None:
            ev.begin()
        self.ctx.do_reduce(self.G.R_L2, self.g, dev_result=self.res)
        if ev is not None:
            ev.end()

    def config(self):
        return {"workload": f"do_reduce L2 norm of a {self.n}^3 FP64 grid"}

    def cpu_baseline(self, budget_s=10.0):
        import numpy as np
        import oracle
        x = self.g.view.cpu().numpy()
        t0 = time.perf_counter()
        reps = 0
        while time.perf_counter() - t0 < budget_s:
            oracle.sumsq(x)
            reps += 1
        dt = time.perf_counter() - t0
        return {"value": round(self.points * reps / dt / 1e9, 4), "unit": self.unit, "cores": 1,
                "kind": "oracle", "sample": f"{reps} pairwise sums of squares in {dt:.1f} s"}


class VC13:
    """Fourth-order 13-point operator on 5 fields sharing 10 coefficient grids,
    512^3.  The timed step is the BF16 apply; after it, per storage dtype
    (BF16, FP16, FP32; FP32 math): apply GB/s, the apply's error against the
    oracle, and an FP64-residual iterative-refinement solve to 1e-10."""
    key = "vc13_512"
    bytes_per_point = 40  # BF16: 5 fields + 10 coefficients read, 5 outputs written, 2 B each

    def __init__(self, ctx, n=512):
        import paper_1207_1746_amd as G
        from paper_1207_1746_amd import workloads as W
        self.G, self.W = G, W
        self.ctx, self.n = ctx, n
        self.c, self.b = W.vc13_grids(n)
        self.fields = W.vc13_fields(n)
        shp = (n, n, n)
        self.gc = [ctx.grid(shp, G.BF16, halo=0, data=x) for x in self.c]
        self.gf = [ctx.grid(shp, G.BF16, halo=2, data=x) for x in self.fields]
        self.go = [ctx.grid(shp, G.BF16, halo=0) for _ in range(5)]
        self.points = n ** 3
        self.units_per_step = self.points
        self.unit = "Gpts/s"
        self.extra = {}

    def step(self, ev=None):
        if ev is not None:
            ev.begin()
        self.ctx.do_all(self.G.K_VC13_APPLY, self.gf + self.gc, self.go, p=(self.W.VC13_KAPPA, 0, 5))
        if ev is not None:
            ev.end()

    def after(self):
        """Per storage dtype (BF16, FP16, FP32; FP32 math): apply time and GB/s,
        the apply's error against the oracle on a sampled field, and the
        FP64-residual refinement solve to 1e-10 with the oracle's recomputed
        FP64 residual of the answer."""
        import numpy as np
        import torch
        import oracle
        G, W, n = self.G, self.W, self.n
        shp = (n, n, n)
        out = {}
        kappa = W.VC13_KAPPA
        bn2 = sum(oracle.sumsq(x) for x in self.b)
        for dt, name, es, prec in ((G.BF16, "bf16", 2, G.PREC_BF16_IR), (G.F16, "f16", 2, G.PREC_F16_IR),
                                   (G.F32, "f32", 4, G.PREC_F32_IR)):
            rec = {}
            if dt == G.BF16:
                gc, gf, go = self.gc, self.gf, self.go
            else:
                gc = [self.ctx.grid(shp, dt, halo=0, data=x) for x in self.c]
                gf = [self.ctx.grid(shp, dt, halo=2, data=x) for x in self.fields]
                go = [self.ctx.grid(shp, dt, halo=0) for _ in range(5)]
            fn = lambda: self.ctx.do_all(G.K_VC13_APPLY, gf + gc, go, p=(kappa, 0, 5))
            fn()
            sync()
            ev = KernelEvents(self.ctx.stream)
            ev.begin()
            for _ in range(5):
                fn()
            ev.end(5)
            sync()
            ms, _ = ev.mean_ms()
            rec["apply_ms"] = round(ms, 4)
            rec["apply_Gpts_s"] = round(n ** 3 / ms / 1e6, 2)
            rec["apply_GBs"] = round(20 * es * n ** 3 / ms / 1e6, 1)
            rec["apply_frac_of_peak"] = round(20 * es * n ** 3 / ms / 1e6 / HBM_PEAK_GBS, 4)
            # error of the apply against the oracle on field 0 (stored values in FP64)
            stored = gf[0].numpy().astype(np.float64)
            ex = oracle.vc13_apply(stored, self.c, kappa)
            got = go[0].numpy().astype(np.float64)
            rec["apply_max_rel_err_field0"] = float("%.3e" % (np.abs(got - ex).max() / np.abs(ex).max()))
            del stored, ex, got
            if dt != G.BF16:
                del gf, go
            torch.cuda.empty_cache()
            # refinement to 1e-10 with corrections stored in this dtype
            gx = [self.ctx.grid(shp, G.F64, halo=2).fill(0.0) for _ in range(5)]
            gb = [self.ctx.grid(shp, G.F64, halo=0, data=x) for x in self.b]
            st = self.ctx.solve(G.K_VC13_APPLY, gx, gb, gc, kappa=kappa, rtol=1e-10, check_every=8,
                                precision=prec, inner_sweeps=16)
            rec["ir_seconds"] = round(st["seconds"], 4)
            rec["ir_outer"] = st["outer"]
            rec["ir_inner_sweeps"] = st["sweeps"]
            rec["ir_rel_residual_device"] = "%.3e" % st["rel_residual"]
            rn2 = 0.0
            for f in range(5):
                rn2 += oracle.sumsq(oracle.vc13_residual(gx[f].numpy(), self.b[f], self.c, kappa))
            rec["ir_rel_residual_oracle"] = "%.3e" % math.sqrt(rn2 / bn2)
            del gx, gb
            if dt != G.BF16:
                del gc
            torch.cuda.empty_cache()
            out[name] = rec
        self.extra = {"per_dtype": out}

    def config(self):
        return {"workload": f"13-point 4th-order operator, 5 fields + 10 coefficient grids, {self.n}^3, "
                            "BF16 storage / FP32 math (apply)", "grid": [self.n] * 3}

    def cpu_baseline(self, budget_s=10.0):
        import oracle
        import numpy as np
        x = self.fields[0].astype(np.float64)
        t0 = time.perf_counter()
        reps = 0
        while time.perf_counter() - t0 < budget_s:
            oracle.vc13_apply(x, self.c, self.W.VC13_KAPPA)
            reps += 1
        dt = time.perf_counter() - t0
        return {"value": round(self.points * reps / 5 / dt / 1e9, 4), "unit": self.unit,
                "cores": oracle.num_threads(), "kind": "oracle",
                "sample": f"{reps} single-field FP64 applies in {dt:.1f} s (scaled to 5 fields)"}


WORKLOADS = {"varcoef": VarCoef, "jacobi": Jacobi, "jacobi_tb": JacobiTB, "rbgs": RBGS, "rbgs_tb": RBGSTB,
             "tridiag": Tridiag,
             "image": Image,
             "serve": Serve, "reduce": Reduce,
             "vc13": VC13}


class KernelEvents:
    """HIP events bracketing launches of the dominant kernel, on the stream the
    library launches on (the context's stream).  A window holds one launch or
    a run of back-to-back launches of that kernel (end(n) closes a window of
    n launches); the mean per launch is the windows' total time over their
    launch count, so the event pairs (each delays the stream by a few
    microseconds) are amortized over the run and the per-launch time summed
    over a step's launches cannot exceed the step.  With `stride` > 1 only
    every stride-th window is timed."""

    def __init__(self, stream, stride=1):
        self.stream = stream
        self.stride = max(1, int(stride))
        self.pairs = []
        self._open = None
        self._count = 0

    def begin(self):
        import torch
        self._open = None
        self._count += 1
        if (self._count - 1) % self.stride:
            return
        e = torch.cuda.Event(enable_timing=True)
        e.record(self.stream)
        self._open = e

    def end(self, n=1):
        import torch
        if self._open is None:
            return
        e = torch.cuda.Event(enable_timing=True)
        e.record(self.stream)
        self.pairs.append((self._open, e, n))
        self._open = None

    def describe(self):
        sizes = sorted({k for _, _, k in self.pairs})
        what = "one launch" if sizes == [1] else f"runs of {'/'.join(map(str, sizes))} back-to-back launches"
        every = "every window" if self.stride == 1 else f"1 of every {self.stride} windows"
        return f"HIP event pairs around {what} of the kernel, {every} of the timed steps"

    def mean_ms(self):
        """(mean milliseconds per launch, launches timed)."""
        t = sum(a.elapsed_time(b) for a, b, _ in self.pairs)
        n = sum(k for _, _, k in self.pairs)
        return t / n if n else float("nan"), n


def copy_bandwidth_gbs(stream, nbytes=1 << 30, reps=10):
    """Read+write rate of a plain device-to-device copy of `nbytes` on the
    same GPU (torch's copy kernel, HIP events around each copy): the HBM rate
    a simple streaming kernel reaches on this particular device, beside the
    published peak.  Measured after the timed steps."""
    import torch
    with torch.cuda.stream(stream):
        x = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        y = torch.empty_like(x)
        for _ in range(2):
            y.copy_(x)
        ts = []
        for _ in range(reps):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(stream)
            y.copy_(x)
            b.record(stream)
            ts.append((a, b))
    sync()
    ms = sorted(a.elapsed_time(b) for a, b in ts)[reps // 2]
    del x, y
    torch.cuda.empty_cache()
    return 2 * nbytes / (ms * 1e-3) / 1e9


def serve_main(args, ctx, wl):
    def note(what, d):
        print(f"[serve] {what}: " + json.dumps({k: d[k] for k in ("solves_per_s", "p50_s", "p99_s", "converged",
                                                                 "oracle_within_rtol") if k in d}),
              file=sys.stderr, flush=True)
    seq = wl.sequential()
    note("sequential f64", seq)
    wl.step()
    bat = wl.last["batched"]
    note("batched closed loop", bat)
    loads = {}
    for factor in (0.5, 1.0, 2.0):
        loads[f"{factor:g}mu"] = wl.loaded(factor)
        note(f"batched at {factor:g} x mu", loads[f"{factor:g}mu"])
    runs = [seq, bat] + list(loads.values())
    out = {"metric": METRIC, "value": round(bat["solves_per_s"], 3), "unit": "solves/s", "n_gpus": 1,
           "steps": 1, "warmup": 0, "ms_per_step": round(bat["wall_s"] * 1e3, 2), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic (seeded)",
           "config": wl.config(),
           "sequential_f64_rate_mu": round(wl.mu, 3),
           "latency_p50_s": {k: round(v["p50_s"], 4) for k, v in loads.items()},
           "latency_p99_s": {k: round(v["p99_s"], 4) for k, v in loads.items()},
           "speedup_vs_sequential_f64": round(bat["solves_per_s"] / seq["solves_per_s"], 3),
           "answers_oracle_checked": sum(r["oracle_checked"] for r in runs),
           "answers_within_rtol": sum(r["oracle_within_rtol"] for r in runs),
           "batched_closed_loop": bat, "batched_offered": loads, "sequential_f64_closed_loop": seq,
           "roofline": None, "cpu_baseline": None}
    if wl.with_sor:
        sor_bat, sor_seq = wl.sor()
        out["batched_rbsor_f64_closed_loop"] = sor_bat
        out["sequential_rbsor_f64_closed_loop"] = sor_seq
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = wl.cpu_baseline()
    ctx.end()
    ctx.finalize()
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="varcoef", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after timing, run a 1 GiB device copy (reference for HBM byte counters)")
    ap.add_argument("--tile", default=None, help="V,NW,cz override for the dominant kernel")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the workload's extra measurements after the timed steps (for profiling runs)")
    ap.add_argument("--print-kernel-hash", action="store_true",
                    help="print the source hash of the selected workload's dominant kernel")
    ap.add_argument("--rtol", type=float, default=1e-10, help="serving: relative residual of every request")
    ap.add_argument("--requests", type=int, default=100,
                    help="serving: the first this many requests of the 2000-request stream")
    ap.add_argument("--sor", action="store_true", help="serving: also red-black SOR, batched and sequential")
    args = ap.parse_args()
    if args.print_kernel_hash:
        print(kernel_hash(WORKLOADS[args.config].key))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU (the multi-GPU path is not implemented); --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    import paper_1207_1746_amd as G
    ctx = G.Context(0)
    if args.config == "serve":
        wl = WORKLOADS[args.config](ctx, count=args.requests, rtol=args.rtol, sor=args.sor)
    else:
        wl = WORKLOADS[args.config](ctx)
    if args.tile:
        V, NW, cz = (int(v) for v in args.tile.split(","))
        kind = {"varcoef": G.K_VARCOEF7, "jacobi": G.K_WJACOBI, "image": G.K_IMG_BOX5_LAP}.get(args.config)
        if kind is not None:
            ref = {"varcoef": lambda: wl.gu, "jacobi": lambda: wl.a, "image": lambda: wl.gi}[args.config]()
            ctx.tile_set(kind, ref, (V, NW, cz))
    stream = ctx.stream
    if args.config == "serve":
        return serve_main(args, ctx, wl)

    for _ in range(args.warmup):
        wl.step()
    sync()
    ev = KernelEvents(stream, getattr(wl, "event_stride", 1))
    t0 = time.perf_counter()
    for _ in range(args.steps):
        wl.step(ev)
    sync()
    t1 = time.perf_counter()
    sec = t1 - t0
    ms_per_step = sec / args.steps * 1e3
    value = wl.units_per_step * args.steps / sec / 1e9
    kmean_ms, nk = ev.mean_ms()
    per_launch_bytes = wl.bytes_per_point * wl.points
    achieved = per_launch_bytes / (kmean_ms * 1e-3) / 1e9
    traffic = measured_traffic(wl.key)

    copy_gbs = copy_bandwidth_gbs(stream)
    if args.copy_calibration:
        x = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        y = torch.empty_like(x)
        y.copy_(x)
        sync()

    out = {
        "metric": METRIC,
        "value": round(value, 4),
        "unit": wl.unit,
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"varcoef": "f32", "jacobi": "f64", "jacobi_tb": "f64", "rbgs": "f64", "rbgs_tb": "f64",
                  "tridiag": "f64",
                  "image": "u8", "reduce": "f64",
                  "vc13": "bf16"}[args.config],
        "data": "synthetic (seeded)",
        "config": wl.config(),
        "hbm_gbs_step": round(per_launch_bytes * wl.units_per_step / wl.points * args.steps / sec / 1e9, 2),
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 2),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "kernel_ms": round(kmean_ms, 5),
            "launches_timed": nk,
            "launch_sampling": ev.describe(),
            "alg_bytes_per_launch": per_launch_bytes,
            "copy_gbs_same_gpu": round(copy_gbs, 1),
            "frac_of_copy": round(achieved / copy_gbs, 4),
        },
        "cpu_baseline": None,
    }
    if hasattr(wl, "after") and not args.no_extras:
        wl.after()
        out["extra"] = wl.extra
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = wl.cpu_baseline()
    ctx.end()
    ctx.finalize()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
