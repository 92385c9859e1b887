"""Python binding of the gfx950 stencil library (libgscl.so).

Argument marshalling only: every computation runs in the HIP kernels behind
the C-ABI declared in ``include/gscl.h``.  PyTorch supplies device memory and
the HIP stream; nothing here computes stencil values.  If the shared library
is missing the binding raises instead of falling back to anything.

Low level: ``lib()`` returns the ctypes handle with the ``gscl_*`` entry points
and their signatures.  High level: ``Context`` / ``Grid`` wrap handles and
torch tensors laid out as the library expects.
"""
from __future__ import annotations

import ctypes
import os
from typing import Iterable, Sequence

__all__ = ["lib", "Context", "Grid", "GsclError", "load_error"]

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgscl.so")

# ---- constants mirrored from include/gscl.h --------------------------------
OK, ERR_ARG, ERR_STATE, ERR_SHAPE, ERR_HALO, ERR_ALIAS, ERR_DTYPE, ERR_NOMEM, ERR_NOCONV, \
    ERR_HIP, ERR_NUMERIC, ERR_UNSUPPORTED = 0, -1, -2, -3, -4, -5, -6, -7, -8, -9, -10, -11
F64, F32, F16, BF16, U8, I16, U32 = range(7)
DIRICHLET, PERIODIC, CLAMP = 0, 1, 2
K_LINEAR, K_WJACOBI, K_VARCOEF7, K_IMG_BOX5_LAP, K_VC13_APPLY, K_VC13_JACOBI, K_VC13_RESID, \
    K_POISSON_RESID, K_WJACOBI_TB, K_RBGS, K_LINE_RECUR, K_TRIDIAG_FWD, K_TRIDIAG_BACK, \
    K_DIAMOND_RECUR, K_GS2D, K_RBGS_TB, K_VC13_JACOBI0 = range(17)
R_SUM, R_SUMSQ, R_L2, R_MAXABS, R_ALL_LE = range(5)
RV_OUT0, RV_UPDATE, RV_RESIDUAL = range(3)
PREC_F64, PREC_F32_IR, PREC_BF16_IR, PREC_F16_IR = range(4)
BATCH_JACOBI, BATCH_RBGS = range(2)
MAX_TERMS = 64

_i32, _i64, _f64, _vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p


class GridDesc(ctypes.Structure):
    _fields_ = [("ndim", _i32), ("halo", _i32), ("n", _i64 * 3), ("dtype", _i32), ("bc", _i32),
                ("bc_value", _f64), ("pitch", _i64 * 2)]


class Term(ctypes.Structure):
    _fields_ = [("out", _i32), ("grid", _i32), ("dx", _i32), ("dy", _i32), ("dz", _i32),
                ("coef", _i32), ("w", _f64)]


class StencilDesc(ctypes.Structure):
    _fields_ = [("kind", _i32), ("nterms", _i32), ("terms", ctypes.POINTER(Term)), ("p", _f64 * 8)]


class ReduceDesc(ctypes.Structure):
    _fields_ = [("op", _i32), ("operand", _i32), ("eps", _f64), ("dev_result", _vp)]


class Tile(ctypes.Structure):
    _fields_ = [("V", _i32), ("NW", _i32), ("cz", _i32)]


class SolveDesc(ctypes.Structure):
    _fields_ = [("omega", _f64), ("h2", _f64), ("kappa", _f64), ("rtol", _f64),
                ("check_every", _i32), ("precision", _i32), ("inner_sweeps", _i32), ("kind", _i32),
                ("max_sweeps", _i64)]


class SolveStats(ctypes.Structure):
    _fields_ = [("sweeps", _i64), ("outer", _i64), ("rel_residual", _f64), ("seconds", _f64)]


class BatchDesc(ctypes.Structure):
    _fields_ = [("max_slots", _i32), ("precision", _i32), ("sweeps_per_step", _i32),
                ("use_graph", _i32), ("omega", _f64), ("rtol", _f64), ("hbm_budget", ctypes.c_size_t),
                ("max_sweeps", _i64), ("method", _i32), ("sweeps_per_pass", _i32)]


class SlotStats(ctypes.Structure):
    _fields_ = [("state", _i32), ("reserved", _i32), ("sweeps", _i64), ("rel_residual", _f64)]


_P = ctypes.POINTER
_SIGS = {
    "gscl_init": (ctypes.c_int, [ctypes.c_int, _P(_vp)]),
    "gscl_begin": (ctypes.c_int, [_vp, _vp]),
    "gscl_end": (ctypes.c_int, [_vp]),
    "gscl_finalize": (ctypes.c_int, [_vp]),
    "gscl_reserve": (ctypes.c_int, [_vp, _i64]),
    "gscl_grid_bytes": (ctypes.c_size_t, [_P(GridDesc)]),
    "gscl_grid_layout": (ctypes.c_int, [_P(GridDesc)]),
    "gscl_grid_create": (ctypes.c_int, [_vp, _P(GridDesc), _vp, _P(_vp)]),
    "gscl_grid_destroy": (ctypes.c_int, [_vp]),
    "gscl_do_all": (ctypes.c_int, [_vp, _P(StencilDesc), _P(_vp), ctypes.c_int, _P(_vp), ctypes.c_int,
                                   _P(ReduceDesc), _P(_f64)]),
    "gscl_do_all_noalloc": (ctypes.c_int, [_vp, _P(StencilDesc), _P(_vp), ctypes.c_int, _P(_vp), ctypes.c_int,
                                           _P(ReduceDesc), _P(_f64)]),
    "gscl_do_line": (ctypes.c_int, [_vp, _P(StencilDesc), ctypes.c_int, ctypes.c_int, _P(_vp), ctypes.c_int,
                                    _P(_vp), ctypes.c_int]),
    "gscl_do_diamond": (ctypes.c_int, [_vp, _P(StencilDesc), _P(_vp), ctypes.c_int, _P(_vp), ctypes.c_int]),
    "gscl_do_reduce": (ctypes.c_int, [_vp, _P(ReduceDesc), _vp, _vp, _P(_f64)]),
    "gscl_tile_get": (ctypes.c_int, [_vp, ctypes.c_int, _P(GridDesc), _P(Tile)]),
    "gscl_tile_set": (ctypes.c_int, [_vp, ctypes.c_int, _P(GridDesc), _P(Tile)]),
    "gscl_tile_clear": (ctypes.c_int, [_vp]),
    "gscl_graph_begin": (ctypes.c_int, [_vp]),
    "gscl_graph_end": (ctypes.c_int, [_vp, _P(_vp)]),
    "gscl_graph_launch": (ctypes.c_int, [_vp, _vp]),
    "gscl_graph_destroy": (ctypes.c_int, [_vp]),
    "gscl_solve_workspace_bytes": (ctypes.c_size_t, [_P(SolveDesc), _vp, ctypes.c_int]),
    "gscl_solve": (ctypes.c_int, [_vp, _P(SolveDesc), _P(_vp), _P(_vp), ctypes.c_int, _P(_vp), ctypes.c_int,
                                  _vp, ctypes.c_size_t, _P(SolveStats)]),
    "gscl_batch_create": (ctypes.c_int, [_vp, _P(BatchDesc), _P(_vp)]),
    "gscl_batch_footprint": (ctypes.c_size_t, [_vp, _P(_i64)]),
    "gscl_batch_tile_rule": (ctypes.c_int, [_vp, ctypes.c_int, _P(ctypes.c_int32), _P(ctypes.c_int32),
                                            _P(ctypes.c_int32)]),
    "gscl_batch_admit": (ctypes.c_int, [_vp, _vp, _vp, _f64, _P(ctypes.c_int)]),
    "gscl_batch_step": (ctypes.c_int, [_vp]),
    "gscl_batch_poll": (ctypes.c_int, [_vp, _P(ctypes.c_int), ctypes.c_int, _P(ctypes.c_int)]),
    "gscl_batch_poll_lagged": (ctypes.c_int, [_vp, _P(ctypes.c_int), ctypes.c_int, _P(ctypes.c_int)]),
    "gscl_batch_retire": (ctypes.c_int, [_vp, ctypes.c_int, _P(SlotStats)]),
    "gscl_batch_destroy": (ctypes.c_int, [_vp]),
    "gscl_last_error": (ctypes.c_char_p, []),
    "gscl_version": (ctypes.c_char_p, []),
}

_lib = None


def load_error() -> str | None:
    """Why the library cannot be loaded (None if it can)."""
    try:
        lib()
        return None
    except Exception as e:  # pragma: no cover - reported to the caller
        return str(e)


def lib():
    """The loaded libgscl.so with typed entry points (raises if it is missing)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library {LIB_PATH} is missing: run paper_1207_1746_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


class GsclError(RuntimeError):
    def __init__(self, code: int, where: str):
        msg = lib().gscl_last_error().decode(errors="replace")
        super().__init__(f"{where}: status {code}: {msg}")
        self.code = code


def check(code: int, where: str) -> int:
    if code != OK:
        raise GsclError(code, where)
    return code


def _torch():
    import torch
    return torch


def torch_dtype(dt: int):
    torch = _torch()
    return {F64: torch.float64, F32: torch.float32, F16: torch.float16, BF16: torch.bfloat16,
            U8: torch.uint8, I16: torch.int16, U32: torch.uint32}[dt]


def gscl_dtype(tdtype) -> int:
    torch = _torch()
    m = {torch.float64: F64, torch.float32: F32, torch.float16: F16, torch.bfloat16: BF16,
         torch.uint8: U8, torch.int16: I16, torch.uint32: U32}
    return m[tdtype]


def make_desc(shape: Sequence[int], dtype: int, halo: int = 1, bc: int = DIRICHLET,
              bc_value: float = 0.0, ndim: int | None = None, pitch=(0, 0)) -> GridDesc:
    """shape is (nz, ny, nx) for 3D or (ny, nx) / (layers, ny, nx) for 2D."""
    d = GridDesc()
    if ndim is None:
        ndim = len(shape)
    d.ndim = ndim
    d.halo = halo
    if len(shape) == 3:
        d.n[0], d.n[1], d.n[2] = shape[2], shape[1], shape[0]
    else:
        d.n[0], d.n[1], d.n[2] = shape[1], shape[0], 1
    d.dtype = dtype
    d.bc = bc
    d.bc_value = bc_value
    d.pitch[0], d.pitch[1] = pitch
    return d


class Grid:
    """A library grid over a torch tensor it owns (or borrows).

    ``storage`` is the flat allocation, ``view`` the (nz, ny, nx) interior."""

    def __init__(self, ctx: "Context", desc: GridDesc, storage=None):
        torch = _torch()
        self.ctx = ctx
        check(lib().gscl_grid_layout(ctypes.byref(desc)), "gscl_grid_layout")
        self.desc = desc
        nbytes = lib().gscl_grid_bytes(ctypes.byref(desc))
        if nbytes == 0:
            raise GsclError(ERR_ARG, "gscl_grid_bytes")
        tdt = torch_dtype(desc.dtype)
        esz = torch.empty((), dtype=tdt).element_size()
        nel = (nbytes + esz - 1) // esz
        if storage is None:
            storage = torch.empty(nel, dtype=tdt, device=ctx.device)
        self.storage = storage
        nx, ny, nz = desc.n[0], desc.n[1], desc.n[2]
        self.view = storage.as_strided((nz, ny, nx), (desc.pitch[1], desc.pitch[0], 1))
        h = _vp()
        check(lib().gscl_grid_create(ctx.handle, ctypes.byref(desc), _vp(storage.data_ptr()),
                                     ctypes.byref(h)), "gscl_grid_create")
        self.handle = h

    @property
    def shape(self):
        return tuple(self.view.shape)

    def upload(self, array) -> "Grid":
        torch = _torch()
        t = torch.as_tensor(array)
        if t.dim() == 2:
            t = t.unsqueeze(0)
        self.view.copy_(t.to(self.view.dtype).reshape(self.view.shape))
        return self

    def fill(self, value) -> "Grid":
        self.view.fill_(value)
        return self

    def numpy(self):
        return self.view.detach().cpu().contiguous().numpy() if self.view.dtype != _torch().bfloat16 \
            else self.view.detach().float().cpu().contiguous().numpy()

    def close(self):
        if self.handle:
            lib().gscl_grid_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _handles(grids: Iterable[Grid]):
    gs = list(grids)
    arr = (_vp * max(len(gs), 1))(*[g.handle for g in gs])
    return arr, len(gs)


class Context:
    """gscl_init + gscl_begin on a torch stream (Section 4 context phases)."""

    def __init__(self, device: int = 0, stream=None, begin: bool = True):
        torch = _torch()
        self.device = torch.device("cuda", device)
        self.index = device
        h = _vp()
        check(lib().gscl_init(device, ctypes.byref(h)), "gscl_init")
        self.handle = h
        self.stream = stream
        if begin:
            self.begin(stream)

    def begin(self, stream=None):
        torch = _torch()
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        check(lib().gscl_begin(self.handle, _vp(stream.cuda_stream)), "gscl_begin")

    def end(self):
        check(lib().gscl_end(self.handle), "gscl_end")

    def finalize(self):
        if self.handle:
            check(lib().gscl_finalize(self.handle), "gscl_finalize")
            self.handle = None

    def reserve(self, max_points: int):
        check(lib().gscl_reserve(self.handle, int(max_points)), "gscl_reserve")

    # grids ------------------------------------------------------------------
    def grid(self, shape, dtype: int, halo: int = 1, bc: int = DIRICHLET, bc_value: float = 0.0,
             ndim: int | None = None, data=None, pitch=(0, 0)) -> Grid:
        g = Grid(self, make_desc(shape, dtype, halo, bc, bc_value, ndim, pitch))
        if data is not None:
            g.upload(data)
        return g

    # iteration spaces ---------------------------------------------------------
    def do_all(self, kind: int, ins: Sequence[Grid], outs: Sequence[Grid], p: Sequence[float] = (),
               terms: Sequence[tuple] | None = None, reduce: tuple | None = None,
               dev_result=None, noalloc: bool = False) -> float | None:
        """reduce = (op, operand[, eps]); returns the host result unless dev_result
        (a device double tensor element) is given.  noalloc=True issues
        gscl_do_all_noalloc (fused-reduction scratch in the library's fixed
        device array)."""
        sd = StencilDesc()
        sd.kind = kind
        for i, v in enumerate(p):
            sd.p[i] = float(v)
        keep = None
        if terms is not None:
            arr = (Term * len(terms))()
            for i, t in enumerate(terms):
                o, g, dx, dy, dz, w, coef = t
                arr[i].out, arr[i].grid, arr[i].dx, arr[i].dy, arr[i].dz = o, g, dx, dy, dz
                arr[i].w, arr[i].coef = float(w), coef
            sd.terms = ctypes.cast(arr, ctypes.POINTER(Term))
            sd.nterms = len(terms)
            keep = arr
        hi, ni = _handles(ins)
        ho, no = _handles(outs)
        rd_p = None
        res = _f64(0.0)
        if reduce is not None:
            rd = ReduceDesc()
            rd.op, rd.operand = reduce[0], reduce[1]
            rd.eps = reduce[2] if len(reduce) > 2 else 0.0
            rd.dev_result = dev_result.data_ptr() if dev_result is not None else None
            rd_p = ctypes.byref(rd)
        fn = lib().gscl_do_all_noalloc if noalloc else lib().gscl_do_all
        rc = fn(self.handle, ctypes.byref(sd), hi, ni, ho, no, rd_p,
                ctypes.byref(res) if reduce is not None else None)
        del keep
        check(rc, "gscl_do_all_noalloc" if noalloc else "gscl_do_all")
        if reduce is not None and dev_result is None:
            return res.value
        return None

    def prepare_all(self, kind: int, ins: Sequence[Grid], outs: Sequence[Grid], p: Sequence[float] = (),
                    reduce: tuple | None = None, dev_result=None) -> "PreparedAll":
        """The same call as do_all, with its descriptors built once: calling the
        returned object issues gscl_do_all again with unchanged arguments (for
        loops of short launches, where building them costs as much as the
        launch)."""
        return PreparedAll(self, kind, ins, outs, p, reduce, dev_result)

    def do_line(self, kind: int, axis: int, direction: int, ins: Sequence[Grid], outs: Sequence[Grid],
                p: Sequence[float] = ()):
        """Ordered line iteration space (do_i/j/k_inc for direction +1, _dec
        for -1 along axis 0/1/2)."""
        sd = StencilDesc()
        sd.kind = kind
        for i, v in enumerate(p):
            sd.p[i] = float(v)
        hi, ni = _handles(ins)
        ho, no = _handles(outs)
        check(lib().gscl_do_line(self.handle, ctypes.byref(sd), int(axis), int(direction), hi, ni, ho, no),
              "gscl_do_line")

    def do_diamond(self, kind: int, ins: Sequence[Grid], outs: Sequence[Grid], p: Sequence[float] = ()):
        """The diamond iteration space (2D): (i-1, j) and (i, j-1) before (i, j)."""
        sd = StencilDesc()
        sd.kind = kind
        for i, v in enumerate(p):
            sd.p[i] = float(v)
        hi, ni = _handles(ins)
        ho, no = _handles(outs)
        check(lib().gscl_do_diamond(self.handle, ctypes.byref(sd), hi, ni, ho, no), "gscl_do_diamond")

    def do_reduce(self, op: int, a: Grid, b: Grid | None = None, eps: float = 0.0,
                  dev_result=None) -> float | None:
        rd = ReduceDesc()
        rd.op = op
        rd.eps = eps
        rd.dev_result = dev_result.data_ptr() if dev_result is not None else None
        res = _f64(0.0)
        check(lib().gscl_do_reduce(self.handle, ctypes.byref(rd), a.handle, b.handle if b else None,
                                   ctypes.byref(res)), "gscl_do_reduce")
        return res.value if dev_result is None else None

    # solver ---------------------------------------------------------------------
    def solve(self, kind: int, x: Sequence[Grid], b: Sequence[Grid], coef: Sequence[Grid] = (),
              omega: float = 6 / 7, h2: float = 1.0, kappa: float = 0.25, rtol: float = 1e-8,
              check_every: int = 32, precision: int = PREC_F64, inner_sweeps: int = 64,
              max_sweeps: int = 10 ** 7) -> dict:
        """gscl_solve; returns {'sweeps', 'outer', 'rel_residual', 'seconds'}."""
        torch = _torch()
        sd = SolveDesc(omega, h2, kappa, rtol, check_every, precision, inner_sweeps, kind, max_sweeps)
        hx, nx_ = _handles(x)
        hb, _ = _handles(b)
        hc, nc = _handles(coef) if coef else (None, 0)
        nbytes = lib().gscl_solve_workspace_bytes(ctypes.byref(sd), x[0].handle, nx_)
        ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=self.device)
        st = SolveStats()
        check(lib().gscl_solve(self.handle, ctypes.byref(sd), hx, hb, nx_, hc, nc, _vp(ws.data_ptr()),
                               nbytes, ctypes.byref(st)), "gscl_solve")
        return {"sweeps": st.sweeps, "outer": st.outer, "rel_residual": st.rel_residual,
                "seconds": st.seconds}

    def batch(self, **kw) -> "Batch":
        return Batch(self, **kw)

    # tiles and graphs -------------------------------------------------------------
    def tile_get(self, kind: int, g: Grid) -> tuple:
        t = Tile()
        check(lib().gscl_tile_get(self.handle, kind, ctypes.byref(g.desc), ctypes.byref(t)), "gscl_tile_get")
        return (t.V, t.NW, t.cz)

    def tile_set(self, kind: int, g: Grid, tile: tuple):
        t = Tile(*tile)
        check(lib().gscl_tile_set(self.handle, kind, ctypes.byref(g.desc), ctypes.byref(t)), "gscl_tile_set")

    def tile_clear(self):
        check(lib().gscl_tile_clear(self.handle), "gscl_tile_clear")

    def graph_begin(self):
        check(lib().gscl_graph_begin(self.handle), "gscl_graph_begin")

    def graph_end(self) -> "Graph":
        h = _vp()
        check(lib().gscl_graph_end(self.handle, ctypes.byref(h)), "gscl_graph_end")
        return Graph(self, h)


class Graph:
    def __init__(self, ctx: Context, handle):
        self.ctx = ctx
        self.handle = handle

    def launch(self):
        check(lib().gscl_graph_launch(self.ctx.handle, self.handle), "gscl_graph_launch")

    def close(self):
        if self.handle:
            lib().gscl_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class PreparedAll:
    """A gscl_do_all call with prebuilt arguments (Context.prepare_all)."""

    def __init__(self, ctx: Context, kind, ins, outs, p, reduce, dev_result):
        self.sd = StencilDesc()
        self.sd.kind = kind
        for i, v in enumerate(p):
            self.sd.p[i] = float(v)
        self.grids = list(ins) + list(outs)  # keep the grids alive
        self.hi, self.ni = _handles(ins)
        self.ho, self.no = _handles(outs)
        self.res = _f64(0.0)
        self.host_result = reduce is not None and dev_result is None
        self.rd = None
        if reduce is not None:
            self.rd = ReduceDesc()
            self.rd.op, self.rd.operand = reduce[0], reduce[1]
            self.rd.eps = reduce[2] if len(reduce) > 2 else 0.0
            self.rd.dev_result = dev_result.data_ptr() if dev_result is not None else None
        self.args = (ctx.handle, ctypes.byref(self.sd), self.hi, self.ni, self.ho, self.no,
                     ctypes.byref(self.rd) if self.rd is not None else None,
                     ctypes.byref(self.res) if self.rd is not None else None)
        self.fn = lib().gscl_do_all

    def __call__(self) -> float | None:
        rc = self.fn(*self.args)
        if rc != OK:
            raise GsclError(rc, "gscl_do_all")
        return self.res.value if self.host_result else None


class Batch:
    """Batched multi-grid Poisson executor (gscl_batch_*).  method BATCH_JACOBI
    sweeps weighted Jacobi (F64 or F32 refinement); BATCH_RBGS sweeps red-black
    SOR in F64 (omega = 0: each slot's optimal model-problem weight).  Either
    may run temporally blocked passes of sweeps_per_pass sweeps (Jacobi) or
    colour passes (red-black, an even number)."""

    def __init__(self, ctx: Context, max_slots: int = 64, precision: int = PREC_F64,
                 sweeps_per_step: int = 32, use_graph: bool = True, omega: float = 6 / 7,
                 rtol: float = 1e-8, hbm_budget: int = 8 << 30, max_sweeps: int = 10 ** 7,
                 method: int = BATCH_JACOBI, sweeps_per_pass: int = 1):
        self.ctx = ctx
        bd = BatchDesc(max_slots, precision, sweeps_per_step, int(use_graph), omega, rtol, hbm_budget,
                       max_sweeps, method, sweeps_per_pass)
        h = _vp()
        check(lib().gscl_batch_create(ctx.handle, ctypes.byref(bd), ctypes.byref(h)), "gscl_batch_create")
        self.handle = h
        self.max_slots = max_slots
        self.sweeps_per_step = sweeps_per_step
        self.tile_rule = []

    def footprint(self, shape) -> int:
        n = (_i64 * 3)(shape[2], shape[1], shape[0])
        return int(lib().gscl_batch_footprint(self.handle, n))

    def set_tile_rule(self, rules: Sequence[tuple]):
        """rules = [(edge, cz, tb_cz), ...] with increasing edges (see
        gscl_batch_tile_rule); applies to requests admitted afterwards."""
        n = len(rules)
        arr = [(ctypes.c_int32 * max(n, 1))(*[int(r[k]) for r in rules]) for k in range(3)]
        check(lib().gscl_batch_tile_rule(self.handle, n, arr[0], arr[1], arr[2]), "gscl_batch_tile_rule")
        self.tile_rule = [tuple(int(v) for v in r) for r in rules]

    def admit(self, u: Grid, f: Grid, h2: float) -> int | None:
        """Slot id, or None when no slot / budget is free (the caller queues)."""
        slot = ctypes.c_int(-1)
        rc = lib().gscl_batch_admit(self.handle, u.handle, f.handle, float(h2), ctypes.byref(slot))
        if rc == ERR_NOMEM:
            return None
        check(rc, "gscl_batch_admit")
        return slot.value

    def step(self):
        check(lib().gscl_batch_step(self.handle), "gscl_batch_step")

    def poll(self, lagged: bool = False) -> list[int]:
        """Finished slots.  lagged=True waits only for the step before the
        latest one (the device keeps working meanwhile)."""
        arr = (ctypes.c_int * self.max_slots)()
        n = ctypes.c_int(0)
        fn = lib().gscl_batch_poll_lagged if lagged else lib().gscl_batch_poll
        check(fn(self.handle, arr, self.max_slots, ctypes.byref(n)), "gscl_batch_poll")
        return [arr[i] for i in range(min(n.value, self.max_slots))]

    def retire(self, slot: int) -> dict:
        st = SlotStats()
        check(lib().gscl_batch_retire(self.handle, slot, ctypes.byref(st)), "gscl_batch_retire")
        return {"state": st.state, "sweeps": st.sweeps, "rel_residual": st.rel_residual}

    def close(self):
        if self.handle:
            lib().gscl_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
