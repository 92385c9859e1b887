"""FP64 CPU oracle for the GSCL stencil hot path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product library never does, and the
two share no code: this module drives ``liboracle.so`` (plain C, ``oracle.c``)
and composes its per-sweep functions into the iterations the paper describes.

Functions follow the paper (A Generic Library for Stencil Computations,
Bianco & Varetto):
  * ``linear``          -- do_all with a linear stencil operator (Section 3, Fig. 1b)
  * ``wjacobi_sweep``   -- the averaging (Jacobi) iteration of Section 5.2
  * ``jacobi_run``      -- that iteration with the update norm checked (Section 5.2)
  * ``poisson_solve``   -- weighted Jacobi to a relative residual, with the check
                           fused into the last sweep of each chunk (Section 5.2 fuse)
  * ``varcoef7_*``      -- multi-grid variable-coefficient sweep (Section 2, 5-15 grids)
  * ``img``             -- integer image filters (Section 1)
  * ``vc13_*``          -- fourth-order 13-point multi-field operator and its FP64
                           weighted-Jacobi solve (Section 2)
  * ``rbgs_*``          -- red-black Gauss-Seidel / SOR passes, sweeps and solve on
                           the Poisson problem (Section 3 stateful stencils)
  * ``line_recur``, ``tridiag_*`` -- ordered line iteration spaces (Section 3
                           do_i/j/k_inc, do_i/j/k_dec): a first-order recurrence
                           and the two passes of the Thomas algorithm
  * ``diamond_recur``, ``gs2d_sweep`` -- the diamond iteration space (Section 3
                           do_diamond, 2D): a two-predecessor recurrence and a
                           lexicographic Gauss-Seidel / SOR sweep
  * ``sum/sumsq/maxabs``-- do_reduce with commutative operators (Section 3)

Parity status: every function is pinned by tests under ``tests/test_oracle_*``
(closed forms, invariants, textbook special cases, brute force on tiny grids).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")

DIRICHLET, PERIODIC, CLAMP = 0, 1, 2

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)
_u8p = ctypes.POINTER(ctypes.c_uint8)
_i16p = ctypes.POINTER(ctypes.c_int16)
_L = ctypes.c_long


def build(force: bool = False) -> str:
    """Compile oracle.c with gcc (no fused multiply-add, OpenMP over the outer loop)."""
    src = os.path.join(_HERE, "oracle.c")
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(src):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC",
                               "-shared", "-o", tmp, src, "-lm"])
        os.replace(tmp, _SO)
    return _SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_SO)
        L.oracle_linear.argtypes = [ctypes.c_int, _L, _L, _L, ctypes.c_int, _dp, _ip, _dp,
                                    ctypes.c_int, _ip, _ip, _ip, _ip, _dp, _ip, _ip,
                                    ctypes.c_int, _dp]
        L.oracle_wjacobi.argtypes = [ctypes.c_int, _L, _L, _L, _dp, _dp, ctypes.c_double,
                                     ctypes.c_double, ctypes.c_int, ctypes.c_double, _dp, _dp, _dp]
        L.oracle_varcoef7.argtypes = [_L, _L, _L, _dp, _dp, _dp, ctypes.c_int, ctypes.c_double,
                                      _dp, _dp, _dp]
        L.oracle_img.argtypes = [_L, _L, _L, _u8p, ctypes.c_int, _u8p, _i16p]
        L.oracle_vc13_apply.argtypes = [_L, _L, _L, _dp, _dp, ctypes.c_double, ctypes.c_double, _dp]
        L.oracle_rbgs_pass.argtypes = [_L, _L, _L, _dp, _dp, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_double, ctypes.c_int, _dp, _dp]
        L.oracle_line_recur.argtypes = [_L, _L, _L, ctypes.c_int, ctypes.c_int, _dp, _dp,
                                        ctypes.c_double, _dp]
        L.oracle_tridiag_fwd.argtypes = [_L, _L, _L, ctypes.c_int, ctypes.c_int, _dp, _dp, _dp, _dp,
                                         _dp, _dp]
        L.oracle_tridiag_back.argtypes = [_L, _L, _L, ctypes.c_int, ctypes.c_int, _dp, _dp, _dp]
        L.oracle_diamond_recur.argtypes = [_L, _L, _L, _dp, _dp, _dp, ctypes.c_double, _dp]
        L.oracle_gs2d.argtypes = [_L, _L, _L, _dp, _dp, ctypes.c_double, ctypes.c_double, ctypes.c_double]
        L.oracle_vc13_diag.argtypes = [_L, _L, _L, _dp, ctypes.c_double, _dp]
        for f in ("oracle_sum", "oracle_sumsq", "oracle_maxabs"):
            getattr(L, f).argtypes = [_dp, _L]
            getattr(L, f).restype = ctypes.c_double
        L.oracle_num_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def num_threads() -> int:
    return int(lib().oracle_num_threads())


def _f64(a) -> np.ndarray:
    """Exact upcast of a stored grid (any float dtype) to a contiguous FP64 array."""
    a = np.asarray(a)
    if a.dtype != np.float64:
        a = a.astype(np.float64)
    return np.ascontiguousarray(a)


def _ptr(a: np.ndarray, t=_dp):
    return a.ctypes.data_as(t)


def _shape3(a: np.ndarray, ndim: int):
    if ndim == 3:
        nz, ny, nx = a.shape
    elif a.ndim == 2:
        nz, (ny, nx) = 1, a.shape
    else:
        nz, ny, nx = a.shape
    return nx, ny, nz


# --------------------------------------------------------------------------- #
# do_all: generic linear operator (Section 3)
# --------------------------------------------------------------------------- #
def linear(ndim: int, ins: Sequence[np.ndarray], terms: Sequence[tuple], nout: int,
           bc: Sequence[int], bcv: Sequence[float]) -> list[np.ndarray]:
    """terms: (out, grid, dx, dy, dz, w, coef) tuples, coef = -1 for none.

    out[o](p) = sum_t w * coef(p) * in[grid](p + d), in list order (FP64)."""
    ins = [_f64(a) for a in ins]
    shape = ins[0].shape
    nx, ny, nz = _shape3(ins[0], ndim)
    packed = np.ascontiguousarray(np.stack(ins))
    out = np.zeros((nout,) + shape, dtype=np.float64)
    ti = lambda col: np.ascontiguousarray(np.array([t[col] for t in terms], dtype=np.int32))
    tg, tdx, tdy, tdz, tcoef, tout = ti(1), ti(2), ti(3), ti(4), ti(6), ti(0)
    tw = np.ascontiguousarray(np.array([t[5] for t in terms], dtype=np.float64))
    bca = np.ascontiguousarray(np.array(bc, dtype=np.int32))
    bcva = np.ascontiguousarray(np.array(bcv, dtype=np.float64))
    lib().oracle_linear(ndim, nx, ny, nz, len(ins), _ptr(packed), _ptr(bca, _ip), _ptr(bcva),
                        len(terms), _ptr(tg, _ip), _ptr(tdx, _ip), _ptr(tdy, _ip), _ptr(tdz, _ip),
                        _ptr(tw), _ptr(tcoef, _ip), _ptr(tout, _ip), nout, _ptr(out))
    return [out[o] for o in range(nout)]


# --------------------------------------------------------------------------- #
# Jacobi averaging iteration (Section 5.2)
# --------------------------------------------------------------------------- #
def wjacobi_sweep(u, f=None, omega=1.0, h2=1.0, bc=DIRICHLET, bcv=0.0, ndim=3):
    """One sweep; returns (unew, update unew-u, residual f - Lap_h u of the input)."""
    u = _f64(u)
    nx, ny, nz = _shape3(u, ndim)
    fa = _f64(f) if f is not None else None
    unew, upd, res = np.empty_like(u), np.empty_like(u), np.empty_like(u)
    lib().oracle_wjacobi(ndim, nx, ny, nz, _ptr(u), _ptr(fa) if fa is not None else None,
                         float(omega), float(h2), int(bc), float(bcv), _ptr(unew), _ptr(upd),
                         _ptr(res))
    return unew, upd, res


def rbgs_pass(u, f=None, omega=1.0, h2=1.0, colour=0, bcv=0.0):
    """One colour pass of red-black relaxation on Lap_h u = f (Dirichlet bcv);
    returns (u after the pass, update at the pass's points, residual before
    the update at the pass's points)."""
    u = _f64(u).copy()
    nz, ny, nx = u.shape
    fa = _f64(f) if f is not None else None
    upd, res = np.empty_like(u), np.empty_like(u)
    lib().oracle_rbgs_pass(nx, ny, nz, _ptr(u), _ptr(fa) if fa is not None else None, float(omega),
                           float(h2), float(bcv), int(colour), _ptr(upd), _ptr(res))
    return u, upd, res


def rbgs_sweep(u, f=None, omega=1.0, h2=1.0, bcv=0.0):
    """One red-black Gauss-Seidel (omega = 1) or SOR sweep: the red points
    ((i+j+k) even), then the black points with the new red values."""
    u, _, _ = rbgs_pass(u, f, omega, h2, 0, bcv)
    u, _, _ = rbgs_pass(u, f, omega, h2, 1, bcv)
    return u


def rbgs_solve(f, h2: float, omega: float, rtol: float, check_every: int, max_sweeps: int):
    """Red-black relaxation on Lap_h u = f (Dirichlet 0) from u = 0, checked
    after every chunk of ``check_every`` sweeps: stops when the residual of
    the current u satisfies ||f - Lap_h u||_2 <= rtol ||f||_2.
    Returns (u, sweeps, rel_residual, converged)."""
    f = _f64(f)
    u = np.zeros_like(f)
    fn = np.sqrt(sumsq(f))
    sweeps = 0
    rel = float("inf")
    while sweeps < max_sweeps:
        for _ in range(check_every):
            u = rbgs_sweep(u, f, omega, h2)
        sweeps += check_every
        _, _, res = wjacobi_sweep(u, f, 1.0, h2)
        rel = float(np.sqrt(sumsq(res)) / fn)
        if rel <= rtol:
            return u, sweeps, rel, True
    return u, sweeps, rel, False


def _line_dims(a):
    a = _f64(a)
    if a.ndim == 2:
        a = a[None]
    nz, ny, nx = a.shape
    return a, nx, ny, nz


def line_recur(a, b, axis: int, direction: int, seed: float = 0.0):
    """Ordered line iteration space (do_i/j/k_inc for direction +1, _dec for
    -1 along axis 0/1/2 = i/j/k) applying out(c) = a(c) * prev + b(c)."""
    a, nx, ny, nz = _line_dims(a)
    b = _line_dims(b)[0]
    out = np.empty_like(a)
    lib().oracle_line_recur(nx, ny, nz, int(axis), int(direction), _ptr(a), _ptr(b), float(seed),
                            _ptr(out))
    return out


def tridiag_fwd(lo, di, up, rhs, axis: int, direction: int):
    """Thomas forward elimination along the lines; returns (cp, dp)."""
    lo, nx, ny, nz = _line_dims(lo)
    di, up, rhs = (_line_dims(x)[0] for x in (di, up, rhs))
    cp, dp = np.empty_like(lo), np.empty_like(lo)
    lib().oracle_tridiag_fwd(nx, ny, nz, int(axis), int(direction), _ptr(lo), _ptr(di), _ptr(up),
                             _ptr(rhs), _ptr(cp), _ptr(dp))
    return cp, dp


def tridiag_back(cp, dp, axis: int, direction: int):
    """Thomas back substitution along the lines (direction opposite to the
    elimination); returns x."""
    cp, nx, ny, nz = _line_dims(cp)
    dp = _line_dims(dp)[0]
    x = np.empty_like(cp)
    lib().oracle_tridiag_back(nx, ny, nz, int(axis), int(direction), _ptr(cp), _ptr(dp), _ptr(x))
    return x


def tridiag_solve(lo, di, up, rhs, axis: int, direction: int = 1):
    """Solve the tridiagonal system of every line: elimination along
    `direction`, substitution back against it."""
    cp, dp = tridiag_fwd(lo, di, up, rhs, axis, direction)
    return tridiag_back(cp, dp, axis, -direction)


def diamond_recur(a, b, c, seed: float = 0.0):
    """Diamond iteration space (cells (i-1, j), (i, j-1) before (i, j); 2D
    layers) applying out = a * out(i-1, j) + b * out(i, j-1) + c."""
    a, nx, ny, nl = _line_dims(a)
    b, c = _line_dims(b)[0], _line_dims(c)[0]
    out = np.empty_like(a)
    lib().oracle_diamond_recur(nx, ny, nl, _ptr(a), _ptr(b), _ptr(c), float(seed), _ptr(out))
    return out


def gs2d_sweep(u, f=None, omega=1.0, h2=1.0, bcv=0.0):
    """One lexicographic Gauss-Seidel / SOR sweep on the 2D 5-point Poisson
    problem (a diamond-ordered operator); returns the new grid."""
    u, nx, ny, nl = _line_dims(u)
    u = u.copy()
    fa = _line_dims(f)[0] if f is not None else None
    lib().oracle_gs2d(nx, ny, nl, _ptr(u), _ptr(fa) if fa is not None else None, float(omega), float(h2),
                      float(bcv))
    return u


def jacobi_run(u0, nsweeps: int, f=None, omega=1.0, h2=1.0, bc=DIRICHLET, bcv=0.0, ndim=3):
    """nsweeps sweeps from u0; returns (u_n, ||u_n - u_{n-1}||_2, max|u_n - u_{n-1}|).

    The last two are the paper's convergence check on the update (Section 5.2),
    taken here as the L2 and the infinity norm of the final update."""
    u = _f64(u0)
    upd = np.zeros_like(u)
    for _ in range(nsweeps):
        u, upd, _ = wjacobi_sweep(u, f, omega, h2, bc, bcv, ndim)
    return u, float(np.sqrt(sumsq(upd))), maxabs(upd)


def poisson_solve(f, h2: float, omega: float, rtol: float, check_every: int,
                  max_sweeps: int, u0=None):
    """Weighted Jacobi on Lap_h u = f (Dirichlet 0) until the relative residual
    meets rtol.

    The convergence test is fused into the last sweep of every chunk of
    ``check_every`` sweeps (Section 5.2 fuse): that sweep produces u_n from
    u_{n-1} and the residual of u_{n-1}; when ||r(u_{n-1})||_2 <= rtol ||f||_2
    the solve returns u_n, the grid the sweep just wrote.

    Returns (u, sweeps, rel_residual_checked, converged)."""
    f = _f64(f)
    u = np.zeros_like(f) if u0 is None else _f64(u0)
    fn = np.sqrt(sumsq(f))
    n = 0
    while n < max_sweeps:
        last = (n + 1) % check_every == 0
        unew, _, res = wjacobi_sweep(u, f, omega, h2, DIRICHLET, 0.0, 3)
        n += 1
        u = unew
        if last:
            rel = np.sqrt(sumsq(res)) / fn if fn > 0 else 0.0
            if rel <= rtol:
                return u, n, float(rel), True
    return u, n, float("nan"), False


# --------------------------------------------------------------------------- #
# Multi-grid variable-coefficient sweep (9 inputs, 3 outputs)
# --------------------------------------------------------------------------- #
def _pack(c) -> np.ndarray:
    if isinstance(c, np.ndarray) and c.dtype == np.float64 and c.ndim == 4 and c.flags.c_contiguous:
        return c
    return np.ascontiguousarray(np.stack([_f64(x) for x in c]))


def varcoef7_sweep(u, c, s, bc=PERIODIC, bcv=0.0):
    """c: the 7 coefficient grids (a list, or one packed (7, nz, ny, nx) FP64 array)."""
    u = _f64(u)
    nz, ny, nx = u.shape
    cp = _pack(c)
    sa = _f64(s)
    unew, r, fm = np.empty_like(u), np.empty_like(u), np.empty_like(u)
    lib().oracle_varcoef7(nx, ny, nz, _ptr(u), _ptr(cp), _ptr(sa), int(bc), float(bcv),
                          _ptr(unew), _ptr(r), _ptr(fm))
    return unew, r, fm


def varcoef7_run(u0, c, s, nsweeps: int, check_every: int, bc=PERIODIC):
    """nsweeps sweeps; the L2 norm of the residual grid written by sweeps
    check_every, 2*check_every, ... is recorded.  Returns (u, r, fmag, norms)."""
    u = _f64(u0)
    cp = _pack(c)
    sa = _f64(s)
    norms = []
    r = fm = None
    for n in range(1, nsweeps + 1):
        u, r, fm = varcoef7_sweep(u, cp, sa, bc)
        if n % check_every == 0:
            norms.append(float(np.sqrt(sumsq(r))))
    return u, r, fm, norms


# --------------------------------------------------------------------------- #
# Integer image filters
# --------------------------------------------------------------------------- #
def img(planes, lap_kind: int = 4):
    """planes: uint8 (nlayers, ny, nx) or (ny, nx).  Returns (box uint8, lap int16)."""
    a = np.ascontiguousarray(np.asarray(planes, dtype=np.uint8))
    squeeze = a.ndim == 2
    if squeeze:
        a = a[None]
    nl, ny, nx = a.shape
    box = np.empty_like(a)
    lap = np.empty(a.shape, dtype=np.int16)
    lib().oracle_img(nl, ny, nx, _ptr(a, _u8p), int(lap_kind), _ptr(box, _u8p), _ptr(lap, _i16p))
    if squeeze:
        return box[0], lap[0]
    return box, lap


# --------------------------------------------------------------------------- #
# Fourth-order 13-point operator on several fields
# --------------------------------------------------------------------------- #
def vc13_apply(u, c: Sequence, kappa: float, bcv: float = 0.0):
    u = _f64(u)
    nz, ny, nx = u.shape
    cp = np.ascontiguousarray(np.stack([_f64(x) for x in c]))
    out = np.empty_like(u)
    lib().oracle_vc13_apply(nx, ny, nz, _ptr(u), _ptr(cp), float(kappa), float(bcv), _ptr(out))
    return out


def vc13_diag(c: Sequence, kappa: float):
    cp = np.ascontiguousarray(np.stack([_f64(x) for x in c]))
    nz, ny, nx = cp.shape[1:]
    d = np.empty((nz, ny, nx), dtype=np.float64)
    lib().oracle_vc13_diag(nx, ny, nz, _ptr(cp), float(kappa), _ptr(d))
    return d


def vc13_residual(x, b, c, kappa: float):
    """r = b - A x in FP64."""
    return _f64(b) - vc13_apply(x, c, kappa)


def vc13_jacobi_solve(b, c, kappa: float, omega: float, rtol: float, max_sweeps: int,
                      x0=None):
    """Weighted Jacobi x <- x + omega D^-1 (b - A x) in FP64 until
    ||b - A x||_2 <= rtol ||b||_2.  Returns (x, sweeps, rel_residual)."""
    b = _f64(b)
    cp = [_f64(x) for x in c]
    d = vc13_diag(cp, kappa)
    x = np.zeros_like(b) if x0 is None else _f64(x0)
    bn = np.sqrt(sumsq(b))
    rel = float("inf")
    for n in range(max_sweeps + 1):
        r = b - vc13_apply(x, cp, kappa)
        rel = float(np.sqrt(sumsq(r)) / bn) if bn > 0 else 0.0
        if rel <= rtol or n == max_sweeps:
            return x, n, rel
        x = x + omega * r / d
    return x, max_sweeps, rel


# --------------------------------------------------------------------------- #
# do_reduce (Section 3)
# --------------------------------------------------------------------------- #
def sum(x) -> float:  # noqa: A001 - the paper's reduction name
    a = _f64(x).ravel()
    return float(lib().oracle_sum(_ptr(a), a.size))


def sumsq(x) -> float:
    a = _f64(x).ravel()
    return float(lib().oracle_sumsq(_ptr(a), a.size))


def maxabs(x) -> float:
    a = _f64(x).ravel()
    return float(lib().oracle_maxabs(_ptr(a), a.size))
