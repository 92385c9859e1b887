"""Seeded synthetic inputs for the stencil workloads.

This module holds random-number draws and closed-form input fields only: none
of the stencil arithmetic.  The same host arrays are handed to the HIP library
and to the CPU oracle, so both sides see bit-identical inputs.

Seeds are ``12071746 + 100 * workload + grid_index``; every generator takes the
grid sizes as arguments so that small parity cases reuse the full-size recipe.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

SEED_BASE = 12071746


def rng(workload: int, index: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(SEED_BASE + 100 * workload + index))


def round_to_bf16(x: np.ndarray) -> np.ndarray:
    """Round float32 values to the nearest bfloat16 (ties to even), returned as
    float32 holding exactly representable bfloat16 values."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    bits = a.view(np.uint32).astype(np.uint64)
    lsb = (bits >> 16) & 1
    rounded = ((bits + 0x7FFF + lsb) >> 16) << 16
    return rounded.astype(np.uint32).view(np.float32).reshape(a.shape)


# --------------------------------------------------------------------------- #
# Jacobi averaging on a cube (64^3 FP64, Dirichlet 0, f = 0, 10 sweeps)
# --------------------------------------------------------------------------- #
def jacobi_cube(n: int = 64, ny: int | None = None, nz: int | None = None):
    """u0 ~ U[-1, 1] on an (nz, ny, n) FP64 grid; grid spacing 1/(n+1)."""
    ny = ny or n
    nz = nz or n
    u0 = rng(1, 0).uniform(-1.0, 1.0, size=(nz, ny, n))
    h = 1.0 / (n + 1)
    return u0, h * h


def jacobi_rhs(n: int, ny: int | None = None, nz: int | None = None) -> np.ndarray:
    """f ~ N(0, 1) on an (nz, ny, n) FP64 grid (right-hand side of the large
    temporally blocked runs)."""
    ny = ny or n
    nz = nz or n
    return rng(1, 1).standard_normal((nz, ny, n))


# --------------------------------------------------------------------------- #
# Variable-coefficient multi-grid sweep (256^3 FP32, periodic)
# --------------------------------------------------------------------------- #
def varcoef_grids(nx: int = 256, ny: int | None = None, nz: int | None = None):
    """u ~ N(0,1), c_0..c_6 ~ U[0.1, 1], s ~ U[-1, 1], all float32."""
    ny = ny or nx
    nz = nz or nx
    shp = (nz, ny, nx)
    u = rng(2, 0).standard_normal(shp, dtype=np.float32)
    c = [rng(2, 1 + k).uniform(0.1, 1.0, size=shp).astype(np.float32) for k in range(7)]
    s = rng(2, 8).uniform(-1.0, 1.0, size=shp).astype(np.float32)
    return u, c, s


# --------------------------------------------------------------------------- #
# Integer image planes (4 x 8192^2 uint8)
# --------------------------------------------------------------------------- #
def image_planes(nx: int = 8192, ny: int | None = None, nplanes: int = 4):
    ny = ny or nx
    return rng(3, 0).integers(0, 256, size=(nplanes, ny, nx), dtype=np.uint8)


# --------------------------------------------------------------------------- #
# Poisson solve requests (cube sides log-uniform in [32, 192])
# --------------------------------------------------------------------------- #
@dataclass
class PoissonRequest:
    rid: int
    n: int
    arrival: float           # seconds after the stream starts
    modes: list              # [(k, l, m, amplitude)]

    @property
    def h2(self) -> float:
        h = 1.0 / (self.n + 1)
        return h * h


def poisson_requests(count: int = 2000, qps: float = 100.0, nmin: int = 32,
                     nmax: int = 192, nmodes: int = 3, kmax: int = 4,
                     seed_index: int = 0) -> list[PoissonRequest]:
    """Poisson arrivals at ``qps`` (qps = inf: everything at t = 0); N =
    floor(exp(U[ln nmin, ln(nmax+1)))); modes with wave numbers in 1..kmax and
    N(0,1) amplitudes, wave-number triples distinct within a request."""
    g = rng(4, seed_index)
    reqs = []
    t = 0.0
    for rid in range(count):
        if math.isfinite(qps):
            t += g.exponential(1.0 / qps)
        n = int(math.floor(math.exp(g.uniform(math.log(nmin), math.log(nmax + 1)))))
        n = min(max(n, nmin), nmax)
        seen = set()
        modes = []
        while len(modes) < nmodes:
            klm = tuple(int(v) for v in g.integers(1, kmax + 1, size=3))
            if klm in seen:
                continue
            seen.add(klm)
            modes.append((*klm, float(g.standard_normal())))
        reqs.append(PoissonRequest(rid, n, t if math.isfinite(qps) else 0.0, modes))
    return reqs


def sine_mode(n: int, k: int, l: int, m: int) -> np.ndarray:
    """phi(i,j,q) = sin(k pi x_i) sin(l pi y_j) sin(m pi z_q) on the interior
    points x = (index+1)/(n+1), as an (n, n, n) array indexed [z][y][x]."""
    x = np.arange(1, n + 1, dtype=np.float64) / (n + 1)
    sx = np.sin(k * math.pi * x)
    sy = np.sin(l * math.pi * x)
    sz = np.sin(m * math.pi * x)
    return sz[:, None, None] * sy[None, :, None] * sx[None, None, :]


def mode_eigenvalue(n: int, k: int, l: int, m: int) -> float:
    """Closed-form eigenvalue of the Dirichlet 7-point discrete Laplacian for
    the sine mode (k, l, m): (2/h^2) (cos k pi h + cos l pi h + cos m pi h - 3)."""
    h = 1.0 / (n + 1)
    return (2.0 / (h * h)) * (math.cos(k * math.pi * h) + math.cos(l * math.pi * h)
                              + math.cos(m * math.pi * h) - 3.0)


def poisson_fields(req: PoissonRequest):
    """(u_star, f): the exact discrete solution sum a*phi and f = sum a*lambda*phi."""
    u = np.zeros((req.n,) * 3)
    f = np.zeros((req.n,) * 3)
    for k, l, m, a in req.modes:
        phi = sine_mode(req.n, k, l, m)
        u += a * phi
        f += a * mode_eigenvalue(req.n, k, l, m) * phi
    return u, f


# --------------------------------------------------------------------------- #
# Fourth-order multi-field operator (512^3, 5 fields, 10 coefficient grids)
# --------------------------------------------------------------------------- #
VC13_KAPPA = 0.25


def vc13_grids(n: int = 512, ny: int | None = None, nz: int | None = None,
               nfields: int = 5):
    """10 coefficient grids ~ U[0.5, 1.5] rounded to bfloat16 (exact in every
    storage type), and nfields right-hand sides b ~ N(0,1) in FP64."""
    ny = ny or n
    nz = nz or n
    shp = (nz, ny, n)
    c = [round_to_bf16(rng(5, k).uniform(0.5, 1.5, size=shp).astype(np.float32))
         for k in range(10)]
    b = [rng(5, 10 + f).standard_normal(shp) for f in range(nfields)]
    return c, b


def vc13_fields(n: int, ny: int | None = None, nz: int | None = None, nfields: int = 5):
    """Prognostic fields ~ N(0,1) (float32) to which the operator is applied."""
    ny = ny or n
    nz = nz or n
    return [rng(5, 20 + f).standard_normal((nz, ny, n), dtype=np.float32)
            for f in range(nfields)]
