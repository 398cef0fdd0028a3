"""Seeded synthetic inputs shared by the GPU path, the tests and the benchmark.

This module only draws and describes inputs (grid shape, physics constants,
boundary kinds and values, coefficient fields, initial fields, request
streams).  It holds none of the solver's arithmetic, so both the HIP path
and the CPU oracle can consume its output without sharing any code.

The paper's workloads are synthetic heat-equation grids (section 3); these
generators stand in for them at the sizes of the benchmark configurations.
All random numbers come from numpy's PCG64 ``default_rng(seed)``, drawn in the
order written below; the GPU never draws random numbers.

Layout: every field is a C-contiguous array of shape (nz, ny, nx), x fastest.
A configuration written "A x B x C" means nx=A, ny=B, nz=C.  Cells are cubes
of side h = 1 / (max(nx, ny, nz) + 1); cell (i, j, k) has its centre at
((i+1) h, (j+1) h, (k+1) h) and the ghost cells of the boundary sit at 0 and
(n+1) h on each axis.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace

import os

import numpy as np

DIRICHLET, ZEROFLUX = 0, 1
FACES = ("x-", "x+", "y-", "y+", "z-", "z+")


@dataclass
class Problem:
    """One backward-Euler transport problem on a structured grid."""
    nx: int
    ny: int
    nz: int
    h: float
    dt: float
    alpha: float = 1.0                    # constant diffusivity (kappa is None)
    kappa: np.ndarray | None = None       # per-cell diffusivity, float32
    u: tuple = (0.0, 0.0, 0.0)            # constant velocity
    bc_kind: tuple = (DIRICHLET,) * 6     # faces x-, x+, y-, y+, z-, z+
    bc_value: tuple = (0.0,) * 6
    T0: np.ndarray | None = field(default=None, repr=False)   # initial field, float64

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def cells(self):
        return self.nx * self.ny * self.nz

    def with_(self, **kw) -> "Problem":
        return replace(self, **kw)


def grid_spacing(nx: int, ny: int, nz: int) -> float:
    return 1.0 / (max(nx, ny, nz) + 1)


# --------------------------------------------------------------------------
# benchmark configurations
# --------------------------------------------------------------------------

def heat_32(seed: int = 1, n: int = 32) -> Problem:
    """32^3 heat diffusion: constant diffusivity 1, dt 1e-3, all faces
    Dirichlet 0; T0 ~ U[0,1).  Solved to 1e-10 for 10 steps."""
    rng = np.random.default_rng(seed)
    T0 = rng.random((n, n, n))
    return Problem(n, n, n, h=grid_spacing(n, n, n), dt=1e-3, alpha=1.0, T0=T0)


MIXED_BC_KIND = (DIRICHLET, DIRICHLET, ZEROFLUX, ZEROFLUX, ZEROFLUX, ZEROFLUX)
MIXED_BC_VALUE = (1.0, 0.0, 0.0, 0.0, 0.0, 0.0)


def convdiff(n: int = 256, seed: int = 2, u=(1.0, 0.5, 0.25), dt: float = 1e-2) -> Problem:
    """Convection-diffusion on n^3: kappa = float32(exp(N(0,1))) per cell,
    constant velocity u with first-order upwind, dt 1e-2, x- Dirichlet 1,
    x+ Dirichlet 0, y and z faces zero-flux; T0 ~ U[0,1).
    Draw order: kappa, then T0."""
    rng = np.random.default_rng(seed)
    kappa = np.exp(rng.standard_normal((n, n, n))).astype(np.float32)
    T0 = rng.random((n, n, n))
    return Problem(n, n, n, h=grid_spacing(n, n, n), dt=dt, kappa=kappa, u=tuple(u),
                   bc_kind=MIXED_BC_KIND, bc_value=MIXED_BC_VALUE, T0=T0)


def convdiff_384(seed: int = 4, n: int = 384) -> Problem:
    """Mixed-precision workload: the convection-diffusion problem at 384^3
    with the velocity scaled by 4, i.e. u = (4, 2, 1)."""
    return convdiff(n=n, seed=seed, u=(4.0, 2.0, 1.0))


def smooth_kappa(nx: int, ny: int, nz: int, rng: np.random.Generator, modes: int = 8):
    """kappa = float32(2**s), s = sum_m a_m sin(2 pi k_m . X + phi_m) / sum_m a_m
    in [-1, 1], so kappa in [0.5, 2].  Draw order per mode: k_m (3 integers in
    [1,4]), a_m ~ U[0.5, 1), phi_m ~ U[0, 2 pi)."""
    ks, amps, phis = [], [], []
    for _ in range(modes):
        ks.append(rng.integers(1, 5, size=3))
        amps.append(rng.uniform(0.5, 1.0))
        phis.append(rng.uniform(0.0, 2 * np.pi))
    h = grid_spacing(nx, ny, nz)
    x = (np.arange(nx) + 1) * h
    y = (np.arange(ny) + 1) * h
    z = (np.arange(nz) + 1) * h
    total = float(sum(amps))
    kappa = np.empty((nz, ny, nx), dtype=np.float32)

    def planes(k0: int, k1: int) -> None:
        for kz in range(k0, k1):             # one plane at a time: bounded memory
            s = np.zeros((ny, nx))
            for km, am, ph in zip(ks, amps, phis):
                s += am * np.sin(2 * np.pi * (km[0] * x[None, :] + km[1] * y[:, None]
                                              + km[2] * z[kz]) + ph)
            kappa[kz] = np.exp2(s / total).astype(np.float32)

    # planes are independent and each is computed the same way whichever
    # thread takes it (numpy releases the GIL inside these array operations)
    workers = max(1, min(16, os.cpu_count() or 1, nz // 8))
    if workers == 1:
        planes(0, nz)
    else:
        from concurrent.futures import ThreadPoolExecutor
        cuts = [nz * w // workers for w in range(workers + 1)]
        with ThreadPoolExecutor(workers) as ex:
            for f in [ex.submit(planes, cuts[w], cuts[w + 1]) for w in range(workers)]:
                f.result()
    return kappa


def poisson_large(nx: int = 512, ny: int = 512, nz: int = 1024, seed: int = 3) -> Problem:
    """Large pure-diffusion step (512 x 512 x 1024 by default): smooth
    8-mode kappa in [0.5, 2], dt 1, all faces Dirichlet 0, T0 ~ U[0,1).
    Run for a fixed 500 BiCGStab iterations.  Draw order: the 8 modes,
    then T0."""
    rng = np.random.default_rng(seed)
    kappa = smooth_kappa(nx, ny, nz, rng)
    T0 = rng.random((nz, ny, nx))
    return Problem(nx, ny, nz, h=grid_spacing(nx, ny, nz), dt=1.0, kappa=kappa, T0=T0)


SERVE_DIMS = (32, 48, 64, 96, 128, 192)


@dataclass
class Request:
    index: int
    arrival: float           # seconds from the start of the stream
    nx: int
    ny: int
    nz: int

    def problem(self) -> Problem:
        """Heat-diffusion physics of the 32^3 case on this request's grid;
        T0 drawn from its own generator (seed 5_000_000 + index)."""
        rng = np.random.default_rng(5_000_000 + self.index)
        T0 = rng.random((self.nz, self.ny, self.nx))
        return Problem(self.nx, self.ny, self.nz, h=grid_spacing(self.nx, self.ny, self.nz),
                       dt=1e-3, alpha=1.0, T0=T0)


def request_stream(count: int = 2000, rate: float = 200.0, seed: int = 5):
    """Poisson arrivals at ``rate`` per second; each grid dimension drawn
    uniformly from SERVE_DIMS.  Draw order: inter-arrival times, then dims."""
    rng = np.random.default_rng(seed)
    arrivals = np.cumsum(rng.exponential(1.0 / rate, count))
    dims = rng.choice(np.array(SERVE_DIMS), size=(count, 3))
    return [Request(q, float(arrivals[q]), int(dims[q, 0]), int(dims[q, 1]), int(dims[q, 2]))
            for q in range(count)]


# --------------------------------------------------------------------------
# generic seeded problems for parity tests
# --------------------------------------------------------------------------

def random_problem(seed: int, nx: int, ny: int, nz: int, *, cell: bool = True,
                   u=(0.0, 0.0, 0.0), bc_kind=(DIRICHLET,) * 6, bc_value=None,
                   dt: float = 1e-2, sigma: float = 1.0) -> Problem:
    """Log-normal kappa (if ``cell``), T0 ~ U[0,1), optional random Dirichlet
    values in [0,1).  Draw order: kappa, T0, boundary values."""
    rng = np.random.default_rng(seed)
    kappa = (np.exp(sigma * rng.standard_normal((nz, ny, nx))).astype(np.float32)
             if cell else None)
    T0 = rng.random((nz, ny, nx))
    if bc_value is None:
        bc_value = tuple(float(v) for v in rng.random(6))
    return Problem(nx, ny, nz, h=grid_spacing(nx, ny, nz), dt=dt, alpha=1.0, kappa=kappa,
                   u=tuple(float(v) for v in u), bc_kind=tuple(bc_kind),
                   bc_value=tuple(bc_value), T0=T0)


def random_field(seed: int, shape, dtype=np.float64) -> np.ndarray:
    return np.random.default_rng(seed).random(shape).astype(dtype)
