"""Helpers for the oracle pins: dense and CSR views of the oracle's operator,
and closed-form fields.  Nothing here restates the oracle's assembly."""
from __future__ import annotations

import os

import numpy as np
import scipy.sparse as sp

from paper_2209_13768_amd.inputs import Problem, grid_spacing


def dense_by_columns(o) -> np.ndarray:
    """A as a dense matrix, column c = A applied to the unit vector e_c."""
    shape = o.shape
    n = int(np.prod(shape))
    A = np.empty((n, n))
    e = np.zeros(n)
    for c in range(n):
        e[c] = 1.0
        A[:, c] = o.apply(e.reshape(shape)).ravel()
        e[c] = 0.0
    return A


def csr_by_rows(o) -> sp.csr_matrix:
    """A in CSR form from the oracle's per-cell rows."""
    p = o.prob
    rows, cols, vals = [], [], []
    steps = [(-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)]
    for k in range(p.nz):
        for j in range(p.ny):
            for i in range(p.nx):
                c = i + p.nx * (j + p.ny * k)
                d, off, _ = o.row(i, j, k)
                rows.append(c); cols.append(c); vals.append(d)
                for f, (di, dj, dk) in enumerate(steps):
                    ii, jj, kk = i + di, j + dj, k + dk
                    if 0 <= ii < p.nx and 0 <= jj < p.ny and 0 <= kk < p.nz:
                        rows.append(c); cols.append(ii + p.nx * (jj + p.ny * kk))
                        vals.append(off[f])
    n = p.cells
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, n))


def sine_mode(nx, ny, nz, mx, my, mz) -> np.ndarray:
    """prod_d sin(pi m_d (i_d + 1) / (n_d + 1)), shape (nz, ny, nx)."""
    sx = np.sin(np.pi * mx * (np.arange(nx) + 1) / (nx + 1))
    sy = np.sin(np.pi * my * (np.arange(ny) + 1) / (ny + 1))
    sz = np.sin(np.pi * mz * (np.arange(nz) + 1) / (nz + 1))
    return sz[:, None, None] * sy[None, :, None] * sx[None, None, :]


def const_problem(nx, ny, nz, *, alpha=1.0, dt=1e-2, u=(0.0, 0.0, 0.0),
                  bc_kind=(0,) * 6, bc_value=(0.0,) * 6) -> Problem:
    return Problem(nx, ny, nz, h=grid_spacing(nx, ny, nz), dt=dt, alpha=alpha,
                   u=tuple(u), bc_kind=tuple(bc_kind), bc_value=tuple(bc_value))


def rel_l2(a, b) -> float:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def worked_examples():
    """Cases of tests/golden/worked_examples.txt: (scheme, Problem, T1) with
    every face a boundary cell at gamma and omega = alpha dt / h^2 = given."""
    from fractions import Fraction
    cases = []
    with open(os.path.join(GOLDEN, "worked_examples.txt")) as f:
        for line in f:
            if not line.strip() or line.startswith("#"):
                continue
            head, t0, t1 = (part.split() for part in line.split("|"))
            scheme, nx, ny, nz, omega, gamma = head
            nx, ny, nz = int(nx), int(ny), int(nz)
            h = grid_spacing(nx, ny, nz)
            shape = (nz, ny, nx)
            T0 = np.array([float(Fraction(v)) for v in t0]).reshape(shape)
            T1 = np.array([float(Fraction(v)) for v in t1]).reshape(shape)
            prob = Problem(nx, ny, nz, h=h, dt=float(Fraction(omega)) * h * h, alpha=1.0,
                                  bc_value=(float(Fraction(gamma)),) * 6, T0=T0)
            cases.append((scheme, prob, T1))
    return cases
