"""Python side of the FP64 CPU oracle (``oracle.c``).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import this module.  It shares nothing with
the HIP library: it takes a problem description from the seeded input
generators and plain NumPy arrays, and returns NumPy arrays.

Every entry point mirrors a function of ``oracle.c``; the mathematics and the
paper passages each one follows are documented there.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
# A test may point the oracle at another build of oracle.c (for instance one
# with a planted mistake, to show that the pins catch it).
_LIB_OVERRIDE = os.environ.get("ORACLE_LIB")

OK, BREAKDOWN, NOCONV, NONFINITE = 0, -4, -5, -6
DIRICHLET, ZEROFLUX = 0, 1


def build(force: bool = True, extra_flags: tuple[str, ...] = (), out: str | None = None) -> str:
    """Compile ``oracle.c`` with gcc into a shared library and return its path."""
    out = out or _LIB
    if not force and os.path.exists(out) and os.path.getmtime(out) >= os.path.getmtime(_SRC):
        return out
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", *extra_flags,
           "-o", out + ".tmp", _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


class _Problem(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("cell_kappa", ctypes.c_int32),
        ("h", ctypes.c_double), ("dt", ctypes.c_double), ("alpha", ctypes.c_double),
        ("kappa", ctypes.c_void_p),
        ("u", ctypes.c_double * 3),
        ("bc_kind", ctypes.c_int32 * 6),
        ("bc_value", ctypes.c_double * 6),
    ]


class _Info(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int32), ("iterations", ctypes.c_int32),
        ("restarts", ctypes.c_int32), ("pad", ctypes.c_int32),
        ("rel_res_recursive", ctypes.c_double), ("rel_res_true", ctypes.c_double),
    ]


@dataclass
class SolveInfo:
    status: int
    iterations: int
    restarts: int
    rel_res_recursive: float
    rel_res_true: float


_lib_cache: dict[str, ctypes.CDLL] = {}


def load(path: str | None = None) -> ctypes.CDLL:
    """Load (building first if absent) the oracle library at ``path``."""
    path = path or _LIB_OVERRIDE or _LIB
    if path in _lib_cache:
        return _lib_cache[path]
    if path == _LIB and not os.path.exists(path):
        build(force=False)
    lib = ctypes.CDLL(path)
    P = ctypes.POINTER(_Problem)
    D = ctypes.POINTER(ctypes.c_double)
    I = ctypes.POINTER(_Info)
    lib.orc_row.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_int, D, D, D]
    lib.orc_apply.argtypes = [P, D, D]
    lib.orc_rhs.argtypes = [P, D, D]
    lib.orc_dot.argtypes = [P, D, D]
    lib.orc_dot.restype = ctypes.c_double
    lib.orc_true_relres.argtypes = [P, D, D]
    lib.orc_true_relres.restype = ctypes.c_double
    lib.orc_bicgstab.argtypes = [P, D, D, ctypes.c_double, ctypes.c_int, D, I]
    lib.orc_cg.argtypes = [P, D, D, ctypes.c_double, ctypes.c_int, D, I]
    lib.orc_cg1.argtypes = [P, D, D, ctypes.c_double, ctypes.c_int, D, I]
    lib.orc_bicgstab2.argtypes = [P, D, D, ctypes.c_double, ctypes.c_int, D, I]
    lib.orc_bicgstab2_shadow.argtypes = [P, D, D, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                         ctypes.c_int, D, I]
    lib.orc_bicgstab_forced.argtypes = [P, D, D, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                        D, I]
    lib.orc_shadow.argtypes = [ctypes.c_long, D]
    lib.orc_bicgstab_jacobi.argtypes = [P, D, D, ctypes.c_double, ctypes.c_int, D, I]
    lib.orc_timestep.argtypes = [P, D, ctypes.c_int, ctypes.c_double, ctypes.c_int, I]
    lib.orc_explicit.argtypes = [P, D, ctypes.c_int]
    lib.orc_num_threads.restype = ctypes.c_int
    lib.orc_set_num_threads.argtypes = [ctypes.c_int]
    _lib_cache[path] = lib
    return lib


class Oracle:
    """Oracle bound to one problem description (any object with the fields of
    ``paper_2209_13768_amd.inputs.Problem``)."""

    def __init__(self, prob, lib_path: str | None = None):
        self.lib = load(lib_path)
        self.prob = prob
        self.shape = (prob.nz, prob.ny, prob.nx)
        self._kappa = None
        s = _Problem()
        s.nx, s.ny, s.nz = prob.nx, prob.ny, prob.nz
        s.cell_kappa = 1 if prob.kappa is not None else 0
        s.h, s.dt, s.alpha = prob.h, prob.dt, prob.alpha
        if prob.kappa is not None:
            k = np.ascontiguousarray(prob.kappa, dtype=np.float32)
            assert k.shape == self.shape
            self._kappa = k
            s.kappa = k.ctypes.data
        s.u = (ctypes.c_double * 3)(*[float(v) for v in prob.u])
        s.bc_kind = (ctypes.c_int32 * 6)(*[int(v) for v in prob.bc_kind])
        s.bc_value = (ctypes.c_double * 6)(*[float(v) for v in prob.bc_value])
        self._s = s

    # -- helpers ----------------------------------------------------------
    def _vec(self, a) -> np.ndarray:
        a = np.ascontiguousarray(a, dtype=np.float64)
        assert a.shape == self.shape, (a.shape, self.shape)
        return a

    @staticmethod
    def _ptr(a: np.ndarray):
        return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))

    @property
    def _p(self):
        return ctypes.byref(self._s)

    # -- entry points ------------------------------------------------------
    def row(self, i: int, j: int, k: int):
        """(diag, off[6], bterm) of the row of A for cell (i, j, k)."""
        d = ctypes.c_double()
        off = (ctypes.c_double * 6)()
        bt = ctypes.c_double()
        self.lib.orc_row(self._p, i, j, k, ctypes.byref(d), off, ctypes.byref(bt))
        return d.value, np.array(off[:], dtype=np.float64), bt.value

    def apply(self, x) -> np.ndarray:
        x = self._vec(x)
        y = np.empty_like(x)
        self.lib.orc_apply(self._p, self._ptr(x), self._ptr(y))
        return y

    def rhs(self, Tn) -> np.ndarray:
        Tn = self._vec(Tn)
        b = np.empty_like(Tn)
        self.lib.orc_rhs(self._p, self._ptr(Tn), self._ptr(b))
        return b

    def dot(self, a, b) -> float:
        a, b = self._vec(a), self._vec(b)
        return float(self.lib.orc_dot(self._p, self._ptr(a), self._ptr(b)))

    def true_relres(self, b, x) -> float:
        b, x = self._vec(b), self._vec(x)
        return float(self.lib.orc_true_relres(self._p, self._ptr(b), self._ptr(x)))

    def _krylov(self, fn, b, x0, tol, maxit, want_r):
        b = self._vec(b)
        x = self._vec(x0).copy()
        r = np.empty_like(x) if want_r else None
        info = _Info()
        fn(self._p, self._ptr(b), self._ptr(x), float(tol), int(maxit),
           self._ptr(r) if want_r else None, ctypes.byref(info))
        out = SolveInfo(info.status, info.iterations, info.restarts,
                        info.rel_res_recursive, info.rel_res_true)
        return (x, out, r) if want_r else (x, out)

    def bicgstab(self, b, x0, tol: float, maxit: int, want_r: bool = False,
                 force_breakdown: int = 0):
        """Textbook BiCGStab (oracle.c).  force_breakdown = n > 0 takes sigma
        of full iteration n as exactly zero, once, so that the method
        restarts there."""
        if not force_breakdown:
            return self._krylov(self.lib.orc_bicgstab, b, x0, tol, maxit, want_r)
        fn = self.lib.orc_bicgstab_forced

        def forced(p, bp, xp, tol_, maxit_, rp, ip):
            return fn(p, bp, xp, tol_, maxit_, int(force_breakdown), rp, ip)
        return self._krylov(forced, b, x0, tol, maxit, want_r)

    def bicgstab2(self, b, x0, tol: float, maxit: int, want_r: bool = False,
                  hashed_shadow: bool = False, force_breakdown: int = 0):
        """BiCGStab with two reductions per iteration (oracle.c); with
        hashed_shadow the shadow residual is the index-hashed field of
        shadow() instead of r0.  force_breakdown as for bicgstab."""
        fn = self.lib.orc_bicgstab2_shadow

        def with_shadow(p, bp, xp, tol_, maxit_, rp, ip):
            return fn(p, bp, xp, tol_, maxit_, 1 if hashed_shadow else 0,
                      int(force_breakdown), rp, ip)
        return self._krylov(with_shadow, b, x0, tol, maxit, want_r)

    def shadow(self):
        """The index-hashed shadow residual (oracle.c, orc_shadow)."""
        rh = np.empty(self.shape)
        self.lib.orc_shadow(int(rh.size), self._ptr(rh))
        return rh

    def bicgstab_jacobi(self, b, x0, tol: float, maxit: int, want_r: bool = False):
        """BiCGStab on D^{-1} A x = D^{-1} b (oracle.c)."""
        return self._krylov(self.lib.orc_bicgstab_jacobi, b, x0, tol, maxit, want_r)

    def cg(self, b, x0, tol: float, maxit: int, want_r: bool = False):
        return self._krylov(self.lib.orc_cg, b, x0, tol, maxit, want_r)

    def cg1(self, b, x0, tol: float, maxit: int, want_r: bool = False):
        """CG with one reduction per iteration (Chronopoulos-Gear; oracle.c)."""
        return self._krylov(self.lib.orc_cg1, b, x0, tol, maxit, want_r)

    def timestep(self, T, nsteps: int, tol: float, maxit: int):
        T = self._vec(T).copy()
        infos = (_Info * max(nsteps, 1))()
        self.lib.orc_timestep(self._p, self._ptr(T), int(nsteps), float(tol), int(maxit), infos)
        return T, [SolveInfo(i.status, i.iterations, i.restarts, i.rel_res_recursive,
                             i.rel_res_true) for i in infos[:nsteps]]


def _explicit(self, T, nsteps: int) -> np.ndarray:
    """nsteps explicit forward-time steps (oracle.c orc_explicit)."""
    T = self._vec(T).copy()
    self.lib.orc_explicit(self._p, self._ptr(T), int(nsteps))
    return T


Oracle.explicit = _explicit


def num_threads() -> int:
    return int(load().orc_num_threads())


def set_num_threads(n: int) -> None:
    load().orc_set_num_threads(int(n))
