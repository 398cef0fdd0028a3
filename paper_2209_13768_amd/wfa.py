"""Thin Python binding of libwfa.so (ctypes).

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  torch provides device memory (tensors; their data_ptr() is
handed to the C-ABI) and streams (torch.cuda.current_stream()).  The names
mirror include/wfa.h.  There is no fallback: if libwfa.so is missing or no
GPU is present, calls raise.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libwfa.so")

OK, PENDING = 0, 1
ERR_INVALID, ERR_NOMEM, ERR_HIP, ERR_BREAKDOWN, ERR_NOCONV, ERR_NONFINITE = -1, -2, -3, -4, -5, -6
F64, F32, F32_IR64 = 0, 1, 2
COEF_CONST, COEF_CELL = 0, 1
BC_DIRICHLET, BC_ZEROFLUX = 0, 1
METHOD_BICGSTAB, METHOD_CG, METHOD_BICGSTAB2, METHOD_CG1 = 0, 1, 2, 3
OPT_METHOD, OPT_PERSISTENT, OPT_PROFILE, OPT_FORCE_BREAKDOWN, OPT_CHECK_EVERY = 1, 2, 3, 4, 5
OPT_IR_INNER_TOL, OPT_ZCHUNK, OPT_RY, OPT_JACOBI, OPT_GRAPH = 6, 7, 8, 9, 10
OPT_EXPLICIT_FUSE, OPT_SHADOW, OPT_FORCE_DIVERGE, OPT_CG1_MAX_CELLS = 11, 12, 13, 14
OPT_RECOMPUTE_T = 15
OPT_SIZE_CLASS_1, OPT_SIZE_CLASS_2, OPT_SIZE_CLASS_3 = 16, 17, 18
K_APPLY, K_INIT, K_PHASE_A, K_PHASE_B, K_PHASE_C, K_RESIDUAL, K_PROMOTE = 0, 1, 2, 3, 4, 5, 6
K_CG_A, K_CG_B, K_PERSISTENT, K_PHASE_AC, K_PHASE_B2, K_EXPLICIT = 7, 8, 9, 10, 11, 12
K_EXPLICIT_FUSED, K_CG1, K_COUNT = 13, 14, 15
VEC_R, VEC_RHAT, VEC_T, VEC_P0, VEC_P1, VEC_V0, VEC_V1, VEC_B, VEC_R1 = range(9)
PROBE_COPY, PROBE_COPY_PLAIN, PROBE_COPY32, PROBE_READ, PROBE_WRITE = range(5)
PROBE_MIX_6R4W, PROBE_MIX_3R1W = 5, 6
PROBE_NAMES = ("copy_nt16", "copy_plain16", "copy_nt32", "read_nt16", "write_nt16",
               "mix_6r4w_nt16", "mix_3r1w_nt16")
# streams read and written by each probe kind (a copy reads one, writes one)
PROBE_STREAMS = ((1, 1), (1, 1), (1, 1), (1, 0), (0, 1), (6, 4), (3, 1))
KERNEL_NAMES = ("apply", "init", "phase_a", "phase_b", "phase_c", "residual", "promote",
                "cg_a", "cg_b", "persistent", "phase_ac", "phase_b2", "explicit", "explicit_fused",
                "cg1")

PRECISIONS = {"f64": F64, "f32": F32, "f32_ir64": F32_IR64}

# Every function the header declares; the library must export all of them.
EXPORTS = (
    "wfa_workspace_bytes", "wfa_grid_create", "wfa_grid_destroy", "wfa_stencil_apply",
    "wfa_rhs", "wfa_explicit_step", "wfa_bicgstab_solve", "wfa_bicgstab2_solve", "wfa_cg_solve", "wfa_cg1_solve", "wfa_timestep", "wfa_true_residual",
    "wfa_grid_set_option", "wfa_kernel_stats", "wfa_grid_tiling", "wfa_grid_vector",
    "wfa_stream_probe", "wfa_bandwidth_probe", "wfa_bicgstab_solve_static",
    "wfa_server_create", "wfa_server_set_option", "wfa_submit", "wfa_poll", "wfa_server_drain",
    "wfa_server_destroy",
    "wfa_last_error", "wfa_version", "wfa_autotune", "wfa_tune_save", "wfa_tune_load",
    "wfa_tune_clear",
)


class WfaError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"wfa error {code}: {msg}")
        self.code = code


class Coeffs(ctypes.Structure):
    _fields_ = [
        ("mode", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("h", ctypes.c_double), ("dt", ctypes.c_double), ("alpha", ctypes.c_double),
        ("kappa", ctypes.c_void_p),
        ("u", ctypes.c_double * 3),
        ("bc", ctypes.c_int32 * 6),
        ("bc_value", ctypes.c_double * 6),
    ]


class _Info(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int32), ("iterations", ctypes.c_int32),
        ("refinements", ctypes.c_int32), ("restarts", ctypes.c_int32),
        ("rel_res_recursive", ctypes.c_double), ("rel_res_true", ctypes.c_double),
        ("seconds", ctypes.c_double),
    ]


class TuneResult(ctypes.Structure):
    _fields_ = [
        ("ry", ctypes.c_int32), ("zc", ctypes.c_int32),
        ("candidates", ctypes.c_int32), ("pad", ctypes.c_int32),
        ("us_per_iter", ctypes.c_double), ("us_per_iter_default", ctypes.c_double),
    ]


@dataclass
class SolveInfo:
    status: int
    iterations: int
    refinements: int
    restarts: int
    rel_res_recursive: float
    rel_res_true: float
    seconds: float

    @staticmethod
    def of(i: _Info) -> "SolveInfo":
        return SolveInfo(i.status, i.iterations, i.refinements, i.restarts,
                         i.rel_res_recursive, i.rel_res_true, i.seconds)


_lib = None


def lib() -> ctypes.CDLL:
    """Load libwfa.so (built in-tree by paper_2209_13768_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libwfa.so not found at {LIB_PATH}: build it first "
                          "(python -m paper_2209_13768_amd.build)")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dbl, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t
    L.wfa_workspace_bytes.argtypes = [i32, i32, i32, i32]
    L.wfa_workspace_bytes.restype = sz
    L.wfa_grid_create.argtypes = [i32, i32, i32, ctypes.POINTER(Coeffs), vp, sz, ctypes.POINTER(vp)]
    L.wfa_grid_destroy.argtypes = [vp]
    L.wfa_stencil_apply.argtypes = [vp, vp, vp, vp]
    L.wfa_rhs.argtypes = [vp, vp, vp, vp]
    L.wfa_explicit_step.argtypes = [vp, vp, i32, vp]
    L.wfa_bicgstab_solve.argtypes = [vp, vp, vp, dbl, i32, ctypes.POINTER(_Info), vp]
    L.wfa_cg_solve.argtypes = [vp, vp, vp, dbl, i32, ctypes.POINTER(_Info), vp]
    L.wfa_cg1_solve.argtypes = [vp, vp, vp, dbl, i32, ctypes.POINTER(_Info), vp]
    L.wfa_bicgstab2_solve.argtypes = [vp, vp, vp, dbl, i32, ctypes.POINTER(_Info), vp]
    L.wfa_bicgstab_solve_static.argtypes = [i32, i32, i32, ctypes.POINTER(Coeffs), vp, vp, dbl,
                                            i32, ctypes.POINTER(_Info), vp]
    L.wfa_timestep.argtypes = [vp, vp, i32, dbl, i32, ctypes.POINTER(_Info), vp]
    L.wfa_true_residual.argtypes = [vp, vp, vp, ctypes.POINTER(dbl), vp]
    L.wfa_grid_set_option.argtypes = [vp, i32, i64]
    L.wfa_kernel_stats.argtypes = [vp, i32, ctypes.POINTER(i64), ctypes.POINTER(dbl),
                                   ctypes.POINTER(dbl), i32]
    L.wfa_grid_tiling.argtypes = [vp] + [ctypes.POINTER(i32)] * 4
    L.wfa_grid_vector.argtypes = [vp, i32, ctypes.POINTER(vp)]
    L.wfa_stream_probe.argtypes = [vp, vp, sz, i32, ctypes.POINTER(dbl), vp]
    L.wfa_bandwidth_probe.argtypes = [i32, i32, vp, vp, sz, i32, ctypes.POINTER(dbl), vp]
    L.wfa_server_create.argtypes = [vp, sz, i32, vp, ctypes.POINTER(vp)]
    L.wfa_server_set_option.argtypes = [vp, i32, i64]
    L.wfa_submit.argtypes = [vp, i32, i32, i32, ctypes.POINTER(Coeffs), vp, dbl, i32,
                             ctypes.POINTER(ctypes.c_uint64)]
    L.wfa_poll.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(_Info)]
    L.wfa_server_drain.argtypes = [vp]
    L.wfa_server_destroy.argtypes = [vp]
    L.wfa_autotune.argtypes = [vp, i32, vp, vp, i32, ctypes.POINTER(TuneResult), vp]
    L.wfa_tune_save.argtypes = [ctypes.c_char_p]
    L.wfa_tune_load.argtypes = [ctypes.c_char_p]
    L.wfa_tune_clear.argtypes = []
    L.wfa_last_error.restype = ctypes.c_char_p
    L.wfa_version.restype = ctypes.c_char_p
    _lib = L
    return L


def last_error() -> str:
    return lib().wfa_last_error().decode()


def _check(rc: int, allow=(OK,)) -> int:
    if rc not in allow:
        raise WfaError(rc, last_error())
    return rc


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("libwfa needs a GPU (torch.cuda.is_available() is False)")
    return torch


def _stream_ptr(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dev(t, dtype, n, name):
    if t.dtype != dtype or not t.is_cuda or not t.is_contiguous() or t.numel() != n:
        raise ValueError(f"{name}: need a contiguous {dtype} CUDA tensor of {n} elements, "
                         f"got {t.dtype} {tuple(t.shape)} on {t.device}")
    return ctypes.c_void_p(t.data_ptr())


def make_coeffs(*, h, dt, alpha=1.0, kappa=None, u=(0.0, 0.0, 0.0), bc=(BC_DIRICHLET,) * 6,
                bc_value=(0.0,) * 6, precision=F64) -> Coeffs:
    c = Coeffs()
    c.mode = COEF_CELL if kappa is not None else COEF_CONST
    c.precision = precision
    c.h, c.dt, c.alpha = float(h), float(dt), float(alpha)
    c.kappa = ctypes.c_void_p(kappa.data_ptr()) if kappa is not None else None
    c.u = (ctypes.c_double * 3)(*[float(v) for v in u])
    c.bc = (ctypes.c_int32 * 6)(*[int(v) for v in bc])
    c.bc_value = (ctypes.c_double * 6)(*[float(v) for v in bc_value])
    return c


def workspace_bytes(nx, ny, nz, precision=F64) -> int:
    return int(lib().wfa_workspace_bytes(nx, ny, nz, precision))


class Grid:
    """A structured grid with its operator and Krylov workspace (wfa_grid)."""

    def __init__(self, nx, ny, nz, *, h, dt, alpha=1.0, kappa=None, u=(0.0, 0.0, 0.0),
                 bc=(BC_DIRICHLET,) * 6, bc_value=(0.0,) * 6, precision=F64, device="cuda"):
        torch = _torch()
        if isinstance(precision, str):
            precision = PRECISIONS[precision]
        self.nx, self.ny, self.nz = nx, ny, nz
        self.shape = (nz, ny, nx)
        self.n = nx * ny * nz
        self.precision = precision
        self.dtype = torch.float32 if precision == F32 else torch.float64
        if kappa is not None:
            kappa = kappa.to(device=device, dtype=torch.float32).contiguous()
            if tuple(kappa.shape) != self.shape:
                raise ValueError(f"kappa must have shape {self.shape}")
        self.kappa = kappa  # kept alive for the grid's lifetime
        self._coeffs = make_coeffs(h=h, dt=dt, alpha=alpha, kappa=kappa, u=u, bc=bc,
                                   bc_value=bc_value, precision=precision)
        nbytes = workspace_bytes(nx, ny, nz, precision)
        if nbytes == 0:
            raise WfaError(ERR_INVALID, "bad grid dimensions")
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        base = self.workspace.data_ptr()
        off = (-base) % 256
        self._ws_ptr = ctypes.c_void_p(base + off)
        h_ = ctypes.c_void_p()
        _check(lib().wfa_grid_create(nx, ny, nz, ctypes.byref(self._coeffs), self._ws_ptr,
                                     nbytes, ctypes.byref(h_)))
        self._h = h_

    @classmethod
    def from_problem(cls, prob, precision=F64, device="cuda") -> "Grid":
        torch = _torch()
        kappa = torch.from_numpy(prob.kappa).to(device) if prob.kappa is not None else None
        return cls(prob.nx, prob.ny, prob.nz, h=prob.h, dt=prob.dt, alpha=prob.alpha,
                   kappa=kappa, u=prob.u, bc=prob.bc_kind, bc_value=prob.bc_value,
                   precision=precision, device=device)

    # -- lifetime -----------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().wfa_grid_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- helpers ------------------------------------------------------------
    def field(self, data=None):
        """A device field of this grid's vector type (zeros, or a copy of data)."""
        torch = _torch()
        if data is None:
            return torch.zeros(self.shape, dtype=self.dtype, device="cuda")
        if not isinstance(data, torch.Tensor):
            data = torch.from_numpy(data)
        return data.to(device="cuda", dtype=self.dtype).reshape(self.shape).contiguous()

    def _v(self, t, name):
        return _dev(t, self.dtype, self.n, name)

    # -- entry points -------------------------------------------------------
    def apply(self, x, y=None, stream=None):
        y = self.field() if y is None else y
        _check(lib().wfa_stencil_apply(self._h, self._v(x, "x"), self._v(y, "y"), _stream_ptr(stream)))
        return y

    def rhs(self, T, b=None, stream=None):
        b = self.field() if b is None else b
        _check(lib().wfa_rhs(self._h, self._v(T, "T"), self._v(b, "b"), _stream_ptr(stream)))
        return b

    def explicit(self, T, nsteps=1, stream=None):
        """nsteps explicit forward-time steps of T in place."""
        _check(lib().wfa_explicit_step(self._h, self._v(T, "T"), int(nsteps), _stream_ptr(stream)))
        return T

    def solve(self, b, x=None, *, tol=1e-10, maxit=1000, method="bicgstab", check=True,
              stream=None):
        """Solve A x = b in place on x (initial guess; zeros when None)."""
        x = self.field() if x is None else x
        info = _Info()
        fn = {"cg": lib().wfa_cg_solve, "bicgstab": lib().wfa_bicgstab_solve,
              "bicgstab2": lib().wfa_bicgstab2_solve, "cg1": lib().wfa_cg1_solve}[method]
        rc = fn(self._h, self._v(b, "b"), self._v(x, "x"), float(tol), int(maxit),
                ctypes.byref(info), _stream_ptr(stream))
        if check:
            _check(rc, allow=(OK, ERR_NOCONV))
        return x, SolveInfo.of(info)

    def timestep(self, T, nsteps=1, *, tol=1e-10, maxit=1000, check=True, stream=None):
        infos = (_Info * max(nsteps, 1))()
        rc = lib().wfa_timestep(self._h, self._v(T, "T"), int(nsteps), float(tol), int(maxit),
                                infos, _stream_ptr(stream))
        if check:
            _check(rc, allow=(OK,))
        return [SolveInfo.of(i) for i in infos[:nsteps]]

    def true_residual(self, b, x, stream=None) -> float:
        rel = ctypes.c_double()
        _check(lib().wfa_true_residual(self._h, self._v(b, "b"), self._v(x, "x"),
                                       ctypes.byref(rel), _stream_ptr(stream)))
        return rel.value

    def autotune(self, method="bicgstab2", iters=20, stream=None) -> dict:
        """Time the candidate tile shapes on this grid, keep the fastest and
        record it for grids of the same key (wfa_autotune)."""
        x, b = self.field(), self.field()
        r = TuneResult()
        m = {"bicgstab": METHOD_BICGSTAB, "cg": METHOD_CG, "bicgstab2": METHOD_BICGSTAB2,
             "cg1": METHOD_CG1}[method]
        _check(lib().wfa_autotune(self._h, m, self._v(x, "x"), self._v(b, "b"), int(iters),
                                  ctypes.byref(r), _stream_ptr(stream)))
        return {"ry": r.ry, "zc": r.zc, "candidates": r.candidates, "us_per_iter": r.us_per_iter,
                "us_per_iter_default": r.us_per_iter_default}

    def set_option(self, option: int, value: int):
        _check(lib().wfa_grid_set_option(self._h, int(option), int(value)))

    def kernel_stats(self, kernel: int, reset: bool = False):
        n = ctypes.c_int64()
        ms = ctypes.c_double()
        by = ctypes.c_double()
        _check(lib().wfa_kernel_stats(self._h, int(kernel), ctypes.byref(n), ctypes.byref(ms),
                                      ctypes.byref(by), int(reset)))
        return n.value, ms.value, by.value

    def tiling(self):
        v = [ctypes.c_int() for _ in range(4)]
        _check(lib().wfa_grid_tiling(self._h, *[ctypes.byref(q) for q in v]))
        return tuple(q.value for q in v)

    def vector(self, which: int):
        """A view (no copy) of one of the grid's Krylov vectors inside its
        workspace (wfa_grid_vector), shape (nz, ny, nx)."""
        torch = _torch()
        ptr = ctypes.c_void_p()
        _check(lib().wfa_grid_vector(self._h, int(which), ctypes.byref(ptr)))
        dt = torch.float64 if self.precision == F64 else torch.float32
        off = ptr.value - self.workspace.data_ptr()
        nbytes = self.n * (8 if dt == torch.float64 else 4)
        assert 0 <= off and off + nbytes <= self.workspace.numel()
        return self.workspace[off:off + nbytes].view(dt).view(self.shape)


STATIC_WORKSPACE_BYTES = 64 << 20


def solve_static(prob_or_grid_args: dict, b, x, *, tol=1e-10, maxit=1000, check=True, stream=None):
    """wfa_bicgstab_solve_static: BiCGStab on A x = b (x in place) with the
    library's static workspace.  prob_or_grid_args: the keyword arguments of
    Grid (nx, ny, nz, h, dt, alpha, kappa, u, bc, bc_value, precision)."""
    torch = _torch()
    a = dict(prob_or_grid_args)
    nx, ny, nz = a.pop("nx"), a.pop("ny"), a.pop("nz")
    precision = a.pop("precision", F64)
    if isinstance(precision, str):
        precision = PRECISIONS[precision]
    kappa = a.pop("kappa", None)
    if kappa is not None:
        kappa = kappa.to(device="cuda", dtype=torch.float32).contiguous()
    c = make_coeffs(kappa=kappa, precision=precision, **a)
    dtype = torch.float32 if precision == F32 else torch.float64
    n = nx * ny * nz
    info = _Info()
    rc = lib().wfa_bicgstab_solve_static(nx, ny, nz, ctypes.byref(c), _dev(b, dtype, n, "b"),
                                         _dev(x, dtype, n, "x"), float(tol), int(maxit),
                                         ctypes.byref(info), _stream_ptr(stream))
    if check:
        _check(rc, allow=(OK, ERR_NOCONV))
    return x, SolveInfo.of(info)


def tune_save(path: str):
    _check(lib().wfa_tune_save(os.fsencode(path)))


def tune_load(path: str):
    _check(lib().wfa_tune_load(os.fsencode(path)))


def tune_clear():
    _check(lib().wfa_tune_clear())


def stream_probe(nbytes: int = 1 << 30, reps: int = 10, stream=None) -> float:
    """Achievable HBM copy bandwidth in GB/s (read + write)."""
    torch = _torch()
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    src.fill_(1)
    g = ctypes.c_double()
    _check(lib().wfa_stream_probe(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()),
                                  nbytes, int(reps), ctypes.byref(g), _stream_ptr(stream)))
    return g.value


def bandwidth_probe(kind: int, src, dst, reps: int = 10, blocks: int = 0, stream=None) -> float:
    """GB/s of one access pattern (PROBE_*) over the device tensors src and
    dst (same size in bytes; src unused by PROBE_WRITE).  The stream mixes
    take src holding their read streams back to back and dst their written
    ones, all of one size."""
    if not (src.is_cuda and dst.is_cuda):
        raise ValueError("src and dst must be CUDA tensors")
    nr, nw = PROBE_STREAMS[kind] if 0 <= kind < len(PROBE_STREAMS) else (1, 1)
    sb, db = src.numel() * src.element_size(), dst.numel() * dst.element_size()
    if kind in (PROBE_MIX_6R4W, PROBE_MIX_3R1W):
        nbytes = db // nw
        if sb != nr * nbytes or db != nw * nbytes:
            raise ValueError(f"this stream mix takes src of {nr} and dst of {nw} streams of one size")
    else:
        nbytes = db
        if sb != nbytes:
            raise ValueError("src and dst must be of the same size in bytes")
    g = ctypes.c_double()
    _check(lib().wfa_bandwidth_probe(int(kind), int(blocks), ctypes.c_void_p(src.data_ptr()),
                                     ctypes.c_void_p(dst.data_ptr()), nbytes, int(reps),
                                     ctypes.byref(g), _stream_ptr(stream)))
    return g.value


class Server:
    """Continuous-batching solve server (wfa_server) over a device arena of
    `budget_bytes` (its HBM budget) with up to `max_slots` resident solves.
    The server's host thread drives its own HIP stream."""

    def __init__(self, budget_bytes: int, max_slots: int = 64):
        torch = _torch()
        self.stream = torch.cuda.Stream()
        self.arena = torch.empty(int(budget_bytes) + 256, dtype=torch.uint8, device="cuda")
        base = self.arena.data_ptr()
        off = (-base) % 256
        h = ctypes.c_void_p()
        _check(lib().wfa_server_create(ctypes.c_void_p(base + off), int(budget_bytes),
                                       int(max_slots), ctypes.c_void_p(self.stream.cuda_stream),
                                       ctypes.byref(h)))
        self._h = h
        self._keep = {}

    def submit(self, T, *, h, dt, alpha=1.0, kappa=None, u=(0.0, 0.0, 0.0),
               bc=(BC_DIRICHLET,) * 6, bc_value=(0.0,) * 6, precision=F32_IR64,
               tol=1e-10, maxit=5000) -> int:
        """Queue one backward-Euler step of the device field T (shape
        (nz, ny, nx), in place).  Returns the ticket."""
        torch = _torch()
        if isinstance(precision, str):
            precision = PRECISIONS[precision]
        dtype = torch.float32 if precision == F32 else torch.float64
        nz, ny, nx = T.shape
        _dev(T, dtype, nx * ny * nz, "T")
        if kappa is not None:
            kappa = kappa.to(device="cuda", dtype=torch.float32).contiguous()
        c = make_coeffs(h=h, dt=dt, alpha=alpha, kappa=kappa, u=u, bc=bc, bc_value=bc_value,
                        precision=precision)
        torch.cuda.current_stream().synchronize()   # T is ready before the server reads it
        t = ctypes.c_uint64()
        _check(lib().wfa_submit(self._h, nx, ny, nz, ctypes.byref(c), ctypes.c_void_p(T.data_ptr()),
                                float(tol), int(maxit), ctypes.byref(t)))
        self._keep[t.value] = (T, kappa)
        return t.value

    def set_option(self, option: int, value: int):
        """A server option (wfa_server_set_option): OPT_CHECK_EVERY
        (iterations per round), OPT_PERSISTENT (one cooperative launch per
        round), OPT_METHOD, OPT_CG1_MAX_CELLS, OPT_SIZE_CLASS_1..3, or
        OPT_IR_INNER_TOL (inner tolerance x 1e12, for requests submitted
        from then on)."""
        _check(lib().wfa_server_set_option(self._h, int(option), int(value)))

    def submit_problem(self, prob, T, **kw) -> int:
        torch = _torch()
        kappa = torch.from_numpy(prob.kappa) if prob.kappa is not None else None
        return self.submit(T, h=prob.h, dt=prob.dt, alpha=prob.alpha, kappa=kappa, u=prob.u,
                           bc=prob.bc_kind, bc_value=prob.bc_value, **kw)

    def poll(self, ticket: int):
        """(code, info): code is PENDING while the request runs."""
        info = _Info()
        rc = lib().wfa_poll(self._h, int(ticket), ctypes.byref(info))
        if rc == ERR_INVALID:       # unknown ticket (requests never end with this code)
            raise WfaError(rc, last_error())
        if rc != PENDING:
            self._keep.pop(ticket, None)
        return rc, SolveInfo.of(info)

    def drain(self):
        _check(lib().wfa_server_drain(self._h))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _check(lib().wfa_server_destroy(self._h))
            self._h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
