/*
 * wfa.h - C-ABI of libwfa.so, an implicit field-equation solver for one
 * AMD Instinct MI355X (gfx950).
 *
 * The problem (Woo et al. 2022, section 1.1.2, Eq. 3, generalised): one
 * backward-Euler step of transport on a uniform Cartesian grid of cubic
 * cells is the sparse linear system A x = b with a 7-point stencil.  The
 * paper's form has diagonal 1 and equal off-diagonals -omega (constant
 * diffusivity, boundary cells held at a constant value); this library
 * also allows a per-cell diffusivity (harmonic mean on each face),
 * constant-velocity first-order upwind convection and per-face Dirichlet or
 * zero-flux boundaries.  Row P of A, for each face f of cell P:
 *   interior face:  D = dt*kf/h^2 (kf harmonic mean of the two cells),
 *                   F = dt*(u.n_f)/h;  A[P,P] += D + max(F,0),
 *                   A[P,N] = -(D + max(-F,0))
 *   Dirichlet face: ghost at distance h with the cell's own diffusivity;
 *                   A[P,P] += D + max(F,0), b[P] += (D + max(-F,0))*value
 *   zero-flux face: no term.
 * and A[P,P] starts at 1.  The system is solved with BiCGStab (van der Vorst
 * 1992), or with conjugate gradients (the paper's solver, section 1.1.2;
 * classic, or reorganised to one reduction per iteration) for the symmetric
 * pure-diffusion case.
 *
 * Conventions
 *   - Fields are dense arrays of nx*ny*nz values, x fastest:
 *     index = i + nx*(j + ny*k) (a torch tensor of shape (nz, ny, nx)).
 *     No pitch, no padding.
 *   - Faces are ordered x-, x+, y-, y+, z-, z+.
 *   - Every data pointer is a caller-owned DEVICE pointer on the current
 *     HIP device.  The library never allocates device memory: the Krylov
 *     workspace and the server arena are caller-provided buffers.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *   - Every function returns a status code (WFA_OK = 0) and records a
 *     message for wfa_last_error().  Arguments are validated before any
 *     launch; nothing is launched when validation fails.  No C++ exception
 *     crosses this interface.
 *   - Functions are thread-safe for distinct grids and servers; calls on one
 *     grid must not overlap.
 */
#ifndef WFA_H
#define WFA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes -------------------------------------------------------- */
#define WFA_OK             0
#define WFA_PENDING        1   /* wfa_poll only: the request is not finished  */
#define WFA_ERR_INVALID   -1   /* bad dimension, null pointer, bad enum,
                                  tol <= 0, maxit < 1, bad option            */
#define WFA_ERR_NOMEM     -2   /* workspace or arena too small               */
#define WFA_ERR_HIP       -3   /* HIP runtime error (text in wfa_last_error) */
#define WFA_ERR_BREAKDOWN -4   /* more than WFA_MAX_RESTARTS BiCGStab restarts,
                                  or a CG step length with a non-positive
                                  denominator (A not positive definite)      */
#define WFA_ERR_NOCONV    -5   /* maxit reached; x holds the last iterate    */
#define WFA_ERR_NONFINITE -6   /* NaN/Inf in the data or a Krylov scalar     */

#define WFA_MAX_RESTARTS 3

/* ---- enums ----------------------------------------------------------------- */
enum {
  WFA_F64 = 0,      /* FP64 vectors and operator                              */
  WFA_F32 = 1,      /* FP32 vectors and operator, FP64 dot accumulation       */
  WFA_F32_IR64 = 2  /* FP64 fields; FP32 inner two-reduction BiCGStab on the
                       Jacobi-scaled system inside FP64 iterative refinement
                       (residual, update and norms in FP64)                  */
};
enum { WFA_COEF_CONST = 0, WFA_COEF_CELL = 1 };
enum { WFA_BC_DIRICHLET = 0, WFA_BC_ZEROFLUX = 1 };
enum {
  WFA_METHOD_BICGSTAB = 0,   /* textbook BiCGStab: 3 reductions per iteration     */
  WFA_METHOD_CG = 1,         /* classic CG (u == 0): 2 reductions per iteration   */
  WFA_METHOD_BICGSTAB2 = 2,  /* BiCGStab reorganised to 2 reductions and 2 passes
                                per iteration (same iterates in exact arithmetic) */
  WFA_METHOD_CG1 = 3         /* CG with 1 reduction and 1 pass per iteration
                                (Chronopoulos-Gear; u == 0; CG's iterates in
                                exact arithmetic)                               */
};

/* ---- problem description --------------------------------------------------- */
typedef struct {
  int32_t mode;          /* WFA_COEF_CONST (alpha) or WFA_COEF_CELL (kappa)    */
  int32_t precision;     /* WFA_F64, WFA_F32 or WFA_F32_IR64                   */
  double  h;             /* cubic cell side, > 0                               */
  double  dt;            /* backward-Euler time step, > 0                      */
  double  alpha;         /* constant diffusivity (CONST), >= 0                 */
  const void* kappa;     /* CELL: device pointer to nx*ny*nz float32 values,
                            > 0; kept by pointer until wfa_grid_destroy        */
  double  u[3];          /* constant velocity; 0 = pure diffusion              */
  int32_t bc[6];         /* WFA_BC_DIRICHLET / WFA_BC_ZEROFLUX per face        */
  double  bc_value[6];   /* Dirichlet ghost values (ignored for zero-flux)     */
} wfa_coeffs;

typedef struct {
  int32_t status;        /* final code of the solve (WFA_OK, NOCONV, ...)      */
  int32_t iterations;    /* full iterations (BiCGStab: 2 operator products;
                            CG: 1)                                            */
  int32_t refinements;   /* WFA_F32_IR64: outer FP64 refinement steps         */
  int32_t restarts;      /* breakdown restarts from the true residual          */
  double  rel_res_recursive; /* recursive ||r|| / ||b|| at exit (FP32_IR64:
                                the inner solver's last value)                */
  double  rel_res_true;  /* ||b - A x|| / ||b|| in FP64, at exit               */
  double  seconds;       /* wall time of the solve (host clock)                */
} wfa_solve_info;

typedef struct wfa_grid wfa_grid;       /* opaque, host-side */
typedef struct wfa_server wfa_server;   /* opaque, host-side */

/* ---- grids ------------------------------------------------------------------ */

/* Bytes of device workspace a grid of this size and precision needs
 * (vectors, per-block partial sums, the device scalar block).  0 when a
 * dimension is < 1. */
size_t wfa_workspace_bytes(int nx, int ny, int nz, int precision);

/* Create a grid descriptor.  `c` is copied (kappa by pointer).  `workspace`
 * is a device buffer of at least wfa_workspace_bytes(...) bytes, 256-byte
 * aligned, owned by the caller and kept alive until wfa_grid_destroy.
 * Errors: WFA_ERR_INVALID (dims < 1, h/dt <= 0, alpha < 0, bad enums, CELL
 * without kappa, null out), WFA_ERR_NOMEM (workspace too small). */
int wfa_grid_create(int nx, int ny, int nz, const wfa_coeffs* c,
                    void* workspace, size_t workspace_bytes, wfa_grid** out);

/* Release the host descriptor (the workspace stays the caller's), with the
 * small pinned host block and the event its first solve set up for reading
 * scalars back (host memory, not device memory). */
int wfa_grid_destroy(wfa_grid* g);

/* y = A x with the ghosts held at zero, i.e. the operator alone (boundary
 * values only enter right-hand sides).  x, y: nx*ny*nz values of the
 * grid's vector type (double for WFA_F64 and WFA_F32_IR64, float for
 * WFA_F32); x and y must not overlap.  Asynchronous on `stream`. */
int wfa_stencil_apply(wfa_grid* g, const void* x, void* y, void* stream);

/* b = T + (Dirichlet boundary terms): the right-hand side of one backward-
 * Euler step from T (section 1.1.2, Eq. 3).  Same types as apply.  Async. */
int wfa_rhs(wfa_grid* g, const void* T, void* b, void* stream);

/* Solve A x = b.  x holds the initial guess on entry and the solution (or,
 * on WFA_ERR_NOCONV, the last iterate) on exit.  Stops at the first full
 * iteration with recursive ||r|| <= tol*||b||; b == 0 gives x = 0.  Exact
 * breakdown (rho, sigma or omega == 0) restarts from b - A x, at most
 * WFA_MAX_RESTARTS times.  `info` may be NULL.  Synchronises `stream`.
 * On a WFA_F32_IR64 grid this is the refinement loop, stopping on the FP64
 * true residual, whose inner FP32 solves use the two-reduction form. */
int wfa_bicgstab_solve(wfa_grid* g, const void* b, void* x, double tol, int maxit,
                       wfa_solve_info* info, void* stream);

/* Classic conjugate gradients on A x = b (valid when A is symmetric
 * positive definite: u == 0).  Same contract as wfa_bicgstab_solve; each
 * iteration is one operator product and two reductions. */
int wfa_cg_solve(wfa_grid* g, const void* b, void* x, double tol, int maxit,
                 wfa_solve_info* info, void* stream);

/* Conjugate gradients reorganised to one global reduction per iteration
 * (Chronopoulos-Gear: w = A r and the pair (r,r), (w,r) give alpha and beta
 * by recurrence; s = A p is carried as a vector).  The update of each
 * iteration is applied on the fly inside the next operator pass, so an
 * iteration is one pass over the grid and one reduction.  The paper solves
 * its symmetric systems with classic CG, two reductions per iteration, and
 * names those reductions the bottleneck at high parallelism (sections 1.1.2,
 * 3.2.2), expecting reorganised Krylov forms to gain more (section 5).  On
 * small grids an iteration here is bound by the same latency.
 * Same iterates as wfa_cg_solve in exact arithmetic.  Same contract as
 * wfa_bicgstab_solve; u == 0 and no Jacobi scaling (WFA_ERR_INVALID
 * otherwise).  A non-positive (p, A p) denominator ends the solve with
 * WFA_ERR_BREAKDOWN.  On a WFA_F32_IR64 grid it is the inner FP32 solve of
 * the refinement, on A itself (BiCGStab's inner solve is Jacobi-scaled); an
 * inner breakdown there ends the inner solve, and the next refinement
 * restarts from the FP64 residual. */
int wfa_cg1_solve(wfa_grid* g, const void* b, void* x, double tol, int maxit,
                  wfa_solve_info* info, void* stream);

/* BiCGStab with two global reductions per iteration: the x and r update of
 * each iteration is applied on the fly inside the next operator pass, and
 * the next rho is predicted from (rh,s) - omega (rh,t) so that beta is
 * known before that pass (the paper points to reduction-limited Krylov
 * variants, sections 3.2.2 and 5).  Same contract as wfa_bicgstab_solve
 * (on a WFA_F32_IR64 grid the two entry points are the same refinement). */
int wfa_bicgstab2_solve(wfa_grid* g, const void* b, void* x, double tol, int maxit,
                        wfa_solve_info* info, void* stream);

/* nsteps backward-Euler steps in place: T holds T^n on entry and T^{n+nsteps}
 * on exit.  Each step forms b = T + boundary terms and solves A T' = b from
 * the initial guess T with the grid's method (BiCGStab unless changed with
 * WFA_OPT_METHOD).  `info` is an array of nsteps records or NULL.  Stops at
 * the first step that fails.  Synchronises `stream`. */
int wfa_timestep(wfa_grid* g, void* T, int nsteps, double tol, int maxit,
                 wfa_solve_info* info, void* stream);

/* nsteps explicit forward-time steps in place (section 1.1.1, Eq. 2,
 * generalised like the operator): T' = T - (A T - T) + boundary terms, i.e.
 * each cell gains the net face flux of the old time level.  Stable only for
 * small steps (Eq. 2: omega = alpha dt / h^2 < 1/6 for pure diffusion); the
 * caller chooses dt.  Uses the grid's workspace as the second time level.
 * With a constant diffusivity (WFA_COEF_CONST) 2 to 4 steps are fused into
 * one pass over memory (temporal blocking, WFA_OPT_EXPLICIT_FUSE); the
 * result is bitwise that of one pass per step.  WFA_F64 and WFA_F32 grids.
 * Asynchronous on `stream`. */
int wfa_explicit_step(wfa_grid* g, void* T, int nsteps, void* stream);

/* FP64 true relative residual ||b - A x|| / ||b|| (FP64 fields only, i.e.
 * WFA_F64 or WFA_F32_IR64 grids).  Synchronises `stream`. */
int wfa_true_residual(wfa_grid* g, const void* b, const void* x, double* rel, void* stream);

/* ---- solve without allocation ----------------------------------------------- */

/* Bytes of the static workspace of wfa_bicgstab_solve_static, per GPU. */
#define WFA_STATIC_WORKSPACE_BYTES (64u << 20)

/* For callers that cannot allocate memory (code that must not call
 * hipMalloc, such as tight serving loops or harnesses that forbid
 * allocation): wfa_bicgstab_solve on the grid wfa_grid_create would make
 * for (nx, ny, nz, c) -- same tiling, same kernels, bitwise the same x and
 * info -- but with no caller workspace.  The workspace is carved out of a
 * static device array of WFA_STATIC_WORKSPACE_BYTES that each GPU the
 * library runs on holds until the process ends, the grid descriptor lives
 * for the call only, and scalars are read back with plain copies and a
 * synchronisation of `stream` instead of a pinned block and an event.  No
 * device or pinned host memory is allocated and no event or stream is
 * created.
 * Limits: wfa_workspace_bytes(nx, ny, nz, c->precision) must not exceed
 * WFA_STATIC_WORKSPACE_BYTES (about 0.9M cells in FP64, 1.3M in
 * WFA_F32_IR64, 1.8M in FP32), else WFA_ERR_NOMEM.  Every call on one GPU
 * uses that GPU's one array, which keeps the last call's contents (each
 * solve initialises what it reads): calls that overlap on one GPU, from
 * several host threads or streams, race and must not be made.  b, x, kappa:
 * caller-owned device buffers as for a grid.  Synchronises `stream`.
 * Errors: those of wfa_grid_create and wfa_bicgstab_solve. */
int wfa_bicgstab_solve_static(int nx, int ny, int nz, const wfa_coeffs* c, const void* b,
                              void* x, double tol, int maxit, wfa_solve_info* info,
                              void* stream);

/* ---- options and instrumentation -------------------------------------------- */
enum {
  WFA_OPT_METHOD = 1,          /* WFA_METHOD_BICGSTAB (default), _CG,
                                  _BICGSTAB2 or _CG1 (used by wfa_timestep;
                                  the *_solve entry points name their method) */
  WFA_OPT_PERSISTENT = 2,      /* 0: one launch per phase (default),
                                  1: one persistent launch per solve chunk,
                                  -1: automatic by grid size                   */
  WFA_OPT_PROFILE = 3,         /* n > 0: time every n-th launch of each
                                  kernel with HIP events (1: every launch;
                                  the count restarts when the option is
                                  set).  While on, the true residual gets its
                                  own pass after the solve, instead of one
                                  queued behind each chunk of iterations.
                                  0 (default): off                             */
  WFA_OPT_FORCE_BREAKDOWN = 4, /* n > 0: treat sigma as exactly 0 at full
                                  iteration n of the next solve (once), to
                                  exercise the restart path from the host      */
  WFA_OPT_CHECK_EVERY = 5,     /* iterations between host convergence checks;
                                  0 = adaptive (default): the first chunk of a
                                  solve takes the iteration count of the grid's
                                  previous converged solve (else 8), later
                                  ones an estimate from the residual history.
                                  Passes queued past convergence exit at
                                  once, so results never depend on this.      */
  WFA_OPT_IR_INNER_TOL = 6,    /* (value / 1e12) = inner relative tolerance of
                                  WFA_F32_IR64; default 1e-4 * 1e12            */
  WFA_OPT_ZCHUNK = 7,          /* z planes per workgroup; 0 = default rule     */
  WFA_OPT_RY = 8,              /* rows per wave of a tile (1, 2 or 4); 0 = default */
  WFA_OPT_JACOBI = 9           /* 1: BiCGStab iterates on D^{-1} A x = D^{-1} b
                                  with D = diag(A), computed in the kernels (the
                                  paper's psi row scaling, section 1.1.2); the
                                  stop test then uses the scaled residual, and
                                  rel_res_true stays the unscaled one.  WFA_F64
                                  and WFA_F32 grids, BiCGStab methods only     */,
  WFA_OPT_GRAPH = 10           /* 1: replay each chunk of iterations between
                                  host checks from captured HIP graphs of 8
                                  iterations (results are bitwise those of
                                  plain launches); 0: plain launches (default);
                                  -1: graphs for grids up to 2^23 cells        */,
  WFA_OPT_EXPLICIT_FUSE = 11   /* explicit steps per pass over memory in
                                  wfa_explicit_step: 1 to 4; 0 = automatic
                                  (with a constant diffusivity 3 in FP32 and
                                  2 in FP64, else 1).  More than 1 needs
                                  WFA_COEF_CONST                               */,
  WFA_OPT_SHADOW = 12,         /* shadow residual of the two-reduction
                                  BiCGStab (also the inner solve of
                                  WFA_F32_IR64): 0 = r0, stored (default); 1 =
                                  a fixed field of the cell index (the 32-bit
                                  PCG hash of the index, top 24 bits mapped to
                                  [-1, 1)), computed where it is used, which
                                  saves one vector stream per pass.  Under
                                  WFA_F32_IR64 a refinement whose inner solve
                                  diverged under 1 without a usable iterate is
                                  repeated with r0, kept for the rest of the
                                  solve                                       */
  WFA_OPT_FORCE_DIVERGE = 13   /* n > 0: the first inner FP32 solve of the
                                  next WFA_F32_IR64 solve counts as diverged at
                                  inner iteration n (once), to exercise the
                                  recovery from the host.  (An inner solve
                                  diverges when ||r|| grows 1000-fold; it is
                                  then repeated once, stopped at the iteration
                                  of its smallest residual, and that
                                  correction is applied.)                      */,
  WFA_OPT_RECOMPUTE_T = 15,    /* two-reduction BiCGStab (also the inner solve
                                  of WFA_F32_IR64): 1 = pass 1 forms t = A s
                                  again from r and v on a two-cell halo, and
                                  pass 2 stores no t, two vector streams fewer
                                  per iteration; the iterates are bitwise
                                  those of 0, t stored by pass 2 and read by
                                  pass 1 (default 0)                          */
  WFA_OPT_CG1_MAX_CELLS = 14,  /* server only: with WFA_OPT_METHOD =
                                  WFA_METHOD_CG1, symmetric requests of more
                                  cells than this keep BiCGStab; 0 = no limit
                                  (default)                                    */
  WFA_OPT_SIZE_CLASS_1 = 16,   /* server only: upper bounds (cells) of the   */
  WFA_OPT_SIZE_CLASS_2 = 17,   /* size classes, each served by its own host  */
  WFA_OPT_SIZE_CLASS_3 = 18    /* thread and HIP stream; 0 = no further class
                                  (defaults 884736, 3511808, 0: three classes,
                                  up to 96^3, 152^3 and above)                */
};
int wfa_grid_set_option(wfa_grid* g, int option, int64_t value);

/* Kernel ids for wfa_kernel_stats. */
enum {
  WFA_K_APPLY = 0, WFA_K_INIT = 1, WFA_K_PHASE_A = 2, WFA_K_PHASE_B = 3,
  WFA_K_PHASE_C = 4, WFA_K_RESIDUAL = 5, WFA_K_PROMOTE = 6, WFA_K_CG_A = 7,
  WFA_K_CG_B = 8, WFA_K_PERSISTENT = 9, WFA_K_PHASE_AC = 10, WFA_K_PHASE_B2 = 11,
  WFA_K_EXPLICIT = 12, WFA_K_EXPLICIT_FUSED = 13, WFA_K_CG1 = 14, WFA_K_COUNT = 15
};
/* With WFA_OPT_PROFILE on: timed launches and their summed event time (ms)
 * of one kernel since the last reset; `bytes` = algorithmic HBM bytes per launch
 * (the streams the kernel must read and write once).  reset != 0 clears. */
int wfa_kernel_stats(wfa_grid* g, int kernel, int64_t* launches, double* ms,
                     double* bytes_per_launch, int reset);

/* Tile shape the grid uses: x cells, y cells, z planes per workgroup, and
 * the number of workgroups of one phase launch. */
int wfa_grid_tiling(wfa_grid* g, int* tx, int* ty, int* zc, int* blocks);

/* Address of one of the grid's Krylov vectors inside the caller's workspace,
 * for inspection (tests, debugging); nothing is copied.  The vector holds
 * nx*ny*nz values of the grid's Krylov type (double on WFA_F64 grids, float
 * on WFA_F32 and WFA_F32_IR64 grids, whose Krylov vectors are the inner FP32
 * solve's) and whatever the last solve left there.  The double-buffered
 * pairs are those of the solve that wrote them last: BiCGStab (either
 * organisation) writes p and v = A p into (P0, V0) or (P1, V1), alternately;
 * CG with one reduction writes r and w = A r into (R, V0) or (R1, V1).
 * Errors: WFA_ERR_INVALID (null grid or ptr, unknown vector). */
enum {
  WFA_VEC_R = 0, WFA_VEC_RHAT = 1, WFA_VEC_T = 2, WFA_VEC_P0 = 3, WFA_VEC_P1 = 4,
  WFA_VEC_V0 = 5, WFA_VEC_V1 = 6, WFA_VEC_B = 7, WFA_VEC_R1 = 8, WFA_VEC_COUNT = 9
};
int wfa_grid_vector(wfa_grid* g, int which, void** ptr);

/* ---- tile-shape autotuner ------------------------------------------------------
 * The stencil passes march 64-cell-wide tiles of 4 x (rows per wave) rows
 * along z, zc planes per workgroup.  wfa_autotune times `iters` iterations
 * of `method` (WFA_METHOD_*) on this grid for the default rule and for every
 * (rows per wave in {1, 2, 4}) x (zc in {1, 2, 4, ..., 64}, zc <= nz), keeps
 * the fastest, applies it to the grid, and records it in a process-wide
 * table under (nx, ny, nz, precision, coefficient mode).  Grids created
 * afterwards with that key start with the recorded tiling, so a grid's
 * tiling -- and with it the order of its reductions -- depends on its key
 * only.  Each candidate's cost per iteration is the time of a 2*iters solve
 * minus that of an iters solve, over the iterations they differ by; a solve
 * that its numbers stop early (non-finite values or breakdown, as a
 * diverging FP32 solve may) is timed over the iterations it ran.  x and b
 * are caller-owned device fields of the grid's vector type (FP64 for
 * WFA_F32_IR64) and are overwritten.  Synchronises `stream`.
 * The solver options of the grid are left as they were. */
typedef struct {
  int32_t ry, zc;              /* chosen rows per wave and z planes per workgroup */
  int32_t candidates, pad;     /* distinct tile shapes timed                      */
  double us_per_iter;          /* chosen shape, microseconds per iteration        */
  double us_per_iter_default;  /* the default rule's shape                        */
} wfa_tune_result;
int wfa_autotune(wfa_grid* g, int method, void* x, void* b, int iters, wfa_tune_result* out,
                 void* stream);
/* The table as text, one entry per line:
 *   nx ny nz precision mode rows_per_wave z_planes us_per_iter
 * wfa_tune_load merges a file into the table (its entries win) and rejects
 * a malformed file as a whole (WFA_ERR_INVALID).  No GPU work. */
int wfa_tune_save(const char* path);
int wfa_tune_load(const char* path);
int wfa_tune_clear(void);

/* Achievable HBM bandwidth probe: copies `bytes` (multiple of 16) from src
 * to dst `reps` times on `stream` and returns GB/s (read + write bytes).
 * The same as wfa_bandwidth_probe(WFA_PROBE_COPY, 0, ...). */
int wfa_stream_probe(const void* src, void* dst, size_t bytes, int reps, double* gbps,
                     void* stream);

/* Bandwidth ceilings of the part, the measured reference for the section
 * 3.1.3 effective-bandwidth figures: `reps` launches (after one untimed
 * launch) of one access pattern over `bytes` with `blocks` workgroups of 256
 * threads (0 = 8192), timed with events on `stream`; *gbps = bytes moved
 * (read + written) per second / 1e9.  Synchronises `stream`.
 *   WFA_PROBE_COPY        dst = src, nontemporal loads and stores, 16 B per lane
 *   WFA_PROBE_COPY_PLAIN  the same with plain loads and stores
 *   WFA_PROBE_COPY32      nontemporal, 32 contiguous bytes per lane
 *   WFA_PROBE_READ        reads src only (nontemporal); may write the first
 *                         4096 bytes of dst
 *   WFA_PROBE_WRITE       writes dst only (nontemporal); src unused
 *   WFA_PROBE_MIX_6R4W    the fused update pass's stream mix: reads six
 *                         streams and writes four, `bytes` each; src holds
 *                         the six back to back (6 * bytes), dst the four
 *                         (4 * bytes); written stream k is the xor of read
 *                         streams k and k + 4 (k < 2) or stream k alone
 *   WFA_PROBE_MIX_3R1W    the second pass's mix: reads three streams (src,
 *                         3 * bytes) and writes their xor (dst, bytes)
 * bytes: a multiple of 16 (32 for COPY32), at least 4096 for READ, at most
 * 2^40; src and dst: device buffers of `bytes` bytes (the stream mixes: as
 * above), 16-byte (COPY32: 32-byte) aligned.
 * Errors: WFA_ERR_INVALID (bad kind, size, alignment or null pointer),
 * WFA_ERR_HIP. */
enum {
  WFA_PROBE_COPY = 0, WFA_PROBE_COPY_PLAIN = 1, WFA_PROBE_COPY32 = 2, WFA_PROBE_READ = 3,
  WFA_PROBE_WRITE = 4, WFA_PROBE_MIX_6R4W = 5, WFA_PROBE_MIX_3R1W = 6
};
int wfa_bandwidth_probe(int kind, int blocks, const void* src, void* dst, size_t bytes, int reps,
                        double* gbps, void* stream);

/* ---- serving ------------------------------------------------------------------ */

/* A server owns a caller-provided device arena of arena_bytes (its HBM
 * budget).  Requests are split by cell count into up to four size classes
 * (WFA_OPT_SIZE_CLASS_*); each class has its own host thread, HIP stream
 * and up to max_slots resident solves, so small requests' rounds do not
 * wait for large requests' passes.  Within a class, requests are admitted
 * in arrival order as arena space and slots free up (a request first in
 * line that does not fit lets up to 16 later ones that fit go ahead); all
 * resident solves of a class advance together in batched launches
 * (continuous batching); a request finishes independently of the others
 * and its result does not depend on which requests ran beside it or in
 * which class.  Every request is solved with the
 * two-reduction BiCGStab and the index-hashed shadow residual, as
 * wfa_timestep does with WFA_OPT_METHOD = WFA_METHOD_BICGSTAB2 and
 * WFA_OPT_SHADOW = 1; WFA_F32_IR64 requests run it as the inner solve of
 * refinement, as wfa_timestep does (including its fall-back to r^ = r0
 * for a refinement whose inner solve diverged without a usable
 * iterate).  The first class's thread drives
 * the GPU on `stream`; the others on streams the server creates (default
 * priority).  Precision of every request: c->precision.  The server also
 * holds a pinned host mirror of its slot tables and scalars, one event per
 * class and the class streams, freed by wfa_server_destroy.
 * Errors: WFA_ERR_INVALID, WFA_ERR_NOMEM (arena smaller than its tables),
 * WFA_ERR_HIP (the pinned mirror, an event or a stream). */
int wfa_server_create(void* arena, size_t arena_bytes, int max_slots, void* stream,
                      wfa_server** out);

/* Server options, applied from the next round on:
 *   WFA_OPT_CHECK_EVERY  iterations per round between the worker's reads of
 *                        the slots' scalars, 1..1024 (default 4);
 *   WFA_OPT_METHOD       WFA_METHOD_BICGSTAB2 (default) or WFA_METHOD_CG1:
 *                        requests submitted afterwards with u == 0 iterate
 *                        with CG with one reduction (the inner solve of
 *                        WFA_F32_IR64 requests, as wfa_cg1_solve on such a
 *                        grid), two CG iterations per BiCGStab iteration of
 *                        a round; other requests keep BiCGStab.  A round with
 *                        a CG request resident makes one launch per pass
 *                        whatever WFA_OPT_PERSISTENT says;
 *   WFA_OPT_CG1_MAX_CELLS  0 (default) or the largest request (in cells)
 *                        that WFA_METHOD_CG1 applies to: latency-bound small
 *                        grids gain from CG's one pass per iteration, while
 *                        bandwidth-bound large ones move fewer bytes with
 *                        BiCGStab;
 *   WFA_OPT_PERSISTENT   1: each round is one cooperative launch per
 *                        precision, with grid barriers in place of the
 *                        per-pass kernel boundaries (bitwise the same
 *                        results); 0: one launch per pass (default).  A
 *                        barrier wait that times out fails the server
 *                        (WFA_ERR_HIP) instead of hanging.  While it is on,
 *                        requests submitted go to the first size class,
 *                        which alone runs cooperative rounds;
 *   WFA_OPT_SIZE_CLASS_1..3  upper cell-count bound of size classes 1..3
 *                        (class 4 takes the rest); 0 ends the list.
 *                        Non-zero bounds must increase.  A request's class
 *                        is fixed when it is submitted;
 *   WFA_OPT_IR_INNER_TOL (value / 1e12) = relative tolerance of the FP32
 *                        inner solves of WFA_F32_IR64 requests submitted
 *                        from then on, in (0, 1); default 1e-4 * 1e12.
 * Errors: WFA_ERR_INVALID (null server, unknown option, value out of range). */
int wfa_server_set_option(wfa_server* sv, int option, int64_t value);

/* Queue one backward-Euler step of T (device, nx*ny*nz, in/out; the
 * caller keeps it, and kappa, alive until wfa_poll reports completion).
 * WFA_ERR_NOMEM if the request can never fit the arena. */
int wfa_submit(wfa_server* sv, int nx, int ny, int nz, const wfa_coeffs* c, void* T,
               double tol, int maxit, uint64_t* ticket);

/* WFA_PENDING while queued or running, otherwise the request's final code
 * (info filled, seconds = completion - submission).  A ticket may be polled
 * again after completion; unknown tickets give WFA_ERR_INVALID. */
int wfa_poll(wfa_server* sv, uint64_t ticket, wfa_solve_info* info);

/* Block until every submitted request has finished. */
int wfa_server_drain(wfa_server* sv);

/* Wait for in-flight work, stop the host thread and free the descriptor. */
int wfa_server_destroy(wfa_server* sv);

/* Thread-local message of the last failing call on this thread. */
const char* wfa_last_error(void);

/* Library version string. */
const char* wfa_version(void);

#ifdef __cplusplus
}
#endif
#endif /* WFA_H */
