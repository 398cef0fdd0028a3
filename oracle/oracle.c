/*
 * Plain FP64 CPU oracle for the implicit 7-point finite-volume operator and
 * the Krylov solves built on it.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * statement of what the GPU library computes.  Only the test suite, the smoke
 * check and the CPU-baseline leg of the benchmark may load it.  It shares no
 * code, header, table or constant with the HIP library, and it must never be
 * used as a fallback for the product path.
 *
 * What it follows (Woo et al., "Disruptive Changes in Field Equation
 * Modeling", 2022):
 *   - the backward-time centred-space system of Eq. 3 (section 1.1.2): one
 *     unknown per cell, boundary cells held at a constant value, one linear
 *     system A x = b per time step;
 *   - generalised, as stated in the design notes, to a per-cell diffusivity
 *     (harmonic mean on faces), constant-velocity first-order upwind
 *     convection, and per-face Dirichlet or zero-flux boundaries;
 *   - Krylov solution of A x = b (section 1.1.2 names classic CG for the
 *     symmetric case, also in its one-reduction form of Chronopoulos and
 *     Gear (1989); BiCGStab of van der Vorst (1992) covers the
 *     non-symmetric upwind operator).
 *
 * Conventions
 *   - Cell (i,j,k), 0 <= i < nx etc., linear index i + nx*(j + ny*k)
 *     (x fastest).  Cubic cells of side h.
 *   - Faces are numbered 0:x-, 1:x+, 2:y-, 3:y+, 4:z-, 5:z+.
 *   - Outside each boundary face sits one ghost cell at distance h that holds
 *     the boundary value; it is not an unknown.
 *   - All arithmetic is IEEE double.  Dot products are summed sequentially
 *     inside each z-plane, then the plane partials are summed in k order, so
 *     the result does not depend on the number of OpenMP threads.
 *
 * Parity pins (tests/test_oracle_*.py): exact discrete eigenmodes (pure
 * diffusion and upwind), exact steady states of layered media, conservation
 * under zero-flux faces, symmetry of pure diffusion, Kronecker-sum assembly,
 * dense LU solves and library BiCGStab.  The BiCGStab iterates themselves
 * have no printed values in the paper; they are pinned by algebraic
 * invariants of the method (see the tests).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* ---- problem description ------------------------------------------------ */

enum { ORC_DIRICHLET = 0, ORC_ZEROFLUX = 1 };

enum {
  ORC_OK = 0,
  ORC_BREAKDOWN = -4,   /* more than ORC_MAX_RESTARTS restarts              */
  ORC_NOCONV = -5,      /* maxit reached; x holds the last iterate           */
  ORC_NONFINITE = -6    /* NaN/Inf in the data or in a Krylov scalar         */
};

#define ORC_MAX_RESTARTS 3

typedef struct {
  int32_t nx, ny, nz;
  int32_t cell_kappa;     /* 0: constant diffusivity alpha; 1: kappa[cell] */
  double h, dt, alpha;
  const float* kappa;     /* per-cell diffusivity (cell_kappa == 1)        */
  double u[3];            /* constant velocity                             */
  int32_t bc_kind[6];     /* ORC_DIRICHLET or ORC_ZEROFLUX, per face       */
  double bc_value[6];     /* ghost value of each Dirichlet face            */
} orc_problem;

typedef struct {
  int32_t status, iterations, restarts, pad;
  double rel_res_recursive, rel_res_true;
} orc_info;

static long cell_index(const orc_problem* p, int i, int j, int k)
{
  return (long)i + (long)p->nx * ((long)j + (long)p->ny * (long)k);
}

static double cell_diffusivity(const orc_problem* p, long c)
{
  return p->cell_kappa ? (double)p->kappa[c] : p->alpha;
}

/*
 * Row of A for cell (i,j,k), and that cell's boundary contribution to b.
 *
 * Backward Euler on the cell balance (section 1.1.2, Eq. 3, before the scaling
 * by psi): the cell's own coefficient starts at 1 (the time derivative) and
 * each face adds its transport coefficient:
 *   interior face:  diffusive conductance D = dt * kf / h^2 with kf the
 *                   harmonic mean of the two cell diffusivities; upwind flux
 *                   number F = dt * (u . n) / h with n the outward normal.
 *                   Outflow max(F,0) stays on the diagonal, inflow
 *                   max(-F,0) multiplies the upwind neighbour.
 *   Dirichlet face: the ghost at distance h carries the cell's own
 *                   diffusivity; its known value moves to b.
 *   zero-flux face: neither diffusive nor convective flux.
 * off[f] is the coefficient of the neighbour across face f (0 on boundaries).
 */
void orc_row(const orc_problem* p, int i, int j, int k,
             double* diag_out, double off[6], double* bterm_out)
{
  const int step[6][3] = {{-1, 0, 0}, {1, 0, 0}, {0, -1, 0},
                          {0, 1, 0},  {0, 0, -1}, {0, 0, 1}};
  const int n[3] = {p->nx, p->ny, p->nz};
  const int c[3] = {i, j, k};
  const double kp = cell_diffusivity(p, cell_index(p, i, j, k));
  double diag = 1.0;
  double bterm = 0.0;

  for (int f = 0; f < 6; ++f) {
    const int axis = f / 2;
    const double normal = (double)step[f][axis];            /* -1 or +1 */
    const double F = p->dt * (p->u[axis] * normal) / p->h;  /* u.n dt/h */
    int nb[3] = {c[0] + step[f][0], c[1] + step[f][1], c[2] + step[f][2]};
    const int inside = nb[axis] >= 0 && nb[axis] < n[axis];

    off[f] = 0.0;
    if (inside) {
      double kf;
      if (p->cell_kappa) {
        const double kn = (double)p->kappa[cell_index(p, nb[0], nb[1], nb[2])];
        kf = 2.0 * kp * kn / (kp + kn);
      } else {
        kf = p->alpha;
      }
      const double D = p->dt * kf / (p->h * p->h);
      diag += D + fmax(F, 0.0);
      off[f] = -(D + fmax(-F, 0.0));
    } else if (p->bc_kind[f] == ORC_DIRICHLET) {
      const double D = p->dt * kp / (p->h * p->h);
      diag += D + fmax(F, 0.0);
      bterm += (D + fmax(-F, 0.0)) * p->bc_value[f];
    }
    /* zero-flux: no contribution at all */
  }
  *diag_out = diag;
  if (bterm_out) *bterm_out = bterm;
}

/* y = A x, ghosts contributing nothing (they only enter b). */
void orc_apply(const orc_problem* p, const double* x, double* y)
{
  const int nx = p->nx, ny = p->ny, nz = p->nz;
#pragma omp parallel for schedule(static)
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        double diag, off[6];
        orc_row(p, i, j, k, &diag, off, NULL);
        double acc = diag * x[cell_index(p, i, j, k)];
        if (i > 0)      acc += off[0] * x[cell_index(p, i - 1, j, k)];
        if (i < nx - 1) acc += off[1] * x[cell_index(p, i + 1, j, k)];
        if (j > 0)      acc += off[2] * x[cell_index(p, i, j - 1, k)];
        if (j < ny - 1) acc += off[3] * x[cell_index(p, i, j + 1, k)];
        if (k > 0)      acc += off[4] * x[cell_index(p, i, j, k - 1)];
        if (k < nz - 1) acc += off[5] * x[cell_index(p, i, j, k + 1)];
        y[cell_index(p, i, j, k)] = acc;
      }
}

/* Right-hand side of one backward-Euler step: b = T^n + Dirichlet terms. */
void orc_rhs(const orc_problem* p, const double* Tn, double* b)
{
  const int nx = p->nx, ny = p->ny, nz = p->nz;
#pragma omp parallel for schedule(static)
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        double diag, off[6], bterm;
        orc_row(p, i, j, k, &diag, off, &bterm);
        const long c = cell_index(p, i, j, k);
        b[c] = Tn[c] + bterm;
      }
}

/* ---- deterministic vector helpers --------------------------------------- */

static double dot(const orc_problem* p, const double* a, const double* b)
{
  const int nz = p->nz;
  const long plane = (long)p->nx * p->ny;
  double* part = (double*)malloc(sizeof(double) * (size_t)nz);
#pragma omp parallel for schedule(static)
  for (int k = 0; k < nz; ++k) {
    double s = 0.0;
    const long o = (long)k * plane;
    for (long c = 0; c < plane; ++c) s += a[o + c] * b[o + c];
    part[k] = s;
  }
  double total = 0.0;
  for (int k = 0; k < nz; ++k) total += part[k];
  free(part);
  return total;
}

double orc_dot(const orc_problem* p, const double* a, const double* b)
{
  return dot(p, a, b);
}

static long cells(const orc_problem* p)
{
  return (long)p->nx * p->ny * p->nz;
}

/*
 * A shadow residual that needs no storage.  BiCGStab accepts any shadow
 * vector r^ with (r^, r0) != 0 (van der Vorst 1992); r^ = r0 is the usual
 * choice, this one is a fixed pseudo-random field computed from the cell
 * index c alone:
 *   h = PCG hash of c: one step of the 32-bit LCG of PCG
 *       (state = c * 747796405 + 2891336453), then PCG's RXS-M-XS output
 *       permutation (O'Neill 2014; as a hash, Jarzynski and Olano 2020);
 *   r^_c = (h >> 8) * 2^-23 - 1, in [-1, 1), exact in float and double.
 */
static uint32_t pcg_hash32(uint32_t c)
{
  const uint32_t state = c * 747796405u + 2891336453u;
  const uint32_t word = ((state >> ((state >> 28u) + 4u)) ^ state) * 277803737u;
  return (word >> 22u) ^ word;
}

void orc_shadow(long n, double* rh)
{
  for (long c = 0; c < n; ++c)
    rh[c] = (double)(pcg_hash32((uint32_t)c) >> 8) * (1.0 / 8388608.0) - 1.0;
}

static int all_finite(const double* a, long n)
{
  int ok = 1;
#pragma omp parallel for reduction(&& : ok) schedule(static)
  for (long c = 0; c < n; ++c) ok = ok && isfinite(a[c]);
  return ok;
}

/* r = b - A x */
static void residual(const orc_problem* p, const double* b, const double* x,
                     double* r)
{
  const long n = cells(p);
  orc_apply(p, x, r);
#pragma omp parallel for schedule(static)
  for (long c = 0; c < n; ++c) r[c] = b[c] - r[c];
}

/*
 * The operator a Krylov solve iterates with: A itself, or D^{-1} A with D the
 * diagonal of A (left Jacobi scaling; for the paper's constant-coefficient
 * system this is its psi = (1 + 6 omega)^{-1} row scaling, section 1.1.2).
 */
static void krylov_apply(const orc_problem* p, int jacobi, const double* x, double* y)
{
  orc_apply(p, x, y);
  if (!jacobi) return;
  const int nx = p->nx, ny = p->ny, nz = p->nz;
#pragma omp parallel for schedule(static)
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        double diag, off[6];
        orc_row(p, i, j, k, &diag, off, NULL);
        y[cell_index(p, i, j, k)] /= diag;
      }
}

/* b' = D^{-1} b */
static void jacobi_scale(const orc_problem* p, const double* b, double* out)
{
  const int nx = p->nx, ny = p->ny, nz = p->nz;
#pragma omp parallel for schedule(static)
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        double diag, off[6];
        orc_row(p, i, j, k, &diag, off, NULL);
        const long c = cell_index(p, i, j, k);
        out[c] = b[c] / diag;
      }
}

/* r = b - M x for the Krylov operator M */
static void krylov_residual(const orc_problem* p, int jacobi, const double* b, const double* x,
                            double* r)
{
  const long n = cells(p);
  krylov_apply(p, jacobi, x, r);
#pragma omp parallel for schedule(static)
  for (long c = 0; c < n; ++c) r[c] = b[c] - r[c];
}

/* ||b - A x|| / ||b|| (0 when b == 0 and x == 0) */
double orc_true_relres(const orc_problem* p, const double* b, const double* x)
{
  const long n = cells(p);
  double* r = (double*)malloc(sizeof(double) * (size_t)n);
  residual(p, b, x, r);
  const double rn = sqrt(dot(p, r, r));
  const double bn = sqrt(dot(p, b, b));
  free(r);
  return bn > 0.0 ? rn / bn : rn;
}

/*
 * Unpreconditioned BiCGStab (van der Vorst 1992) on A x = b.
 *   x      in: initial guess, out: solution or last iterate
 *   r_out  optional: the recursively updated residual at exit
 *   tol    stop when ||r|| <= tol * ||b|| after a full iteration
 *   maxit  number of full iterations (each = two products with A)
 *   force_bd  n > 0: take sigma of full iteration n as exactly zero (once),
 *          so that the restart path runs on demand; 0: never
 * Shadow residual r^ = r0.  Exactly-zero rho, sigma or omega restarts the
 * method from the true residual b - A x, with r^ reset to that residual (at
 * most ORC_MAX_RESTARTS times).  The iteration count continues across a
 * restart and counts completed iterations only: one that breaks down on rho
 * or sigma, before its update of x, is not counted, while a zero omega comes
 * after the update and its iteration counts.  A non-finite Krylov scalar
 * stops with ORC_NONFINITE.  tt == 0 means s == 0: the half step is the
 * solution.
 */
static int bicgstab_core(const orc_problem* p, int jacobi, const double* b_in, double* x,
                         double tol, int maxit, int force_bd, double* r_out, orc_info* info)
{
  const long n = cells(p);
  const size_t bytes = sizeof(double) * (size_t)n;
  double* bs = NULL;          /* D^{-1} b when scaling */
  const double* b = b_in;
  if (jacobi) {
    bs = (double*)malloc(bytes);
    jacobi_scale(p, b_in, bs);
    b = bs;
  }
  double* r = (double*)malloc(bytes);
  double* rh = (double*)malloc(bytes);
  double* pv = (double*)malloc(bytes);
  double* v = (double*)malloc(bytes);
  double* s = (double*)malloc(bytes);
  double* t = (double*)malloc(bytes);
  int status = ORC_NOCONV, it = 0, restarts = 0;
  double rnorm = 0.0;

  const double bn = sqrt(dot(p, b, b));
  if (!isfinite(bn) || !all_finite(x, n)) {
    status = ORC_NONFINITE;
    goto done;
  }
  if (bn == 0.0) {                       /* the solution of A x = 0 */
    memset(x, 0, bytes);
    memset(r, 0, bytes);
    status = ORC_OK;
    goto done;
  }

  double rho_prev, alpha, omega;
restart:
  krylov_residual(p, jacobi, b, x, r);
  memcpy(rh, r, bytes);
  memset(pv, 0, bytes);
  memset(v, 0, bytes);
  rho_prev = alpha = omega = 1.0;
  rnorm = sqrt(dot(p, r, r));
  if (!isfinite(rnorm)) { status = ORC_NONFINITE; goto done; }
  if (rnorm <= tol * bn) { status = ORC_OK; goto done; }

  while (it < maxit) {
    ++it;
    const double rho = dot(p, rh, r);
    if (!isfinite(rho)) { status = ORC_NONFINITE; goto done; }
    if (rho == 0.0) goto broken;
    const double beta = (rho / rho_prev) * (alpha / omega);
#pragma omp parallel for schedule(static)
    for (long c = 0; c < n; ++c) pv[c] = r[c] + beta * (pv[c] - omega * v[c]);
    krylov_apply(p, jacobi, pv, v);
    double sigma = dot(p, rh, v);
    if (force_bd > 0 && it == force_bd) { sigma = 0.0; force_bd = 0; }
    if (!isfinite(sigma)) { status = ORC_NONFINITE; goto done; }
    if (sigma == 0.0) goto broken;
    alpha = rho / sigma;
#pragma omp parallel for schedule(static)
    for (long c = 0; c < n; ++c) s[c] = r[c] - alpha * v[c];
    krylov_apply(p, jacobi, s, t);
    const double tt = dot(p, t, t);
    const double ts = dot(p, t, s);
    if (!isfinite(tt) || !isfinite(ts)) { status = ORC_NONFINITE; goto done; }
    if (tt == 0.0) {                     /* s == 0: x + alpha p solves it */
#pragma omp parallel for schedule(static)
      for (long c = 0; c < n; ++c) { x[c] += alpha * pv[c]; r[c] = s[c]; }
      rnorm = sqrt(dot(p, r, r));
      status = ORC_OK;
      goto done;
    }
    omega = ts / tt;
#pragma omp parallel for schedule(static)
    for (long c = 0; c < n; ++c) {
      x[c] = x[c] + alpha * pv[c] + omega * s[c];
      r[c] = s[c] - omega * t[c];
    }
    rho_prev = rho;
    rnorm = sqrt(dot(p, r, r));
    if (!isfinite(rnorm)) { status = ORC_NONFINITE; goto done; }
    if (rnorm <= tol * bn) { status = ORC_OK; goto done; }
    if (omega == 0.0) goto do_restart;
    continue;
  broken:
    --it;                                /* ended before its update of x */
  do_restart:
    if (++restarts > ORC_MAX_RESTARTS) { status = ORC_BREAKDOWN; goto done; }
    goto restart;
  }
  status = ORC_NOCONV;

done:
  if (info) {
    info->status = status;
    info->iterations = it;
    info->restarts = restarts;
    info->rel_res_recursive = bn > 0.0 ? rnorm / bn : 0.0;
    info->rel_res_true = (status == ORC_NONFINITE) ? NAN : orc_true_relres(p, b_in, x);
  }
  if (r_out) memcpy(r_out, r, bytes);
  free(r); free(rh); free(pv); free(v); free(s); free(t); free(bs);
  return status;
}

int orc_bicgstab(const orc_problem* p, const double* b, double* x,
                 double tol, int maxit, double* r_out, orc_info* info)
{
  return bicgstab_core(p, 0, b, x, tol, maxit, 0, r_out, info);
}

/* orc_bicgstab with sigma of full iteration force_bd taken as zero (once). */
int orc_bicgstab_forced(const orc_problem* p, const double* b, double* x, double tol,
                        int maxit, int force_bd, double* r_out, orc_info* info)
{
  return bicgstab_core(p, 0, b, x, tol, maxit, force_bd, r_out, info);
}

/*
 * BiCGStab on the left-Jacobi-scaled system D^{-1} A x = D^{-1} b.  The
 * stop test and the recursive residual refer to the scaled system
 * (||D^{-1} r|| <= tol ||D^{-1} b||); rel_res_true is the unscaled one.
 */
int orc_bicgstab_jacobi(const orc_problem* p, const double* b, double* x,
                        double tol, int maxit, double* r_out, orc_info* info)
{
  return bicgstab_core(p, 1, b, x, tol, maxit, 0, r_out, info);
}

/*
 * BiCGStab with two global reductions per iteration (the paper suggests
 * pipelined / reduction-limited Krylov variants, sections 3.2.2 and 5).
 * Same iterates as orc_bicgstab in exact arithmetic, reorganised so that
 * each iteration needs two synchronisation points:
 *   pass 1: apply the previous iteration's update
 *             s = r - alpha v,  r <- s - omega t,  x <- x + alpha p + omega s
 *           then p <- r + beta (p - omega v)  (p = r on the first pass)
 *           v = A p; reduce sigma = (rh, v), and (rh, r), ||r||^2 of the
 *           updated r: the iteration just completed is checked here.
 *   pass 2: s = r - alpha v, t = A s; reduce (t,s), (t,t), (rh,s), (rh,t):
 *           omega = (t,s)/(t,t), and the next rho is predicted from
 *           (rh, s - omega t) = (rh,s) - omega (rh,t) so that beta is known
 *           before the next pass 1.
 * alpha uses the exact rho of pass 1; beta the predicted one.  Breakdown
 * (exact zero rho, sigma or omega) restarts from b - A x as in
 * orc_bicgstab; a zero omega is applied (x += alpha p, r = s) before the
 * restart; tt == 0 (s == 0) ends with x + alpha p.  Iterations are counted
 * when their update has been applied, as in orc_bicgstab.  force_bd = n > 0
 * takes sigma of full iteration n as exactly zero (once); 0: never.  A
 * restart takes r^ = r again for the r0 shadow and keeps the hashed field.
 */
int orc_bicgstab2_shadow(const orc_problem* p, const double* b, double* x, double tol,
                         int maxit, int hashed_shadow, int force_bd, double* r_out,
                         orc_info* info)
{
  const long n = cells(p);
  const size_t bytes = sizeof(double) * (size_t)n;
  double* r = (double*)malloc(bytes);
  double* rh = (double*)malloc(bytes);
  double* pv = (double*)malloc(bytes);
  double* v = (double*)malloc(bytes);
  double* s = (double*)malloc(bytes);
  double* t = (double*)malloc(bytes);
  int status = ORC_NOCONV, it = 0, restarts = 0;
  double rnorm = 0.0;

  const double bn = sqrt(dot(p, b, b));
  if (!isfinite(bn) || !all_finite(x, n)) { status = ORC_NONFINITE; goto done; }
  if (bn == 0.0) {
    memset(x, 0, bytes);
    memset(r, 0, bytes);
    status = ORC_OK;
    goto done;
  }

  double rho, alpha, omega, beta;
  int first, pending_restart, szero;
restart:
  residual(p, b, x, r);
  if (hashed_shadow) orc_shadow(n, rh);
  else memcpy(rh, r, bytes);
  rho = dot(p, rh, r);
  rnorm = sqrt(dot(p, r, r));
  if (!isfinite(rnorm)) { status = ORC_NONFINITE; goto done; }
  if (rnorm <= tol * bn) { status = ORC_OK; goto done; }
  if (it >= maxit) { status = ORC_NOCONV; goto done; }
  alpha = omega = beta = 0.0;
  first = 1;
  pending_restart = 0;
  szero = 0;

  for (;;) {
    /* ---- pass 1 */
    if (first) {
      memcpy(pv, r, bytes);
    } else {
#pragma omp parallel for schedule(static)
      for (long c = 0; c < n; ++c) {
        const double sc = r[c] - alpha * v[c];
        r[c] = sc - omega * t[c];
        x[c] = x[c] + alpha * pv[c] + omega * sc;
        pv[c] = r[c] + beta * (pv[c] - omega * v[c]);
      }
    }
    orc_apply(p, pv, v);
    double sigma = dot(p, rh, v);
    if (!first) {
      ++it;
      const double rho_exact = dot(p, rh, r);
      rnorm = sqrt(dot(p, r, r));
      if (!isfinite(rnorm)) { status = ORC_NONFINITE; goto done; }
      if (szero || rnorm <= tol * bn) { status = ORC_OK; goto done; }
      if (pending_restart) goto do_restart;
      if (it >= maxit) { status = ORC_NOCONV; goto done; }
      if (!isfinite(rho_exact)) { status = ORC_NONFINITE; goto done; }
      if (rho_exact == 0.0) goto do_restart;
      rho = rho_exact;
    }
    if (force_bd > 0 && it + 1 == force_bd) { sigma = 0.0; force_bd = 0; }
    if (!isfinite(sigma)) { status = ORC_NONFINITE; goto done; }
    if (sigma == 0.0) goto do_restart;
    alpha = rho / sigma;
    /* ---- pass 2 */
#pragma omp parallel for schedule(static)
    for (long c = 0; c < n; ++c) s[c] = r[c] - alpha * v[c];
    orc_apply(p, s, t);
    const double ts = dot(p, t, s);
    const double tt = dot(p, t, t);
    const double rs = dot(p, rh, s);
    const double rt = dot(p, rh, t);
    if (!isfinite(ts) || !isfinite(tt) || !isfinite(rs) || !isfinite(rt)) {
      status = ORC_NONFINITE;
      goto done;
    }
    if (tt == 0.0) {
      omega = 0.0;
      szero = 1;
    } else {
      omega = ts / tt;
      if (omega == 0.0) pending_restart = 1;
    }
    if (!szero && !pending_restart) {
      const double rho_pred = rs - omega * rt;
      beta = (rho_pred / rho) * (alpha / omega);
    } else {
      beta = 0.0;
    }
    first = 0;
    continue;
  do_restart:
    if (++restarts > ORC_MAX_RESTARTS) { status = ORC_BREAKDOWN; goto done; }
    goto restart;
  }

done:
  if (info) {
    info->status = status;
    info->iterations = it;
    info->restarts = restarts;
    info->rel_res_recursive = bn > 0.0 ? rnorm / bn : 0.0;
    info->rel_res_true = (status == ORC_NONFINITE) ? NAN : orc_true_relres(p, b, x);
  }
  if (r_out) memcpy(r_out, r, bytes);
  free(r); free(rh); free(pv); free(v); free(s); free(t);
  return status;
}

int orc_bicgstab2(const orc_problem* p, const double* b, double* x, double tol,
                  int maxit, double* r_out, orc_info* info)
{
  return orc_bicgstab2_shadow(p, b, x, tol, maxit, 0, 0, r_out, info);
}

/*
 * Classic conjugate gradients (section 1.1.2: the paper's solver for the
 * symmetric positive-definite pure-diffusion system), unpreconditioned, with
 * the same stopping test as orc_bicgstab.  Each iteration is one product
 * with A and two global reductions.
 */
int orc_cg(const orc_problem* p, const double* b, double* x, double tol,
           int maxit, double* r_out, orc_info* info)
{
  const long n = cells(p);
  const size_t bytes = sizeof(double) * (size_t)n;
  double* r = (double*)malloc(bytes);
  double* d = (double*)malloc(bytes);
  double* q = (double*)malloc(bytes);
  int status = ORC_NOCONV, it = 0;
  double rnorm = 0.0;

  const double bn = sqrt(dot(p, b, b));
  if (!isfinite(bn) || !all_finite(x, n)) { status = ORC_NONFINITE; goto done; }
  if (bn == 0.0) {
    memset(x, 0, bytes);
    memset(r, 0, bytes);
    status = ORC_OK;
    goto done;
  }
  residual(p, b, x, r);
  memcpy(d, r, bytes);
  double rr = dot(p, r, r);
  rnorm = sqrt(rr);
  if (!isfinite(rnorm)) { status = ORC_NONFINITE; goto done; }
  if (rnorm <= tol * bn) { status = ORC_OK; goto done; }
  while (it < maxit) {
    ++it;
    orc_apply(p, d, q);
    const double dq = dot(p, d, q);
    if (!isfinite(dq) || dq <= 0.0) { status = ORC_BREAKDOWN; goto done; }
    const double a = rr / dq;
#pragma omp parallel for schedule(static)
    for (long c = 0; c < n; ++c) { x[c] += a * d[c]; r[c] -= a * q[c]; }
    const double rr_new = dot(p, r, r);
    rnorm = sqrt(rr_new);
    if (!isfinite(rnorm)) { status = ORC_NONFINITE; goto done; }
    if (rnorm <= tol * bn) { status = ORC_OK; goto done; }
    const double beta = rr_new / rr;
#pragma omp parallel for schedule(static)
    for (long c = 0; c < n; ++c) d[c] = r[c] + beta * d[c];
    rr = rr_new;
  }
  status = ORC_NOCONV;
done:
  if (info) {
    info->status = status;
    info->iterations = it;
    info->restarts = 0;
    info->rel_res_recursive = bn > 0.0 ? rnorm / bn : 0.0;
    info->rel_res_true = (status == ORC_NONFINITE) ? NAN : orc_true_relres(p, b, x);
  }
  if (r_out) memcpy(r_out, r, bytes);
  free(r); free(d); free(q);
  return status;
}

/*
 * Conjugate gradients with one global reduction per iteration (Chronopoulos
 * and Gear, 1989).  Besides p it carries s = A p and w = A r by recurrence, so
 * that the two inner products an iteration needs, gamma = (r, r) and
 * delta = (A r, r), are formed together after the only operator product of
 * the iteration, w = A r.  The step length follows from them:
 *   beta = gamma / gamma_old,  alpha = gamma / (delta - beta * gamma / alpha_old),
 * the CG step lengths in exact arithmetic, so the iterates are those of
 * orc_cg up to rounding (the paper's reduction-bound CG, section 3.2.2,
 * needs two reductions per iteration in its textbook form).
 *   r = b - A x, w = A r, gamma = (r, r), delta = (w, r); stop if ||r|| <= tol ||b||
 *   alpha = gamma / delta, p = r, s = w
 *   repeat: x += alpha p; r -= alpha s; w = A r; gamma' = (r, r), delta = (w, r)
 *           stop if ||r|| <= tol ||b||
 *           beta = gamma' / gamma; alpha = gamma' / (delta - beta gamma' / alpha)
 *           p = r + beta p; s = w + beta s; gamma = gamma'
 * A denominator that is not positive (A not positive definite) ends the solve
 * with ORC_BREAKDOWN, as in orc_cg.
 */
int orc_cg1(const orc_problem* p, const double* b, double* x, double tol,
            int maxit, double* r_out, orc_info* info)
{
  const long n = cells(p);
  const size_t bytes = sizeof(double) * (size_t)n;
  double* r = (double*)malloc(bytes);
  double* w = (double*)malloc(bytes);
  double* pv = (double*)malloc(bytes);
  double* s = (double*)malloc(bytes);
  int status = ORC_NOCONV, it = 0;
  double rnorm = 0.0;

  const double bn = sqrt(dot(p, b, b));
  if (!isfinite(bn) || !all_finite(x, n)) { status = ORC_NONFINITE; goto done; }
  if (bn == 0.0) {
    memset(x, 0, bytes);
    memset(r, 0, bytes);
    status = ORC_OK;
    goto done;
  }
  residual(p, b, x, r);
  double gamma = dot(p, r, r);
  rnorm = sqrt(gamma);
  if (!isfinite(rnorm)) { status = ORC_NONFINITE; goto done; }
  if (rnorm <= tol * bn) { status = ORC_OK; goto done; }
  orc_apply(p, r, w);
  double delta = dot(p, w, r);
  if (!isfinite(delta) || delta <= 0.0) { status = ORC_BREAKDOWN; goto done; }
  double alpha = gamma / delta;
  memcpy(pv, r, bytes);
  memcpy(s, w, bytes);
  while (it < maxit) {
    ++it;
#pragma omp parallel for schedule(static)
    for (long c = 0; c < n; ++c) { x[c] += alpha * pv[c]; r[c] -= alpha * s[c]; }
    orc_apply(p, r, w);
    const double gamma_new = dot(p, r, r);
    delta = dot(p, w, r);
    rnorm = sqrt(gamma_new);
    if (!isfinite(rnorm) || !isfinite(delta)) { status = ORC_NONFINITE; goto done; }
    if (rnorm <= tol * bn) { status = ORC_OK; goto done; }
    const double beta = gamma_new / gamma;
    const double denom = delta - beta * gamma_new / alpha;
    if (!(denom > 0.0)) { status = ORC_BREAKDOWN; goto done; }
    alpha = gamma_new / denom;
#pragma omp parallel for schedule(static)
    for (long c = 0; c < n; ++c) { pv[c] = r[c] + beta * pv[c]; s[c] = w[c] + beta * s[c]; }
    gamma = gamma_new;
  }
  status = ORC_NOCONV;
done:
  if (info) {
    info->status = status;
    info->iterations = it;
    info->restarts = 0;
    info->rel_res_recursive = bn > 0.0 ? rnorm / bn : 0.0;
    info->rel_res_true = (status == ORC_NONFINITE) ? NAN : orc_true_relres(p, b, x);
  }
  if (r_out) memcpy(r_out, r, bytes);
  free(r); free(w); free(pv); free(s);
  return status;
}

/*
 * nsteps backward-Euler steps (section 1.1.2): for each step form
 * b = T^n + boundary terms, solve A T^{n+1} = b from the initial guess T^n,
 * and overwrite T.  infos[step] is filled when infos is not NULL.  Stops at
 * the first step that does not return ORC_OK.
 */
int orc_timestep(const orc_problem* p, double* T, int nsteps, double tol,
                 int maxit, orc_info* infos)
{
  const long n = cells(p);
  double* b = (double*)malloc(sizeof(double) * (size_t)n);
  int status = ORC_OK;
  for (int s = 0; s < nsteps; ++s) {
    orc_rhs(p, T, b);
    orc_info info;
    status = orc_bicgstab(p, b, T, tol, maxit, NULL, &info);
    if (infos) infos[s] = info;
    if (status != ORC_OK) break;
  }
  free(b);
  return status;
}

/*
 * Explicit forward-time step (section 1.1.1, Eq. 2), generalised like the
 * implicit operator: each cell gains the net flux through its faces at the
 * old time level,
 *   T'_P = T_P - [ (A[P,P] - 1) T_P + sum_f A[P,N_f] T_N ] + bterm_P,
 * which for a constant diffusivity and Dirichlet faces is Eq. 2 with the
 * ghost cells as the boundary cells held at their value.  nsteps steps in
 * place.
 */
void orc_explicit(const orc_problem* p, double* T, int nsteps)
{
  const int nx = p->nx, ny = p->ny, nz = p->nz;
  const long n = cells(p);
  double* Tn = (double*)malloc(sizeof(double) * (size_t)n);
  for (int step = 0; step < nsteps; ++step) {
    memcpy(Tn, T, sizeof(double) * (size_t)n);
#pragma omp parallel for schedule(static)
    for (int k = 0; k < nz; ++k)
      for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
          double diag, off[6], bterm;
          orc_row(p, i, j, k, &diag, off, &bterm);
          const long c = cell_index(p, i, j, k);
          double flux = (diag - 1.0) * Tn[c];
          if (i > 0)      flux += off[0] * Tn[cell_index(p, i - 1, j, k)];
          if (i < nx - 1) flux += off[1] * Tn[cell_index(p, i + 1, j, k)];
          if (j > 0)      flux += off[2] * Tn[cell_index(p, i, j - 1, k)];
          if (j < ny - 1) flux += off[3] * Tn[cell_index(p, i, j + 1, k)];
          if (k > 0)      flux += off[4] * Tn[cell_index(p, i, j, k - 1)];
          if (k < nz - 1) flux += off[5] * Tn[cell_index(p, i, j, k + 1)];
          T[c] = Tn[c] - flux + bterm;
        }
  }
  free(Tn);
}

int orc_num_threads(void)
{
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void orc_set_num_threads(int n)
{
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}
