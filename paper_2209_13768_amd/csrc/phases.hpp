// Phase policies of the z-marching engine (march_tile) and the finalizers
// that turn each pass's global sums into the next Krylov scalars.  Shared by
// the single-solve kernels and the batched serving kernels, so that a solve
// computes exactly the same values in either.
#pragma once
#include <math.h>

#include "device.hpp"

namespace wfa {

// Loads and stores of values no neighbouring tile reads back soon
// (epilogue inputs, pass outputs) carry a streaming (non-temporal) hint so
// that they do not displace the halo rows and planes the L2 is holding.
// Measured 2-4% faster per iteration; WFA_NO_STREAM_HINTS turns it off.
#ifndef WFA_NO_STREAM_HINTS
template <typename T> __device__ __forceinline__ T ld_once(const T* p) { return __builtin_nontemporal_load(p); }
template <typename T> __device__ __forceinline__ void st_once(T* p, T v) { __builtin_nontemporal_store(v, p); }
#else
template <typename T> __device__ __forceinline__ T ld_once(const T* p) { return *p; }
template <typename T> __device__ __forceinline__ void st_once(T* p, T v) { *p = v; }
#endif

// Policies whose own cells stage like halo cells (no side effects).
#define WFA_PLAIN_OWN_STAGE                                                     \
  using ORaw = Raw;                                                            \
  __device__ Raw fetch_own(size_t i) const { return fetch(i); }                \
  template <int N>                                                             \
  __device__ St combine_own(const Raw& q, size_t, double (&)[N]) const {       \
    return combine(q);                                                         \
  }                                                                            \
  __device__ auto value_own(const Raw& q) const { return val(combine(q)); }

// ============================================================================
// staged Krylov updates
// ============================================================================
// A staged value is computed once for the cell that stores it (combine_own)
// and again by every neighbouring tile that reads the cell on its halo
// (combine).  Both copies must round the same way, or the operator would be
// applied to a vector that differs from the stored one at tile edges.  The
// updates are therefore written with explicit fused multiply-adds, with
// contraction off, so that no call site is left to the compiler's choice.
// y - a x
template <typename T>
__device__ __forceinline__ T minus_ax(T y, T a, T x) {
#pragma clang fp contract(off)
  return fma_t(-a, x, y);
}
// p' = r' + beta (p - omega v)
template <typename T>
__device__ __forceinline__ T next_p(T rn, T p, T v, T beta, T omega) {
#pragma clang fp contract(off)
  return fma_t(beta, minus_ax(p, omega, v), rn);
}
// x' = x + alpha p + omega s, summed in that order
template <typename T>
__device__ __forceinline__ T next_x(T x, T p, T s, T alpha, T omega) {
#pragma clang fp contract(off)
  return fma_t(omega, s, fma_t(alpha, p, x));
}

// ============================================================================
// finalizers (thread 0 of the last workgroup)
// ============================================================================
__device__ __forceinline__ bool fin_ok(double v) { return isfinite(v); }

struct FinInit {
  Scalars* sc;
  __device__ void operator()(const double (&s)[3]) const {
    const double bb = s[0], rr = s[1], rho = s[2];
    sc->bb = bb; sc->rr = rr; sc->rr0 = rr;
    sc->rho = rho; sc->rho_prev = 1.0; sc->alpha = 1.0; sc->omega = 1.0; sc->beta = 0.0;
    sc->first = 1; sc->restart = 0; sc->szero = 0; sc->restart_pending = 0;
    sc->rr_min = rr; sc->it_min = 0; sc->stage = 0;
    if (!fin_ok(bb) || !fin_ok(rr) || !fin_ok(rho)) sc->status = ST_NONFINITE;
    else if (bb == 0.0) sc->status = ST_BZERO;
    else if (sqrt(rr) <= sc->tol * sqrt(bb)) sc->status = ST_CONV;
    else if (sc->iter >= sc->maxit) sc->status = ST_NOCONV;
    else sc->status = ST_RUN;
  }
};

struct FinA {
  Scalars* sc;
  __device__ void operator()(const double (&s)[1]) const {
    double sigma = s[0];
    if (sc->force_bd > 0 && sc->iter + 1 == sc->force_bd) { sigma = 0.0; sc->force_bd = 0; }
    sc->sigma = sigma;
    if (!fin_ok(sigma)) sc->status = ST_NONFINITE;
    else if (sigma == 0.0) sc->restart = 1;
    else sc->alpha = sc->rho / sigma;
  }
};

struct FinB {
  Scalars* sc;
  __device__ void operator()(const double (&s)[2]) const {
    const double ts = s[0], tt = s[1];
    sc->ts = ts; sc->tt = tt;
    if (!fin_ok(ts) || !fin_ok(tt)) sc->status = ST_NONFINITE;
    else if (tt == 0.0) { sc->szero = 1; sc->omega = 0.0; }
    else sc->omega = ts / tt;
  }
};

struct FinC {
  Scalars* sc;
  __device__ void operator()(const double (&s)[2]) const {
    const double rho_new = s[0], rr = s[1];
    sc->iter += 1;
    sc->rr = rr;
    sc->x_zero = 0;
    if (rr < sc->rr_min) { sc->rr_min = rr; sc->it_min = sc->iter; }
    if (sc->szero) sc->status = ST_CONV;
    else if (!fin_ok(rr)) sc->status = ST_NONFINITE;
    else if (sqrt(rr) <= sc->tol * sqrt(sc->bb)) sc->status = ST_CONV;
    else if ((sc->guard > 0.0 && rr > sc->guard * sc->rr0) || sc->iter == sc->force_div) {
      sc->status = ST_NOCONV;
      sc->diverged = 1;
    }
    else if (sc->omega == 0.0) sc->restart = 1;
    else if (sc->iter >= sc->maxit) sc->status = ST_NOCONV;
    else if (!fin_ok(rho_new)) sc->status = ST_NONFINITE;
    else if (rho_new == 0.0) sc->restart = 1;
    else {
      sc->beta = (rho_new / sc->rho) * (sc->alpha / sc->omega);
      sc->rho_prev = sc->rho;
      sc->rho = rho_new;
      sc->first = 0;
    }
  }
};

struct FinCgA {
  Scalars* sc;
  __device__ void operator()(const double (&s)[1]) const {
    const double dq = s[0];
    sc->sigma = dq;
    if (!fin_ok(dq)) sc->status = ST_NONFINITE;
    else if (dq <= 0.0) sc->status = ST_BREAKDOWN;
    else sc->alpha = sc->rho / dq;
  }
};

struct FinCgB {
  Scalars* sc;
  __device__ void operator()(const double (&s)[1]) const {
    const double rr = s[0];
    sc->iter += 1;
    sc->rr = rr;
    if (!fin_ok(rr)) sc->status = ST_NONFINITE;
    else if (sqrt(rr) <= sc->tol * sqrt(sc->bb)) sc->status = ST_CONV;
    else if (sc->iter >= sc->maxit) sc->status = ST_NOCONV;
    else {
      sc->beta = rr / sc->rho;
      sc->rho = rr;
      sc->first = 0;
    }
  }
};

// CG with one reduction per iteration (Chronopoulos-Gear), after its pass:
// gamma = (r, r), delta = (A r, r) of the iterate the pass produced.  The
// pass of stage 0 only formed w0 = A r0: alpha0 = gamma / delta.  Later
// passes apply one iteration each: convergence and limits on gamma, then
// beta = gamma / gamma_old and alpha = gamma / (delta - beta gamma / alpha_old)
// for the update the next pass applies.  A step denominator that is not
// positive means A is not positive definite: ST_BREAKDOWN, as for CG.
struct FinCg1 {
  Scalars* sc;
  __device__ void operator()(const double (&s)[2]) const {
    const double gamma = s[0], delta = s[1];
    sc->sigma = delta;
    if (!fin_ok(gamma) || !fin_ok(delta)) { sc->status = ST_NONFINITE; return; }
    if (sc->stage == 0) {
      if (!(delta > 0.0)) { sc->status = ST_BREAKDOWN; return; }
      sc->alpha = gamma / delta;
      sc->beta = 0.0;
      sc->rho = gamma;
      sc->stage = 1;
      return;
    }
    sc->iter += 1;
    sc->rr = gamma;
    sc->x_zero = 0;
    if (gamma < sc->rr_min) { sc->rr_min = gamma; sc->it_min = sc->iter; }
    if (sqrt(gamma) <= sc->tol * sqrt(sc->bb)) { sc->status = ST_CONV; return; }
    // the divergence guard of an inner refinement solve (as for BiCGStab)
    if ((sc->guard > 0.0 && gamma > sc->guard * sc->rr0) || sc->iter == sc->force_div) {
      sc->status = ST_NOCONV;
      sc->diverged = 1;
      return;
    }
    if (sc->iter >= sc->maxit) { sc->status = ST_NOCONV; return; }
    const double beta = gamma / sc->rho;
    const double denom = delta - beta * gamma / sc->alpha;
    if (!(denom > 0.0)) { sc->status = ST_BREAKDOWN; return; }
    sc->alpha = gamma / denom;
    sc->beta = beta;
    sc->rho = gamma;
    sc->stage = 2;
  }
};

// True residual: (r,r), (b,b) into sc.  IR mode: also set up the inner solve.
struct FinResid {
  Scalars* sc;
  Scalars* inner;  // may be null
  __device__ void operator()(const double (&s)[4]) const {
    const double rr = s[0], bb = s[1], r2 = s[2], rho = s[3];
    sc->rr = rr; sc->bb = bb;
    if (!fin_ok(rr) || !fin_ok(bb)) sc->status = ST_NONFINITE;
    else if (bb == 0.0) sc->status = ST_BZERO;
    else if (sqrt(rr) <= sc->tol * sqrt(bb)) sc->status = ST_CONV;
    else sc->status = ST_RUN;
    if (inner) {
      inner->bb = r2; inner->rr = r2; inner->rr0 = r2;
      inner->rho = rho; inner->rho_prev = 1.0; inner->alpha = 1.0; inner->omega = 1.0;
      inner->beta = 0.0; inner->first = 1; inner->restart = 0; inner->szero = 0;
      inner->x_zero = 1; inner->iter = 0; inner->diverged = 0;
      inner->rr_min = r2; inner->it_min = 0; inner->stage = 0;
      if (sc->status != ST_RUN) inner->status = ST_CONV;
      else if (!fin_ok(r2) || !fin_ok(rho)) inner->status = ST_NONFINITE;
      else if (r2 == 0.0) inner->status = ST_CONV;
      else {
        inner->status = ST_RUN;
        if (rho == 0.0) inner->restart = 1;  // (r^, r0) = 0: breakdown at the start
      }
    }
  }
};

struct FinNone {
  __device__ void operator()(const double (&)[1]) const {}
};

// ============================================================================
// stencil phase policies (see march_tile)
// ============================================================================
template <typename T>
struct PhApply {
  static constexpr int NV = 1;
  static constexpr int PD = 1;
  using St = T;
  static __device__ __forceinline__ T val(T u) { return u; }
  const T* __restrict__ x;
  T* __restrict__ y;
  struct Raw { T x; };
  struct ERaw {};
  WFA_PLAIN_OWN_STAGE
  __device__ void bind(const Scalars*) {}
  __device__ Raw fetch(size_t i) const { return {x[i]}; }
  __device__ T combine(const Raw& r) const { return r.x; }
  __device__ ERaw efetch(size_t) const { return {}; }
  __device__ void epilogue(size_t i, T, T Au, T, uint32_t, const ERaw&, T dg, double (&)[NV]) const {
    y[i] = Au;
  }
};

template <typename T, bool CELL>
struct PhRhs {
  static constexpr int NV = 1;
  static constexpr int PD = 1;
  using St = T;
  static __device__ __forceinline__ T val(T u) { return u; }
  Op<T> op;
  const T* __restrict__ x;
  T* __restrict__ b;
  struct Raw { T x; };
  struct ERaw {};
  WFA_PLAIN_OWN_STAGE
  __device__ void bind(const Scalars*) {}
  __device__ Raw fetch(size_t i) const { return {x[i]}; }
  __device__ T combine(const Raw& r) const { return r.x; }
  __device__ ERaw efetch(size_t) const { return {}; }
  __device__ void epilogue(size_t i, T u, T, T kP, uint32_t ins, const ERaw&, T dg,
                           double (&)[NV]) const {
    b[i] = u + cell_bterm<T, CELL>(op, kP, ins);
  }
};

// Explicit forward-time step (the paper's Eq. 2, generalised like the
// operator): y = x - (A x - x) + boundary terms.
template <typename T, bool CELL>
struct PhExplicit {
  static constexpr int NV = 1;
  static constexpr int PD = 2;
  using St = T;
  static __device__ __forceinline__ T val(T u) { return u; }
  Op<T> op;
  const T* __restrict__ x;
  T* __restrict__ y;
  struct Raw { T x; };
  struct ERaw {};
  WFA_PLAIN_OWN_STAGE
  __device__ void bind(const Scalars*) {}
  __device__ Raw fetch(size_t i) const { return {x[i]}; }
  __device__ T combine(const Raw& r) const { return r.x; }
  __device__ ERaw efetch(size_t) const { return {}; }
  __device__ void epilogue(size_t i, T u, T Au, T kP, uint32_t ins, const ERaw&, T dg,
                           double (&)[NV]) const {
    st_once(y + i, explicit_update(u, Au, cell_bterm<T, CELL>(op, kP, ins)));
  }
};

template <typename T, bool CELL, bool FORM_B>
struct PhInit {
  static constexpr int NV = 3;
  static constexpr int PD = 1;
  using St = T;
  static __device__ __forceinline__ T val(T u) { return u; }
  Op<T> op;
  const T* __restrict__ x;
  const T* __restrict__ b_in;
  T* __restrict__ b_out;
  T* __restrict__ r;
  T* __restrict__ rh;
  int hashed;      // shadow residual from the cell index (not stored)
  struct Raw { T x; };
  struct ERaw { T b; };
  WFA_PLAIN_OWN_STAGE
  __device__ void bind(const Scalars*) {}
  __device__ Raw fetch(size_t i) const { return {x[i]}; }
  __device__ T combine(const Raw& q) const { return q.x; }
  __device__ ERaw efetch(size_t i) const {
    if (FORM_B) return {T(0)};
    return {b_in[i]};
  }
  __device__ void epilogue(size_t i, T u, T Au, T kP, uint32_t ins, const ERaw& e, T dg,
                           double (&acc)[NV]) const {
    const T b0 = FORM_B ? u + cell_bterm<T, CELL>(op, kP, ins) : e.b;
    const T bv = op.jac ? b0 * pos_rcp(dg) : b0;   // D^{-1} b under Jacobi scaling
    const T rv = bv - Au;
    if (FORM_B) b_out[i] = b0;
    r[i] = rv;
    T sh = rv;
    if (hashed) sh = hashed_shadow<T>(i);
    else rh[i] = rv;
    dot_acc(acc[0], (double)bv, (double)bv);
    dot_acc(acc[1], (double)rv, (double)rv);
    dot_acc(acc[2], (double)sh, (double)rv);
  }
};

// Staged value of an own cell that also carries the shadow residual the
// epilogue's dot product needs.
template <typename T>
struct StageP {
  T p;
  T rh;
};

template <typename T>
struct PhA {
  static constexpr int NV = 1;
  static constexpr int PD = 1;
  using St = StageP<T>;
  static __device__ __forceinline__ T val(const St& u) { return u.p; }
  static __device__ __forceinline__ T val(T u) { return u; }
  const T* __restrict__ r;
  const T* __restrict__ p;
  const T* __restrict__ v;
  T* __restrict__ p_out;
  T* __restrict__ v_out;
  const T* __restrict__ rh;
  T beta, omega;
  int first;
  struct Raw { T r, p, v; };
  struct ORaw { T r, p, v, rh; };
  struct ERaw {};
  __device__ void bind(const Scalars* sc) {
    beta = (T)sc->beta;
    omega = (T)sc->omega;
    first = sc->first;
  }
  __device__ Raw fetch(size_t i) const {
    if (first) return {r[i], T(0), T(0)};
    return {r[i], p[i], v[i]};
  }
  __device__ T combine(const Raw& q) const {
    return first ? q.r : next_p(q.r, q.p, q.v, beta, omega);
  }
  __device__ ORaw fetch_own(size_t i) const {
    if (first) return {r[i], T(0), T(0), ld_once(rh + i)};
    return {r[i], p[i], v[i], ld_once(rh + i)};
  }
  // p' is stored as soon as it is staged
  __device__ St combine_own(const ORaw& q, size_t i, double (&)[NV]) const {
    const T pn = combine(Raw{q.r, q.p, q.v});
    st_once(p_out + i, pn);
    return {pn, q.rh};
  }
  __device__ T value_own(const ORaw& q) const { return combine(Raw{q.r, q.p, q.v}); }
  __device__ ERaw efetch(size_t) const { return {}; }
  __device__ void epilogue(size_t i, const St& u, T Au, T, uint32_t, const ERaw&, T dg,
                           double (&acc)[NV]) const {
    st_once(v_out + i, Au);
    dot_acc(acc[0], (double)u.rh, (double)Au);
  }
};

template <typename T>
struct PhB {
  static constexpr int NV = 2;
  static constexpr int PD = 2;
  using St = T;
  static __device__ __forceinline__ T val(T u) { return u; }
  const T* __restrict__ r;
  const T* __restrict__ v;
  T* __restrict__ t;
  T alpha;
  struct Raw { T r, v; };
  struct ERaw {};
  WFA_PLAIN_OWN_STAGE
  __device__ void bind(const Scalars* sc) { alpha = (T)sc->alpha; }
  __device__ Raw fetch(size_t i) const { return {r[i], v[i]}; }
  __device__ T combine(const Raw& q) const { return minus_ax(q.r, alpha, q.v); }
  __device__ ERaw efetch(size_t) const { return {}; }
  __device__ void epilogue(size_t i, T s, T Au, T, uint32_t, const ERaw&, T dg,
                           double (&acc)[NV]) const {
    st_once(t + i, Au);
    dot_acc(acc[0], (double)Au, (double)s);
    dot_acc(acc[1], (double)Au, (double)Au);
  }
};

template <typename T>
struct PhCgA {
  static constexpr int NV = 1;
  static constexpr int PD = 1;
  using St = T;
  static __device__ __forceinline__ T val(T u) { return u; }
  const T* __restrict__ r;
  const T* __restrict__ d;
  T* __restrict__ d_out;
  T* __restrict__ q;
  T beta;
  int first;
  struct Raw { T r, d; };
  struct ERaw {};
  WFA_PLAIN_OWN_STAGE
  __device__ void bind(const Scalars* sc) {
    beta = (T)sc->beta;
    first = sc->first;
  }
  __device__ Raw fetch(size_t i) const {
    if (first) return {r[i], T(0)};
    return {r[i], d[i]};
  }
  __device__ T combine(const Raw& z) const { return first ? z.r : fma_t(beta, z.d, z.r); }
  __device__ ERaw efetch(size_t) const { return {}; }
  __device__ void epilogue(size_t i, T u, T Au, T, uint32_t, const ERaw&, T dg,
                           double (&acc)[NV]) const {
    d_out[i] = u;
    q[i] = Au;
    dot_acc(acc[0], (double)u, (double)Au);
  }
};

// FP64 residual of Tin fields (mode 0: norms only; mode 1: also emit the
// scaled FP32 residual for the inner solve of iterative refinement).
template <typename Tin>
struct PhResid {
  static constexpr int NV = 4;
  static constexpr int PD = 1;
  using St = double;
  static __device__ __forceinline__ double val(double u) { return u; }
  const Tin* __restrict__ x;
  const Tin* __restrict__ b;
  float* __restrict__ r32;
  float* __restrict__ rh32;
  double scale;
  int emit;
  int hashed;      // inner shadow residual from the cell index (not stored)
  struct Raw { double x; };
  struct ERaw { double b; };
  WFA_PLAIN_OWN_STAGE
  __device__ void bind(const Scalars* sc) { scale = sc->scale; }
  __device__ Raw fetch(size_t i) const { return {(double)x[i]}; }
  __device__ double combine(const Raw& q) const { return q.x; }
  __device__ ERaw efetch(size_t i) const { return {(double)b[i]}; }
  __device__ void epilogue(size_t i, double, double Au, double, uint32_t, const ERaw& e, double dg,
                           double (&acc)[NV]) const {
    const double rv = e.b - Au;
    dot_acc(acc[0], rv, rv);
    dot_acc(acc[1], e.b, e.b);
    if (emit) {
      // emit == 2: the inner solve iterates on D^{-1} A, so its right-hand
      // side is D^{-1} r
      const float r32v = (float)((emit == 2 ? rv / dg : rv) * scale);
      r32[i] = r32v;
      float sh = r32v;
      if (hashed) sh = hashed_shadow<float>(i);
      else rh32[i] = r32v;
      dot_acc(acc[2], (double)r32v, (double)r32v);
      dot_acc(acc[3], (double)sh, (double)r32v);
    }
  }
};

// ============================================================================
// BiCGStab with two reductions per iteration
// ============================================================================
// Pass 1 applies the previous iteration's update on the fly,
//   s = r - alpha v,  r' = s - omega t,  x' = x + alpha p + omega s,
// and stages p' = r' + beta (p - omega v) (with halo) for v' = A p';
// reduces sigma = (rh, v'), (rh, r'), ||r'||^2.  On the first pass of a
// (re)start p' = r (and r is copied through so the r buffers alternate).
// HASHED: the build for the index-hashed shadow residual alone; it forms rh
// when the cell is staged instead of when its loads are issued (PD planes
// earlier), so no register holds it meanwhile: the same value.
template <typename T, bool HASHED = false>
struct PhAC {
  static constexpr int NV = 3;
  static constexpr int PD = 2;  // measured: 4% faster than 1 at 256^3 FP64
  using St = StageP<T>;
  static __device__ __forceinline__ T val(const St& u) { return u.p; }
  static __device__ __forceinline__ T val(T u) { return u; }
  const T* __restrict__ r;
  const T* __restrict__ v;
  const T* __restrict__ t;
  const T* __restrict__ p;
  const T* __restrict__ rh;
  T* __restrict__ x;
  T* __restrict__ r_out;
  T* __restrict__ p_out;
  T* __restrict__ v_out;
  T alpha, omega, beta;
  int first;
  int x_zero;      // x is still the zero initial guess (refinement's correction)
  int hashed;      // shadow residual from the cell index (not stored)
  struct Raw { T r, v, t, p; };
  struct ORawStored { T r, v, t, p, x, rh; };
  struct ORawHashed { T r, v, t, p, x; };
  using ORaw = std::conditional_t<HASHED, ORawHashed, ORawStored>;
  struct ERaw {};
  __device__ void bind(const Scalars* sc) {
    alpha = (T)sc->alpha;
    omega = (T)sc->omega;
    beta = (T)sc->beta;
    first = sc->first;
    x_zero = sc->x_zero;
  }
  __device__ Raw fetch(size_t i) const {
    if (first) return {r[i], T(0), T(0), T(0)};
    return {r[i], v[i], t[i], p[i]};
  }
  __device__ T combine(const Raw& q) const {
    if (first) return q.r;
    const T rn = minus_ax(minus_ax(q.r, alpha, q.v), omega, q.t);
    return next_p(rn, q.p, q.v, beta, omega);
  }
  __device__ ORaw fetch_own(size_t i) const {
    if constexpr (HASHED) {
      if (first) return {r[i], T(0), T(0), T(0), T(0)};
      return {r[i], v[i], t[i], p[i], x_zero ? T(0) : ld_once(x + i)};
    } else {
      const T sh = hashed ? hashed_shadow<T>(i) : ld_once(rh + i);
      if (first) return {r[i], T(0), T(0), T(0), T(0), sh};
      return {r[i], v[i], t[i], p[i], x_zero ? T(0) : ld_once(x + i), sh};
    }
  }
  // The previous iteration's update of this cell, applied and stored as soon
  // as the cell is staged: x' = x + alpha p + omega s, r' = s - omega t,
  // p' = r' + beta (p - omega v); (rh, r') and ||r'||^2 accumulate here.
  __device__ St combine_own(const ORaw& q, size_t i, double (&acc)[NV]) const {
    T sh;
    if constexpr (HASHED) sh = hashed_shadow<T>(i);
    else sh = q.rh;
    T rn, pn;
    if (first) {
      rn = q.r;
      pn = q.r;
    } else {
      const T s = minus_ax(q.r, alpha, q.v);
      rn = minus_ax(s, omega, q.t);
      pn = next_p(rn, q.p, q.v, beta, omega);
      st_once(x + i, next_x(q.x, q.p, s, alpha, omega));
    }
    st_once(r_out + i, rn);
    st_once(p_out + i, pn);
    dot_acc(acc[1], (double)sh, (double)rn);
    dot_acc(acc[2], (double)rn, (double)rn);
    return {pn, sh};
  }
  __device__ T value_own(const ORaw& q) const {
    return combine(Raw{q.r, q.v, q.t, q.p});
  }
  __device__ ERaw efetch(size_t) const { return {}; }
  __device__ void epilogue(size_t i, const St& u, T Au, T, uint32_t, const ERaw&, T dg,
                           double (&acc)[NV]) const {
    st_once(v_out + i, Au);
    dot_acc(acc[0], (double)u.rh, (double)Au);
  }
};

// Pass 2: s = r - alpha v staged, t = A s; (t,s), (t,t), (rh,s), (rh,t).
// HASHED: the build for the index-hashed shadow residual alone, which forms
// rh from the cell index in the epilogue (the `hashed` flag is not read), so
// that no register holds it from the plane's load issue to its epilogue:
// the same value, computed later.  The other build takes either shadow.
template <typename T, bool HASHED = false>
struct PhB2 {
  static constexpr int NV = 4;
  static constexpr int PD = 1;  // measured: 4-6% faster than 2 (its epilogue loads nothing)
  static constexpr bool kCarryZ = true;  // measured: 3% (FP64) / 5% (FP32) faster
  using St = T;
  static __device__ __forceinline__ T val(T u) { return u; }
  const T* __restrict__ r;
  const T* __restrict__ v;
  const T* __restrict__ rh;
  T* __restrict__ t;
  T alpha;
  int hashed;      // shadow residual from the cell index (not stored)
  struct Raw { T r, v; };
  struct StoredRh { T rh; };
  struct NoRh {};
  using ERaw = std::conditional_t<HASHED, NoRh, StoredRh>;
  WFA_PLAIN_OWN_STAGE
  __device__ void bind(const Scalars* sc) { alpha = (T)sc->alpha; }
  __device__ Raw fetch(size_t i) const { return {r[i], v[i]}; }
  __device__ T combine(const Raw& q) const { return minus_ax(q.r, alpha, q.v); }
  __device__ ERaw efetch(size_t i) const {
    if constexpr (HASHED) return {};
    else return {hashed ? hashed_shadow<T>(i) : ld_once(rh + i)};
  }
  __device__ void epilogue(size_t i, T s, T Au, T, uint32_t, const ERaw& e, T dg,
                           double (&acc)[NV]) const {
    if (t) st_once(t + i, Au);   // none when pass 1 forms t again
    T rhv;
    if constexpr (HASHED) rhv = hashed_shadow<T>(i);
    else rhv = e.rh;
    dot_acc(acc[0], (double)Au, (double)s);
    dot_acc(acc[1], (double)Au, (double)Au);
    dot_acc(acc[2], (double)rhv, (double)s);
    dot_acc(acc[3], (double)rhv, (double)Au);
  }
};

// ============================================================================
// CG with one reduction per iteration (Chronopoulos-Gear)
// ============================================================================
// One pass per iteration.  It applies the previous iteration's update on the
// fly, s' = w + beta s, p' = r + beta p, x' = x + alpha p', r' = r - alpha s'
// (stage 1: p' = r, s' = w), stages r' (with halo, from r, w, s) for
// w' = A r', and reduces (r', r') and (w', r').  Stage 0 stages r itself
// (copied through so the r buffers alternate) and only forms w0 = A r0.
// r, w and s are read on neighbour cells and double-buffered; p and x are
// read and written on own cells only, in place.
template <typename T>
struct PhCg1 {
  static constexpr int NV = 2;
  static constexpr int PD = 2;
  using St = T;
  static __device__ __forceinline__ T val(T u) { return u; }
  const T* __restrict__ r;
  const T* __restrict__ w;
  const T* __restrict__ s;
  T* __restrict__ p;
  T* __restrict__ x;
  T* __restrict__ r_out;
  T* __restrict__ w_out;
  T* __restrict__ s_out;
  T alpha, beta;
  int stage;
  int x_zero;      // x is still the zero initial guess (refinement's correction)
  struct Raw { T r, w, s; };
  struct ORaw { T r, w, s, p, x; };
  struct ERaw {};
  __device__ void bind(const Scalars* sc) {
    alpha = (T)sc->alpha;
    beta = (T)sc->beta;
    stage = sc->stage;
    x_zero = sc->x_zero;
  }
  // s' of this cell (the same expression for own and halo cells, so both
  // stage the same r')
  __device__ T s_new(T w_, T s_) const { return stage == 1 ? w_ : fma_t(beta, s_, w_); }
  __device__ T r_new(T r_, T sn) const { return fma_t(-alpha, sn, r_); }
  __device__ Raw fetch(size_t i) const {
    if (stage == 0) return {r[i], T(0), T(0)};
    if (stage == 1) return {r[i], w[i], T(0)};
    return {r[i], w[i], s[i]};
  }
  __device__ T combine(const Raw& q) const {
    if (stage == 0) return q.r;
    return r_new(q.r, s_new(q.w, q.s));
  }
  __device__ ORaw fetch_own(size_t i) const {
    if (stage == 0) return {r[i], T(0), T(0), T(0), T(0)};
    if (stage == 1) return {r[i], w[i], T(0), T(0), x_zero ? T(0) : ld_once(x + i)};
    return {r[i], w[i], s[i], ld_once(p + i), ld_once(x + i)};
  }
  __device__ St combine_own(const ORaw& q, size_t i, double (&acc)[NV]) const {
    T rn;
    if (stage == 0) {
      rn = q.r;
    } else {
      const T sn = s_new(q.w, q.s);
      const T pn = stage == 1 ? q.r : fma_t(beta, q.p, q.r);
      rn = r_new(q.r, sn);
      st_once(s_out + i, sn);
      st_once(p + i, pn);
      st_once(x + i, fma_t(alpha, pn, q.x));
    }
    st_once(r_out + i, rn);
    dot_acc(acc[0], (double)rn, (double)rn);
    return rn;
  }
  __device__ T value_own(const ORaw& q) const { return combine(Raw{q.r, q.w, q.s}); }
  __device__ ERaw efetch(size_t) const { return {}; }
  __device__ void epilogue(size_t i, T rn, T Au, T, uint32_t, const ERaw&, T dg,
                           double (&acc)[NV]) const {
    st_once(w_out + i, Au);
    dot_acc(acc[1], (double)Au, (double)rn);
  }
};

// After pass 1: the iteration whose update was just applied is checked
// (convergence on the exact ||r||, limits, a pending restart), then alpha
// from the exact rho.
struct FinAC {
  Scalars* sc;
  __device__ void operator()(const double (&s)[3]) const {
    const double sigma = s[0], rho_exact = s[1], rr = s[2];
    sc->sigma = sigma;
    if (!sc->first) {
      sc->iter += 1;
      sc->rr = rr;
      sc->x_zero = 0;
      if (rr < sc->rr_min) { sc->rr_min = rr; sc->it_min = sc->iter; }
      if (!fin_ok(rr)) { sc->status = ST_NONFINITE; return; }
      if (sc->szero || sqrt(rr) <= sc->tol * sqrt(sc->bb)) { sc->status = ST_CONV; return; }
      if ((sc->guard > 0.0 && rr > sc->guard * sc->rr0) || sc->iter == sc->force_div) {
        sc->status = ST_NOCONV;
        sc->diverged = 1;
        return;
      }
      if (sc->restart_pending) { sc->restart = 1; return; }
      if (sc->iter >= sc->maxit) { sc->status = ST_NOCONV; return; }
      if (!fin_ok(rho_exact)) { sc->status = ST_NONFINITE; return; }
      if (rho_exact == 0.0) { sc->restart = 1; return; }
      sc->rho = rho_exact;
    }
    if (sc->force_bd > 0 && sc->iter + 1 == sc->force_bd) { sc->sigma = 0.0; sc->force_bd = 0; }
    if (!fin_ok(sc->sigma)) sc->status = ST_NONFINITE;
    else if (sc->sigma == 0.0) sc->restart = 1;
    else sc->alpha = sc->rho / sc->sigma;
  }
};

// After pass 2: omega, and beta from the predicted next rho.
struct FinB2 {
  Scalars* sc;
  __device__ void operator()(const double (&s)[4]) const {
    const double ts = s[0], tt = s[1], rs = s[2], rt = s[3];
    sc->ts = ts; sc->tt = tt;
    if (!fin_ok(ts) || !fin_ok(tt) || !fin_ok(rs) || !fin_ok(rt)) {
      sc->status = ST_NONFINITE;
      return;
    }
    if (tt == 0.0) {
      sc->omega = 0.0;
      sc->szero = 1;
    } else {
      sc->omega = ts / tt;
      if (sc->omega == 0.0) sc->restart_pending = 1;
    }
    if (!sc->szero && !sc->restart_pending) {
      const double rho_pred = rs - sc->omega * rt;
      sc->beta = (rho_pred / sc->rho) * (sc->alpha / sc->omega);
    } else {
      sc->beta = 0.0;
    }
    sc->first = 0;
  }
};

// ============================================================================
// pointwise passes: the range of elements one workgroup of a `blocks`-wide
// launch covers (the same split in single-solve and batched launches)
// ============================================================================
template <typename T>
struct alignas(16) V16 {
  static constexpr int N = 16 / sizeof(T);
  T v[N];
};

__device__ __forceinline__ bool aligned16(const void* a, const void* b, const void* c,
                                          const void* d, const void* e, const void* f) {
  return ((((uintptr_t)a) | ((uintptr_t)b) | ((uintptr_t)c) | ((uintptr_t)d) | ((uintptr_t)e) |
           ((uintptr_t)f)) & 15) == 0;
}

template <typename T>
__device__ __forceinline__ void phase_c_elem(T& x, T p, T& r, T v, T t, T rh, T alpha, T omega,
                                             bool xz, double (&acc)[2]) {
  const T s = minus_ax(r, alpha, v);
  const T xo = xz ? T(0) : x;
  x = next_x(xo, p, s, alpha, omega);
  const T rn = minus_ax(s, omega, t);
  r = rn;
  dot_acc(acc[0], (double)rh, (double)rn);
  dot_acc(acc[1], (double)rn, (double)rn);
}

// 16-byte vector loads when every stream is 16-byte aligned; the scalar
// loop covers the remainder (and unaligned streams).
template <typename T>
__device__ __forceinline__ void phase_c_range(size_t n, int blk, int blocks, T* __restrict__ x,
                                              const T* __restrict__ p, T* __restrict__ r,
                                              const T* __restrict__ v, const T* __restrict__ t,
                                              const T* __restrict__ rh, const Scalars* sc,
                                              double (&acc)[2]) {
  const T alpha = (T)sc->alpha, omega = (T)sc->omega;
  const bool xz = sc->x_zero != 0;
  const size_t stride = (size_t)blocks * kThreads;
  size_t done = 0;
  if (aligned16(x, p, r, v, t, rh)) {
    using VT = V16<T>;
    constexpr int N = VT::N;
    const size_t nv = n / N;
    VT* xv = (VT*)x;
    VT* rv = (VT*)r;
    for (size_t e = (size_t)blk * kThreads + threadIdx.x; e < nv; e += stride) {
      VT xa = xz ? VT{} : xv[e];
      VT ra = rv[e];
      const VT pa = ((const VT*)p)[e], va = ((const VT*)v)[e];
      const VT ta = ((const VT*)t)[e], ha = ((const VT*)rh)[e];
#pragma unroll
      for (int c = 0; c < N; ++c)
        phase_c_elem<T>(xa.v[c], pa.v[c], ra.v[c], va.v[c], ta.v[c], ha.v[c], alpha, omega, xz, acc);
      xv[e] = xa;
      rv[e] = ra;
    }
    done = nv * N;
  }
  for (size_t e = done + (size_t)blk * kThreads + threadIdx.x; e < n; e += stride)
    phase_c_elem<T>(x[e], p[e], r[e], v[e], t[e], rh[e], alpha, omega, xz, acc);
}

template <typename T>
__device__ __forceinline__ void cg_b_range(size_t n, int blk, int blocks, T* __restrict__ x,
                                           const T* __restrict__ d, T* __restrict__ r,
                                           const T* __restrict__ q, const Scalars* sc,
                                           double (&acc)[1]) {
  const T alpha = (T)sc->alpha;
  const size_t stride = (size_t)blocks * kThreads;
  size_t done = 0;
  if (aligned16(x, d, r, q, x, x)) {
    using VT = V16<T>;
    constexpr int N = VT::N;
    const size_t nv = n / N;
    VT* xv = (VT*)x;
    VT* rv = (VT*)r;
    for (size_t e = (size_t)blk * kThreads + threadIdx.x; e < nv; e += stride) {
      VT xa = xv[e], ra = rv[e];
      const VT da = ((const VT*)d)[e], qa = ((const VT*)q)[e];
#pragma unroll
      for (int c = 0; c < N; ++c) {
        xa.v[c] = fma_t(alpha, da.v[c], xa.v[c]);
        ra.v[c] = minus_ax(ra.v[c], alpha, qa.v[c]);
        dot_acc(acc[0], (double)ra.v[c], (double)ra.v[c]);
      }
      xv[e] = xa;
      rv[e] = ra;
    }
    done = nv * N;
  }
  for (size_t e = done + (size_t)blk * kThreads + threadIdx.x; e < n; e += stride) {
    x[e] = fma_t(alpha, d[e], x[e]);
    const T rn = minus_ax(r[e], alpha, q[e]);
    r[e] = rn;
    dot_acc(acc[0], (double)rn, (double)rn);
  }
}

}  // namespace wfa
