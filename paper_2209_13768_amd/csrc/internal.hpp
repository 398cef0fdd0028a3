// Host-side interfaces between the solver driver and the kernel launchers.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "device.hpp"
#include "wfa.h"

namespace wfa {

// Tile shape of one grid.  A function of the grid shape and vector type
// only, so that a solve's reduction order does not depend on anything else
// (other requests in a batch, the launch mode).
struct Tiling {
  int ry;          // rows per wave (TY = 4 * ry)
  Geo geo;         // tile grid
  int pw_blocks;   // workgroups of the pointwise kernels
};

Tiling make_tiling(int nx, int ny, int nz, int elem_bytes, int zc_override, int ry_override);

// Pointers of one phase launch.
template <typename T>
struct Launch {
  Tiling tl;
  Op<T> op;
  bool cell;
  const float* kappa;
  double* partials;
  Scalars* sc;
  hipStream_t stream;
  int shadow;   // 1: the two-reduction BiCGStab's shadow residual is index-hashed
};

// y = A x
template <typename T>
void launch_apply(const Launch<T>& L, const T* x, T* y);
// b = T + boundary terms (form_b) or given b; r = b - A x; rh = r; partial
// sums (b,b), (r,r); finalize sets up the first iteration.
template <typename T>
void launch_init(const Launch<T>& L, bool form_b, const T* x, const T* b_in, T* b_out, T* r,
                 T* rh);
// b = T + boundary terms only
template <typename T>
void launch_rhs(const Launch<T>& L, const T* x, T* b);
// One explicit forward-time step: y = x - (A x - x) + boundary terms
template <typename T>
void launch_explicit(const Launch<T>& L, const T* x, T* y);
// `steps` (2 to 4) explicit steps in one pass, constant diffusivity only;
// zc_override > 0 sets the output planes per workgroup
template <typename T>
void launch_explicit_fused(const Launch<T>& L, const T* x, T* y, int steps, int zc_override);
// p' = r + beta (p - omega v) (p' = r on the first iteration); v' = A p';
// sigma = (rh, v')
template <typename T>
void launch_phase_a(const Launch<T>& L, const T* r, const T* p, const T* v, T* p_out, T* v_out,
                    const T* rh);
// s = r - alpha v; t = A s; (t,s), (t,t)
template <typename T>
void launch_phase_b(const Launch<T>& L, const T* r, const T* v, T* t);
// x += alpha p + omega s; r = s - omega t; (rh, r), (r, r)
template <typename T>
void launch_phase_c(const Launch<T>& L, T* x, const T* p, T* r, const T* v, const T* t,
                    const T* rh);
// Two-reduction BiCGStab, pass 1: apply the previous update (x, r -> r_out)
// and stage p_out = r' + beta (p - omega v); v_out = A p_out; sigma,
// (rh, r'), ||r'||^2
template <typename T>
void launch_phase_ac(const Launch<T>& L, const T* r, const T* v, const T* t, const T* p,
                     const T* rh, T* x, T* r_out, T* p_out, T* v_out);
// pass 2: s = r - alpha v; t = A s; (t,s), (t,t), (rh,s), (rh,t); t is
// stored unless t == nullptr (pass 1 then forms it again: launch_phase_act)
template <typename T>
void launch_phase_b2(const Launch<T>& L, const T* r, const T* v, const T* rh, T* t);
// Pass 1 with t = A s formed again from r and v instead of read (the same
// stores and sums, bitwise, as launch_phase_ac with the t pass 2 formed)
template <typename T>
void launch_phase_act(const Launch<T>& L, const T* r, const T* v, const T* p, const T* rh, T* x,
                      T* r_out, T* p_out, T* v_out);
// One iteration of CG with one reduction (Chronopoulos-Gear): the previous
// update applied on the fly (p, x in place; s' into s_out, r' into r_out),
// w' = A r' into w_out; (r', r') and (w', r') reduced.  Stage 0 (after
// init) only forms w0 = A r0 and copies r through.
template <typename T>
void launch_phase_cg1(const Launch<T>& L, const T* r, const T* w, const T* s, T* p, T* x,
                      T* r_out, T* w_out, T* s_out);
// CG: d' = r + beta d (d' = r first); q = A d'; (d', q)
template <typename T>
void launch_cg_a(const Launch<T>& L, const T* r, const T* d, T* d_out, T* q);
// CG: x += alpha d; r -= alpha q; (r, r)
template <typename T>
void launch_cg_b(const Launch<T>& L, T* x, const T* d, T* r, const T* q);
// FP64 residual of Tin-typed x, b: (r,r), (b,b); optionally r32 = fp32(r *
// scale) into r32, the inner shadow residual (r32 itself into rh32, or the
// index-hashed field when `hashed`), and (r32, r32), (rh, r32) for the inner
// solve (sc_inner).  With `after`, the pass runs only if the solve whose
// scalars `after` points at has converged or reached its iteration limit
// when the pass starts; otherwise it leaves everything untouched.
template <typename Tin>
void launch_residual(const Launch<double>& L, const Tin* x, const Tin* b, float* r32,
                     float* rh32, Scalars* sc_inner, int mode, int hashed,
                     const Scalars* after = nullptr);
// *dst = v, stream-ordered, from a kernel argument (no host copy to wait on)
void launch_set_scalars(Scalars* dst, const Scalars& v, hipStream_t s);
// x64 += inv_scale * d32 (scalars of the inner solve)
void launch_promote(size_t n, int blocks, double* x, const float* d, const Scalars* sc_inner,
                    hipStream_t s);
template <typename T>
void launch_fill(size_t n, T* y, T v, hipStream_t s);
// Up to `iters` BiCGStab iterations in one cooperative launch; the same
// iterates as launch_phase_a/b/c.  p0/v0 hold the inputs of the first
// iteration when parity == 0.
template <typename T>
hipError_t launch_persistent_bicgstab(const Launch<T>& L, T* x, T* r, const T* rh, T* p0, T* p1,
                                      T* v0, T* v1, T* t, int iters, int parity,
                                      GridBarrier* bar);

// Streams a probe kind reads and writes: `bytes` each (a copy: 2; a stream
// mix: its reads and writes).
inline int probe_reads(int kind) {
  return kind == WFA_PROBE_WRITE ? 0 : kind == WFA_PROBE_MIX_6R4W ? 6 : kind == WFA_PROBE_MIX_3R1W ? 3 : 1;
}
inline int probe_writes(int kind) {
  return kind == WFA_PROBE_READ ? 0 : kind == WFA_PROBE_MIX_6R4W ? 4 : 1;
}
inline int probe_streams(int kind) { return probe_reads(kind) + probe_writes(kind); }

// HBM bandwidth probe of one kind (WFA_PROBE_*): GB/s over `reps` launches
// of `blocks` workgroups.
double bandwidth_probe(int kind, int blocks, const void* src, void* dst, size_t bytes, int reps,
                       hipStream_t s, hipError_t* err);

}  // namespace wfa
