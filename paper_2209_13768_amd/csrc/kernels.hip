// Kernels of libwfa and their host launchers.
//
// One BiCGStab iteration (van der Vorst 1992) is three streaming passes, one
// per global reduction it needs (the paper, section 1.1.2, notes that each
// Krylov reduction is a global synchronisation; section 3.2.2 overlaps the
// solution update with the residual-norm reduction, as phase C does here):
//   phase A  p' = r + beta (p - omega v)   staged on the fly, with halo
//            v' = A p'                     z-march, LDS plane + registers
//            sigma = (rh, v')              -> alpha = rho / sigma
//   phase B  s = r - alpha v'              staged on the fly (never stored)
//            t = A s                       z-march
//            (t,s), (t,t)                  -> omega = (t,s)/(t,t)
//   phase C  x += alpha p' + omega s; r = s - omega t        pointwise
//            rho' = (rh, r), ||r||^2       -> beta, convergence
// Vector streams per iteration: 6 + 3 + 8 = 17 (+ one diffusivity read per
// operator product in CELL mode).  Each pass ends with a deterministic
// last-workgroup reduction that writes the next scalars on the device, so
// the host never sits inside an iteration.
#include <math.h>

#include "device.hpp"
#include "wfa.h"
#include "internal.hpp"
#include "phases.hpp"

namespace wfa {

// ============================================================================
// generic stencil-pass kernel
// ============================================================================
// Waves per SIMD a build is compiled for (1: the compiler's choice).  The
// hashed-shadow builds of the no-scaling operators at two rows per wave fit
// 5 waves without spilling: the FP64 second pass in 93 VGPRs (98 and 4 waves
// otherwise; measured 3-4% faster on 256^3), the FP32 fused update pass in
// 96.
template <typename T, bool CELL, int RY, class Ph, int FORM>
struct MinWaves {
  static constexpr int value = 1;
};
template <int FORM>
struct MinWaves<double, true, 2, PhB2<double, true>, FORM> {
  static constexpr int value = 5;
};
template <int FORM>
struct MinWaves<float, true, 2, PhAC<float, true>, FORM> {
  static constexpr int value = 5;
};

template <typename T, bool CELL, int RY, class Ph, class Fin, int FORM = kFormGeneral>
__global__ void __launch_bounds__(kThreads)
__attribute__((amdgpu_waves_per_eu(MinWaves<T, CELL, RY, Ph, FORM>::value)))
k_march(Geo g, Op<T> op, const float* __restrict__ kappa, Ph ph, double* partials,
        Scalars* sc, Fin fin, const Scalars* gate, int gated, int publish) {
  static_assert(Ph::NV <= kMaxReduce, "the workspace holds kMaxReduce partials per tile");
  using TS = TileShape<RY>;
  __shared__ T su[2 * TS::LH * TS::LW];
  __shared__ float sk[CELL ? 2 * TS::LH * TS::LW : 1];
  __shared__ double red[kWaves * Ph::NV];
  // gated 1: an iteration pass, skipped once its solve has stopped or awaits
  // a restart; gated 2: a true-residual pass queued behind a chunk of
  // iterations, run only once the solve `gate` has converged or reached its
  // iteration limit
  if (gated == 1 && (gate->status != ST_RUN || gate->restart)) return;
  if (gated == 2 && gate->status != ST_CONV && gate->status != ST_NOCONV) return;
  ph.bind(sc);
  double acc[Ph::NV];
#pragma unroll
  for (int q = 0; q < Ph::NV; ++q) acc[q] = 0.0;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  march_tile<T, CELL, RY, Ph, FORM>(g, op, kappa, tile, ph, acc, su, sk);
  if (publish) publish_and_finalize<Ph::NV>(acc, tile, g.ntiles, partials, sc, red, fin);
}

// FORMS: the phase also has the builds of the cell operator without the
// Jacobi scaling select and without the convective terms, launched for an
// operator that has neither (op_form): the same values with fewer vector
// instructions.  Only the two-reduction BiCGStab's passes on a per-cell
// diffusivity carry them, to keep the number of kernels down.
// FORMS_ONLY: only those two builds exist (the general ones are not
// instantiated); the caller launches it for an operator that has one of
// them, on a per-cell diffusivity.
template <typename T, class Ph, class Fin, bool FORMS = false, bool FORMS_ONLY = false>
void dispatch_march(const Launch<T>& L, const Ph& ph, const Fin& fin, bool gated, bool publish,
                    const Scalars* after = nullptr) {
  static_assert(FORMS || !FORMS_ONLY, "FORMS_ONLY needs FORMS");
  const Geo g = L.tl.geo;
  dim3 grid(g.ntiles), block(kThreads);
  const int G = after ? 2 : gated ? 1 : 0, P = publish ? 1 : 0;
  const Scalars* gate = after ? after : L.sc;
#define WFA_MARCH_F(RYV, FORMV)                                                               \
  hipLaunchKernelGGL((k_march<T, true, RYV, Ph, Fin, FORMV>), grid, block, 0, L.stream, g,     \
                     L.op, L.kappa, ph, L.partials, L.sc, fin, gate, G, P)
#define WFA_MARCH_FORM(FORMV)                      \
  switch (L.tl.ry) {                               \
    case 1: WFA_MARCH_F(1, FORMV); break;          \
    case 4: WFA_MARCH_F(4, FORMV); break;          \
    default: WFA_MARCH_F(2, FORMV); break;         \
  }
  if constexpr (FORMS) {
    if (L.cell && op_form(L.op) == kFormDiffusion) {
      WFA_MARCH_FORM(kFormDiffusion);
      return;
    }
    if (L.cell && op_form(L.op) == kFormConvection) {
      WFA_MARCH_FORM(kFormConvection);
      return;
    }
  }
#undef WFA_MARCH_FORM
#undef WFA_MARCH_F
  if constexpr (FORMS_ONLY) return;
  else {
#define WFA_MARCH(CELLV, RYV)                                                              \
  hipLaunchKernelGGL((k_march<T, CELLV, RYV, Ph, Fin>), grid, block, 0, L.stream, g, L.op, \
                     L.kappa, ph, L.partials, L.sc, fin, gate, G, P)
  if (L.cell) {
    switch (L.tl.ry) {
      case 1: WFA_MARCH(true, 1); break;
      case 4: WFA_MARCH(true, 4); break;
      default: WFA_MARCH(true, 2); break;
    }
  } else {
    switch (L.tl.ry) {
      case 1: WFA_MARCH(false, 1); break;
      case 4: WFA_MARCH(false, 4); break;
      default: WFA_MARCH(false, 2); break;
    }
  }
#undef WFA_MARCH
  }
}

template <typename T>
void launch_apply(const Launch<T>& L, const T* x, T* y) {
  PhApply<T> ph{x, y};
  dispatch_march(L, ph, FinNone{}, false, false);
}

template <typename T>
void launch_rhs(const Launch<T>& L, const T* x, T* b) {
  if (L.cell) {
    PhRhs<T, true> ph{L.op, x, b};
    dispatch_march(L, ph, FinNone{}, false, false);
  } else {
    PhRhs<T, false> ph{L.op, x, b};
    dispatch_march(L, ph, FinNone{}, false, false);
  }
}

template <typename T>
void launch_explicit(const Launch<T>& L, const T* x, T* y) {
  if (L.cell) {
    PhExplicit<T, true> ph{L.op, x, y};
    dispatch_march(L, ph, FinNone{}, false, false);
  } else {
    PhExplicit<T, false> ph{L.op, x, y};
    dispatch_march(L, ph, FinNone{}, false, false);
  }
}

template <typename T>
void launch_init(const Launch<T>& L, bool form_b, const T* x, const T* b_in, T* b_out, T* r,
                 T* rh) {
  FinInit fin{L.sc};
  if (L.cell) {
    if (form_b) dispatch_march(L, PhInit<T, true, true>{L.op, x, b_in, b_out, r, rh, L.shadow}, fin, false, true);
    else dispatch_march(L, PhInit<T, true, false>{L.op, x, b_in, b_out, r, rh, L.shadow}, fin, false, true);
  } else {
    if (form_b) dispatch_march(L, PhInit<T, false, true>{L.op, x, b_in, b_out, r, rh, L.shadow}, fin, false, true);
    else dispatch_march(L, PhInit<T, false, false>{L.op, x, b_in, b_out, r, rh, L.shadow}, fin, false, true);
  }
}

template <typename T>
void launch_phase_a(const Launch<T>& L, const T* r, const T* p, const T* v, T* p_out, T* v_out,
                    const T* rh) {
  PhA<T> ph{};
  ph.r = r; ph.p = p; ph.v = v; ph.p_out = p_out; ph.v_out = v_out; ph.rh = rh;
  dispatch_march(L, ph, FinA{L.sc}, true, true);
}

template <typename T>
void launch_phase_b(const Launch<T>& L, const T* r, const T* v, T* t) {
  PhB<T> ph{};
  ph.r = r; ph.v = v; ph.t = t;
  dispatch_march(L, ph, FinB{L.sc}, true, true);
}

template <typename T>
void launch_phase_ac(const Launch<T>& L, const T* r, const T* v, const T* t, const T* p,
                     const T* rh, T* x, T* r_out, T* p_out, T* v_out) {
  if (L.shadow && L.cell && op_form(L.op) != kFormGeneral) {
    PhAC<T, true> ph{};
    ph.hashed = 1;
    ph.r = r; ph.v = v; ph.t = t; ph.p = p; ph.rh = rh; ph.x = x;
    ph.r_out = r_out; ph.p_out = p_out; ph.v_out = v_out;
    dispatch_march<T, PhAC<T, true>, FinAC, true, true>(L, ph, FinAC{L.sc}, true, true);
    return;
  }
  PhAC<T> ph{};
  ph.hashed = L.shadow;
  ph.r = r; ph.v = v; ph.t = t; ph.p = p; ph.rh = rh; ph.x = x;
  ph.r_out = r_out; ph.p_out = p_out; ph.v_out = v_out;
  dispatch_march<T, PhAC<T>, FinAC, true>(L, ph, FinAC{L.sc}, true, true);
}

template <typename T>
void launch_phase_b2(const Launch<T>& L, const T* r, const T* v, const T* rh, T* t) {
  if (L.shadow && L.cell && op_form(L.op) != kFormGeneral) {
    PhB2<T, true> ph{};
    ph.hashed = 1;
    ph.r = r; ph.v = v; ph.rh = rh; ph.t = t;
    dispatch_march<T, PhB2<T, true>, FinB2, true, true>(L, ph, FinB2{L.sc}, true, true);
    return;
  }
  PhB2<T> ph{};
  ph.hashed = L.shadow;
  ph.r = r; ph.v = v; ph.rh = rh; ph.t = t;
  dispatch_march<T, PhB2<T>, FinB2, true>(L, ph, FinB2{L.sc}, true, true);
}

template <typename T>
void launch_phase_cg1(const Launch<T>& L, const T* r, const T* w, const T* s, T* p, T* x,
                      T* r_out, T* w_out, T* s_out) {
  PhCg1<T> ph{};
  ph.r = r; ph.w = w; ph.s = s; ph.p = p; ph.x = x;
  ph.r_out = r_out; ph.w_out = w_out; ph.s_out = s_out;
  dispatch_march(L, ph, FinCg1{L.sc}, true, true);
}

template <typename T>
void launch_cg_a(const Launch<T>& L, const T* r, const T* d, T* d_out, T* q) {
  PhCgA<T> ph{};
  ph.r = r; ph.d = d; ph.d_out = d_out; ph.q = q;
  dispatch_march(L, ph, FinCgA{L.sc}, true, true);
}

template <typename Tin>
void launch_residual(const Launch<double>& L, const Tin* x, const Tin* b, float* r32,
                     float* rh32, Scalars* sc_inner, int mode, int hashed, const Scalars* after) {
  PhResid<Tin> ph{};
  ph.x = x; ph.b = b; ph.r32 = r32; ph.rh32 = rh32; ph.emit = mode; ph.hashed = hashed;
  dispatch_march(L, ph, FinResid{L.sc, mode ? sc_inner : nullptr}, false, true, after);
}

// The host's values arrive as a kernel argument, so setting a scalar block
// never waits on a host copy.
__global__ void __launch_bounds__(64) k_set_scalars(Scalars* __restrict__ dst, Scalars v) {
  if (threadIdx.x == 0) *dst = v;
}

void launch_set_scalars(Scalars* dst, const Scalars& v, hipStream_t s) {
  hipLaunchKernelGGL(k_set_scalars, dim3(1), dim3(64), 0, s, dst, v);
}

// ============================================================================
// pointwise kernels
// ============================================================================
template <typename T>
__global__ void __launch_bounds__(kThreads)
k_phase_c(size_t n, T* __restrict__ x, const T* __restrict__ p, T* __restrict__ r,
          const T* __restrict__ v, const T* __restrict__ t, const T* __restrict__ rh,
          double* partials, Scalars* sc) {
  __shared__ double red[kWaves * 2];
  if (sc->status != ST_RUN || sc->restart) return;
  double acc[2] = {0.0, 0.0};
  phase_c_range<T>(n, blockIdx.x, gridDim.x, x, p, r, v, t, rh, sc, acc);
  publish_and_finalize<2>(acc, blockIdx.x, gridDim.x, partials, sc, red, FinC{sc});
}

template <typename T>
__global__ void __launch_bounds__(kThreads)
k_cg_b(size_t n, T* __restrict__ x, const T* __restrict__ d, T* __restrict__ r,
       const T* __restrict__ q, double* partials, Scalars* sc) {
  __shared__ double red[kWaves];
  if (sc->status != ST_RUN) return;
  double acc[1] = {0.0};
  cg_b_range<T>(n, blockIdx.x, gridDim.x, x, d, r, q, sc, acc);
  publish_and_finalize<1>(acc, blockIdx.x, gridDim.x, partials, sc, red, FinCgB{sc});
}

__global__ void __launch_bounds__(kThreads)
k_promote(size_t n, double* __restrict__ x, const float* __restrict__ d, const Scalars* sc) {
  if (sc->status == ST_NONFINITE) return;
  const double inv = sc->inv_scale;
  const size_t stride = (size_t)gridDim.x * kThreads;
  for (size_t e = (size_t)blockIdx.x * kThreads + threadIdx.x; e < n; e += stride)
    x[e] = __builtin_fma(inv, (double)d[e], x[e]);   // one rounding, as written
}

template <typename T>
__global__ void __launch_bounds__(kThreads) k_fill(size_t n, T* __restrict__ y, T v) {
  const size_t stride = (size_t)gridDim.x * kThreads;
  for (size_t e = (size_t)blockIdx.x * kThreads + threadIdx.x; e < n; e += stride) y[e] = v;
}

static size_t cells_of(const Geo& g) { return (size_t)g.plane * (size_t)g.nz; }

template <typename T>
void launch_phase_c(const Launch<T>& L, T* x, const T* p, T* r, const T* v, const T* t,
                    const T* rh) {
  hipLaunchKernelGGL(k_phase_c<T>, dim3(L.tl.pw_blocks), dim3(kThreads), 0, L.stream,
                     cells_of(L.tl.geo), x, p, r, v, t, rh, L.partials, L.sc);
}

template <typename T>
void launch_cg_b(const Launch<T>& L, T* x, const T* d, T* r, const T* q) {
  hipLaunchKernelGGL(k_cg_b<T>, dim3(L.tl.pw_blocks), dim3(kThreads), 0, L.stream,
                     cells_of(L.tl.geo), x, d, r, q, L.partials, L.sc);
}

void launch_promote(size_t n, int blocks, double* x, const float* d, const Scalars* sc_inner,
                    hipStream_t s) {
  hipLaunchKernelGGL(k_promote, dim3(blocks), dim3(kThreads), 0, s, n, x, d, sc_inner);
}

template <typename T>
void launch_fill(size_t n, T* y, T v, hipStream_t s) {
  const int blocks = (int)((n + kThreads - 1) / kThreads < 4096 ? (n + kThreads - 1) / kThreads : 4096);
  hipLaunchKernelGGL(k_fill<T>, dim3(blocks > 0 ? blocks : 1), dim3(kThreads), 0, s, n, y, v);
}

// ============================================================================
// tiling
// ============================================================================
Tiling make_tiling(int nx, int ny, int nz, int elem_bytes, int zc_override, int ry_override) {
  Tiling t{};
  // 2 rows per wave (8-row tiles) measured fastest on 256^3 FP64 and
  // 512x512x1024 FP32 among 1, 2 and 4 rows
  t.ry = (ry_override == 1 || ry_override == 2 || ry_override == 4) ? ry_override : 2;
  const int TY = kWaves * t.ry;
  Geo& g = t.geo;
  g.nx = nx; g.ny = ny; g.nz = nz;
  g.plane = (long long)nx * ny;
  g.tiles_x = (nx + kTX - 1) / kTX;
  g.tiles_y = (ny + TY - 1) / TY;
  const long long txy = (long long)g.tiles_x * g.tiles_y;
  int zc;
  if (zc_override > 0) {
    zc = zc_override;
  } else {
    // 16 planes per tile (the two z-halo planes cost 1/8 extra stage reads)
    // unless the grid has enough columns for >= 2048 tiles of 32 planes
    zc = (txy * nz >= 2048LL * 32) ? 32 : 16;
  }
  if (zc > nz) zc = nz;
  if (zc < 1) zc = 1;
  // small grids: thinner tiles until there are >= 128 of them (measured on
  // 32^3 and 64^3, where a pass is a few microseconds and parallelism wins;
  // more tiles per grid cost the batched server more than they gain)
  if (zc_override <= 0)
    while (zc > 2 && txy * ((nz + zc - 1) / zc) < 128) zc /= 2;
  g.zc = zc;
  g.zchunks = (nz + zc - 1) / zc;
  g.ntiles = (int)(txy * g.zchunks);
  const size_t n = (size_t)g.plane * nz;
  const size_t per_block = (size_t)kThreads * 8;
  size_t pb = (n + per_block - 1) / per_block;
  if (pb > 2048) pb = 2048;
  if (pb < 1) pb = 1;
  t.pw_blocks = (int)pb;
  (void)elem_bytes;
  return t;
}

// ============================================================================
// explicit instantiations
// ============================================================================
#define WFA_INST(T)                                                                           \
  template void launch_apply<T>(const Launch<T>&, const T*, T*);                             \
  template void launch_rhs<T>(const Launch<T>&, const T*, T*);                               \
  template void launch_explicit<T>(const Launch<T>&, const T*, T*);                          \
  template void launch_init<T>(const Launch<T>&, bool, const T*, const T*, T*, T*, T*);      \
  template void launch_phase_a<T>(const Launch<T>&, const T*, const T*, const T*, T*, T*,    \
                                  const T*);                                                 \
  template void launch_phase_b<T>(const Launch<T>&, const T*, const T*, T*);                 \
  template void launch_phase_c<T>(const Launch<T>&, T*, const T*, T*, const T*, const T*,    \
                                  const T*);                                                 \
  template void launch_cg_a<T>(const Launch<T>&, const T*, const T*, T*, T*);                \
  template void launch_phase_ac<T>(const Launch<T>&, const T*, const T*, const T*, const T*, \
                                   const T*, T*, T*, T*, T*);                                \
  template void launch_phase_b2<T>(const Launch<T>&, const T*, const T*, const T*, T*);      \
  template void launch_phase_cg1<T>(const Launch<T>&, const T*, const T*, const T*, T*, T*,  \
                                    T*, T*, T*);                                             \
  template void launch_cg_b<T>(const Launch<T>&, T*, const T*, T*, const T*);                \
  template void launch_fill<T>(size_t, T*, T, hipStream_t);
WFA_INST(double)
WFA_INST(float)
#undef WFA_INST
template void launch_residual<double>(const Launch<double>&, const double*, const double*,
                                      float*, float*, Scalars*, int, int, const Scalars*);
template void launch_residual<float>(const Launch<double>&, const float*, const float*, float*,
                                     float*, Scalars*, int, int, const Scalars*);

}  // namespace wfa
