// Device-side building blocks of libwfa: the 7-point operator on one cell,
// the z-marching LDS-staged plane engine, deterministic block and grid
// reductions, and the device scalar block of a Krylov solve.
//
// Operator (Woo et al. 2022, section 1.1.2, Eq. 3, generalised to a per-cell
// diffusivity, constant-velocity first-order upwind convection and per-face
// Dirichlet / zero-flux boundaries): for cell P and each face f,
//   interior:  D = cD * harmonic(kP, kN)   (cD = dt/h^2; CONST: D = dt*alpha/h^2)
//              diag += D + out_f,  coupling (D + in_f) with the neighbour,
//              where out_f = max(F_f, 0), in_f = max(-F_f, 0), F_f = dt (u.n_f)/h
//   Dirichlet: D = cD * kP at distance h;  diag += D + out_f,
//              b += (D + in_f) * value_f
//   zero-flux: nothing.
// diag starts at 1.  (A x)_P = diag x_P - sum_f coupling_f x_N.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>
#include <stdint.h>

namespace wfa {

constexpr int kThreads = 256;      // 4 wave64 per workgroup
constexpr int kWaves = kThreads / 64;
constexpr int kTX = 64;            // tile width in x: one wave spans one row
constexpr int kMaxReduce = 4;      // most global sums one pass reduces (per-tile
                                   // partial slots the workspace holds per tile)

// ---- device status of a solve ---------------------------------------------
enum DevStatus : int32_t {
  ST_RUN = 0,        // iterating
  ST_CONV = 1,       // converged
  ST_NOCONV = 2,     // iteration limit reached
  ST_NONFINITE = 3,  // NaN / Inf in a reduction
  ST_BZERO = 4,      // right-hand side is exactly zero: x = 0
  ST_BREAKDOWN = 5   // CG: non-positive curvature
};

// Scalars of one Krylov solve, resident in device memory.  Written only by
// the last workgroup of a phase launch (or by one thread of a persistent
// launch between grid barriers); read by every workgroup of the next phase.
struct alignas(64) Scalars {
  double rho, rho_prev, alpha, omega, beta;
  double bb, rr, tol;          // ||b||^2, last ||r||^2, relative tolerance
  double sigma, ts, tt, rr0;   // last reduced values (diagnostics / trace)
  double scale, inv_scale;     // mixed precision: residual scaling by 2^-e
  double guard;                // > 0: stop (diverged) once ||r||^2 > guard * ||r0||^2
  double rr_min;               // smallest ||r||^2 so far (textbook BiCGStab) ...
  int32_t status, iter, maxit, first, restart, szero, x_zero, force_bd;
  uint32_t counter;            // last-workgroup arrival counter (self-resetting)
  int32_t restart_pending;     // two-reduction BiCGStab: restart after the update
  int32_t diverged;            // set with ST_NOCONV when the guard tripped
  int32_t it_min;              // ... and the iteration that reached it
  int32_t force_div;           // n > 0: declare the solve diverged at iteration n (test hook)
  int32_t stage;               // CG with one reduction: 0 w0 = A r0, 1 first update, 2 steady
  int32_t pad[2];
};
static_assert(sizeof(Scalars) == 192, "the scalar block is three 64-byte lines");

// Grid-wide barrier state of a persistent launch (self-resetting count).
struct GridBarrier {
  uint32_t count, gen, timeout, pad;
};

// ---- geometry and operator constants (kernel arguments, by value) ----------
struct Geo {
  int nx, ny, nz;
  int tiles_x, tiles_y, zchunks, zc;  // tile grid; zc = planes per tile
  int ntiles;                         // tiles_x * tiles_y * zchunks
  long long plane;                    // nx * ny
};

template <typename T>
struct Op {
  T cD;            // dt/h^2 (CELL) or dt*alpha/h^2 (CONST)
  T in[6];         // inflow coupling per face:  max(-F_f, 0)
  T out[6];        // outflow diagonal per face: max( F_f, 0)
  T bval[6];       // Dirichlet ghost values
  uint32_t dir;    // bit f set: face f is Dirichlet
  uint32_t jac;    // 1: the Krylov operator is D^{-1} A (left Jacobi scaling)
  uint32_t conv;   // 1: some face has a convective term (in[f] or out[f] != 0)
};

// Builds of the cell operator (cell_apply's FORM): the general one, and two
// that leave out terms an operator does not have -- the Jacobi scaling
// select, and also the convective terms -- for fewer vector instructions.
// Each gives the general build's values bit for bit on the operators it is
// chosen for (op_form).
enum OpForm : int { kFormDiffusion = 0, kFormConvection = 1, kFormGeneral = 2 };

template <typename T>
__host__ __device__ inline int op_form(const Op<T>& op) {
  if (op.jac) return kFormGeneral;
  return op.conv ? kFormConvection : kFormDiffusion;
}

// Reciprocal of a positive normal number: the hardware estimate (relative
// error 2^-24.4 at most, measured over sums of two FP32 diffusivities) refined
// by one Newton step, which squares the error: 2^-48.7, some 20 ulp.  The
// harmonic-mean faces need no IEEE-exact division (the operator's relative
// error stays near 1e-15), and a second step, which rounds correctly, costs
// 6% of the FP64 pass without the update's streams.
__device__ __forceinline__ double pos_rcp(double a) {
  const double y = __builtin_amdgcn_rcp(a);
  const double e = __builtin_fma(-a, y, 1.0);
  return __builtin_fma(y, e, y);
}
__device__ __forceinline__ float pos_rcp(float a) {
  float y = __builtin_amdgcn_rcpf(a);
  const float e = __builtin_fmaf(-a, y, 1.0f);
  return __builtin_fmaf(y, e, y);
}

__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// Faces: 0 x-, 1 x+, 2 y-, 3 y+, 4 z-, 5 z+.  `inside` bit f: the neighbour
// across face f exists.
// Returns (A x)_P, or (A x)_P / A[P,P] when op.jac; the diagonal in `dg`.
// The operation sequence is pinned (explicit fused multiply-adds, no other
// contraction), so every kernel that applies the operator -- one pass per
// phase, persistent, batched, several explicit steps per pass -- rounds
// identically.
// kz: with `carry`, the z- face's harmonic mean on entry (the previous
// plane's z+ face: the same two diffusivities, and the products of two FP32
// values are exact, so the value is the one this call would form); the z+
// face's on exit.
// FORM = kFormConvection leaves out the Jacobi scaling select, for an
// operator without scaling; kFormDiffusion also the convective terms, for
// an operator without them (op_form(op) picks): with in[f] = out[f] = 0
// each fma(cD, kf, 0) is the product cD kf rounded once, so every value is
// bit for bit the general build's.
template <typename T, bool CELL, int FORM = kFormGeneral>
__device__ __forceinline__ T cell_apply(const Op<T>& op, T c, const T nb[6], T kP,
                                        const T kN[6], uint32_t inside, T& dg, T& kz,
                                        bool carry) {
#pragma clang fp contract(off)
  T diag = T(1), acc = T(0);
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    if (inside & (1u << f)) {
      constexpr bool CONV = FORM != kFormDiffusion;
      T d_out, d_in;  // D + max(F,0), D + max(-F,0)
      if (CELL) {
        const T kf = (f == 4 && carry) ? kz
                                       : T(2) * kP * kN[f] * pos_rcp(kP + kN[f]);  // harmonic mean
        if (f == 5) kz = kf;
        if (CONV) {
          d_out = fma_t(op.cD, kf, op.out[f]);
          d_in = fma_t(op.cD, kf, op.in[f]);
        } else {
          d_out = d_in = op.cD * kf;
        }
      } else if (CONV) {
        d_out = op.cD + op.out[f];
        d_in = op.cD + op.in[f];
      } else {
        d_out = d_in = op.cD;
      }
      diag += d_out;
      acc = fma_t(d_in, nb[f], acc);
    } else if (op.dir & (1u << f)) {
      if (FORM != kFormDiffusion) diag += CELL ? fma_t(op.cD, kP, op.out[f]) : op.cD + op.out[f];
      else diag += CELL ? op.cD * kP : op.cD;
    }
  }
  dg = diag;
  const T y = fma_t(diag, c, -acc);
  if (FORM != kFormGeneral) return y;
  return op.jac ? y * pos_rcp(diag) : y;
}

template <typename T, bool CELL, int FORM = kFormGeneral>
__device__ __forceinline__ T cell_apply(const Op<T>& op, T c, const T nb[6], T kP,
                                        const T kN[6], uint32_t inside, T& dg) {
  T kz = T(0);
  return cell_apply<T, CELL, FORM>(op, c, nb, kP, kN, inside, dg, kz, false);
}

// The diffusion-only operator (op_form(op) == kFormDiffusion, per-cell
// diffusivity) split into its coefficients and their application, for a
// pass that applies A to two vectors on the same cells: D[f] = cD
// harmonic(kP, kN[f]) on faces with a neighbour and 0 on the others, and
// the diagonal 1 + sum_f (D[f], or cD kP on a Dirichlet face) summed in
// face order.  With `carry` the z- face takes dz (the previous plane's z+
// coefficient, the same value: see cell_apply); dz returns this plane's z+
// one.  apply_coefs(D, diag, c, nb) then gives cell_apply's value bit for
// bit: the zero coefficients add fma(0, nb, acc) = acc for finite nb.
template <typename T>
__device__ __forceinline__ T diffusion_coefs(const Op<T>& op, T kP, const T kN[6],
                                             uint32_t inside, T (&D)[6], T& dz, bool carry) {
#pragma clang fp contract(off)
  T diag = T(1);
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    T d = T(0);
    if (inside & (1u << f)) {
      d = (f == 4 && carry) ? dz : op.cD * (T(2) * kP * kN[f] * pos_rcp(kP + kN[f]));
      diag += d;
    } else if (op.dir & (1u << f)) {
      diag += op.cD * kP;
    }
    if (f == 5) dz = d;
    D[f] = d;
  }
  return diag;
}

template <typename T>
__device__ __forceinline__ T apply_coefs(const T (&D)[6], T diag, T c, const T nb[6]) {
#pragma clang fp contract(off)
  T acc = T(0);
#pragma unroll
  for (int f = 0; f < 6; ++f) acc = fma_t(D[f], nb[f], acc);
  return fma_t(diag, c, -acc);
}

// Dirichlet contribution of cell P to the right-hand side.
template <typename T, bool CELL>
__device__ __forceinline__ T cell_bterm(const Op<T>& op, T kP, uint32_t inside) {
#pragma clang fp contract(off)
  T s = T(0);
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    if (!(inside & (1u << f)) && (op.dir & (1u << f))) {
      const T d_in = CELL ? fma_t(op.cD, kP, op.in[f]) : op.cD + op.in[f];
      s = fma_t(d_in, op.bval[f], s);
    }
  }
  return s;
}

// Coefficients of a constant-diffusivity operator at a cell whose six
// neighbours all exist, formed in the order cell_apply forms them, so that
// cell_apply_interior returns cell_apply's value bit for bit.
template <typename T>
struct InteriorCoef {
  T coef[6];  // D + in[f]
  T diag;     // 1 + sum_f (D + out[f]), summed in face order
};

template <typename T>
__device__ __forceinline__ InteriorCoef<T> interior_coef(const Op<T>& op) {
#pragma clang fp contract(off)
  InteriorCoef<T> k;
  T diag = T(1);
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    diag += op.cD + op.out[f];
    k.coef[f] = op.cD + op.in[f];
  }
  k.diag = diag;
  return k;
}

// (A x)_P of a constant-diffusivity operator at a cell with all six
// neighbours inside and no Jacobi scaling: cell_apply's operation sequence
// with the face tests resolved.
template <typename T>
__device__ __forceinline__ T cell_apply_interior(const InteriorCoef<T>& k, T c, const T nb[6]) {
#pragma clang fp contract(off)
  T acc = T(0);
#pragma unroll
  for (int f = 0; f < 6; ++f) acc = fma_t(k.coef[f], nb[f], acc);
  return fma_t(k.diag, c, -acc);
}

// Shadow residual computed from the cell index instead of stored: the
// 32-bit PCG hash of the index (an LCG step, state = i * 747796405 +
// 2891336453, then PCG's RXS-M-XS output permutation; O'Neill 2014), whose
// top 24 bits give r^_i = (h >> 8) 2^-23 - 1 in [-1, 1), exact in FP32 and
// FP64.  Any r^ with (r^, r0) != 0 serves BiCGStab; this one costs no HBM
// traffic where r^ = r0 costs one stream per reduction pass.
__device__ __forceinline__ uint32_t pcg_hash(uint32_t i) {
  const uint32_t state = i * 747796405u + 2891336453u;
  const uint32_t word = ((state >> ((state >> 28u) + 4u)) ^ state) * 277803737u;
  return (word >> 22u) ^ word;
}
template <typename T>
__device__ __forceinline__ T hashed_shadow(size_t i) {
  return T(pcg_hash((uint32_t)i) >> 8) * T(1.0 / 8388608.0) - T(1);
}

// One explicit forward-time step of cell P from its old value c and (A x)_P.
template <typename T>
__device__ __forceinline__ T explicit_update(T c, T Au, T bterm) {
#pragma clang fp contract(off)
  return c - (Au - c) + bterm;
}

__device__ __forceinline__ uint32_t inside_mask(const Geo& g, int i, int j, int k) {
  return (i > 0 ? 1u : 0u) | (i < g.nx - 1 ? 2u : 0u) | (j > 0 ? 4u : 0u) |
         (j < g.ny - 1 ? 8u : 0u) | (k > 0 ? 16u : 0u) | (k < g.nz - 1 ? 32u : 0u);
}

// ---- XCD-aware workgroup -> tile mapping ------------------------------------
// Workgroups are dispatched round-robin over the 8 XCDs (each with its own
// L2).  Give each XCD a contiguous range of tiles so that tiles sharing halo
// rows run on the same L2.
__device__ __forceinline__ int xcd_tile(int b, int nb) {
  const int q = nb >> 3, rem = nb & 7;
  const int xcd = b & 7, slot = b >> 3;
  const int start = xcd < rem ? xcd * (q + 1) : rem * (q + 1) + (xcd - rem) * q;
  return start + slot;
}

// ---- reductions ---------------------------------------------------------------
// One term of a dot product, accumulated in FP64 with a single rounding.  It
// is an explicit fused multiply-add because, left to the compiler, whether a
// product and the sum it feeds are fused depends on how the code around them
// is laid out (both must sit in one basic block), so two builds of the same
// pass could round a partial sum differently.
__device__ __forceinline__ void dot_acc(double& a, double x, double y) {
  a = __builtin_fma(x, y, a);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

// Deterministic block sum of NV values; result valid in thread 0.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* red /*LDS kWaves*NV*/) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < NV; ++q) v[q] = wave_sum(v[q]);
  if (lane == 0) {
#pragma unroll
    for (int q = 0; q < NV; ++q) red[wave * NV + q] = v[q];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      double s = 0.0;
      for (int w = 0; w < kWaves; ++w) s += red[w * NV + q];
      v[q] = s;
    }
  }
  __syncthreads();
}

// Fixed-order sum of partials[q*n + t] over t, by one workgroup; result in
// thread 0.  Identical for any launch that produced the same partials.  The
// loads are agent-scope atomics: they read the coherent copy whichever XCD
// wrote it.
template <int NV>
__device__ __forceinline__ void reduce_partials(double* partials, int n, double (&out)[NV],
                                                double* red) {
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    const double* pq = partials + (size_t)q * n;
    double s = 0.0;
    int t = threadIdx.x;
    // batches of 8 loads in flight, summed in index order
    for (; t + 7 * kThreads < n; t += 8 * kThreads) {
      double a[8];
#pragma unroll
      for (int u = 0; u < 8; ++u)
        a[u] = __hip_atomic_load(pq + t + u * kThreads, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
      for (int u = 0; u < 8; ++u) s += a[u];
    }
    for (; t < n; t += kThreads)
      s += __hip_atomic_load(pq + t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    out[q] = s;
  }
  block_sum<NV>(out, red);
}

// Publish this workgroup's partial sums; the last workgroup to arrive
// reduces all of them in fixed order and calls fin(sums) in thread 0.
//
// Cross-XCD ordering without cache-wide fences: the partials are written
// with agent-scope atomic stores (coherent across the XCDs' L2s), the
// writer waits for their completion before its arrival increments the
// counter, and the last workgroup reads them back with agent-scope atomic
// loads.  A release/acquire fence would instead write back and invalidate
// the whole L2 of the XCD at every workgroup's end, evicting the halo
// planes the neighbouring tiles are about to read.
template <int NV, class Fin>
__device__ __forceinline__ void publish_and_finalize(double (&v)[NV], int slot, int nslots,
                                                     double* partials, Scalars* sc,
                                                     double* red, Fin fin) {
  __shared__ int last;
  block_sum<NV>(v, red);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < NV; ++q)
      __hip_atomic_store(&partials[(size_t)q * nslots + slot], v[q], __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    const uint32_t prev = __hip_atomic_fetch_add(&sc->counter, 1u, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT);
    last = (prev == (uint32_t)(nslots - 1));
  }
  __syncthreads();
  if (!last) return;
  double s[NV];
  reduce_partials<NV>(partials, nslots, s, red);
  if (threadIdx.x == 0) {
    fin(s);
    __hip_atomic_store(&sc->counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// ---- grid-wide barrier of a persistent (cooperative) launch -------------------
// Sense-free barrier: arrivals counted in `count`, release by bumping `gen`.
// Waits are bounded: after `spin_limit` polls the waiter records a timeout
// and leaves, so every wave of the grid always exits.
__device__ __forceinline__ bool grid_sync(GridBarrier* b, uint32_t nblocks, int spin_limit) {
  __shared__ int ok;
  // every wave's stores have reached its XCD's L2 ...
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();
  if (threadIdx.x == 0) {
    // ... one wave writes that L2 back (release) for the whole workgroup
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    int good = 1;
    const uint32_t gen = __hip_atomic_load(&b->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    const uint32_t arrived =
        __hip_atomic_fetch_add(&b->count, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (arrived == nblocks - 1) {
      __hip_atomic_store(&b->count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
      __hip_atomic_store(&b->gen, gen + 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      int spins = 0;
      while (__hip_atomic_load(&b->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gen) {
        __builtin_amdgcn_s_sleep(1);
        if (++spins > spin_limit) {
          __hip_atomic_store(&b->timeout, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          good = 0;
          break;
        }
      }
    }
    // and invalidates stale lines of the CU's L1 and the XCD's L2 (acquire)
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    ok = good;
  }
  __syncthreads();
  return ok != 0;
}

// One workgroup's partial sums into slot `slot` of a region of NV x nslots
// values (the layout publish_and_finalize uses), without the arrival count:
// a persistent launch reduces them after a grid barrier instead.
template <int NV>
__device__ __forceinline__ void store_partial(double* region, int nslots, int slot,
                                              const double (&v)[NV]) {
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < NV; ++q)
      __hip_atomic_store(&region[(size_t)q * nslots + slot], v[q], __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
  }
}

// ---- the z-marching plane engine ----------------------------------------------
//
// A tile is kTX x TY cells of the x-y plane times zc planes in z.  Each of
// the 4 waves owns RY consecutive rows; lane l owns column x0 + l.  For each
// output plane k the staged vector u (computed on the fly from the phase's
// input arrays, also on the x-y halo) is written to an LDS plane with a
// one-cell halo; the x and y neighbours come from LDS and the z neighbours
// from registers (u at k-1 and k+1).  Loads for plane k+2 and the
// epilogue's loads for plane k+1 are issued before plane k is computed, so
// one plane of work hides each load's latency.
//
// Phase policy Ph provides:
//   struct Raw;  Raw fetch(size_t idx);  T-like combine(const Raw&)  -- stage of
//                                         halo cells and the z-halo plane k0-1
//   struct ORaw; ORaw fetch_own(size_t idx);                        -- own cells
//   St combine_own(const ORaw&, size_t idx, acc)  -- own cells of output planes;
//                                         may store and accumulate (once per cell)
//   T value_own(const ORaw&)              -- own cells of the z-halo plane k1
//   St;  static T val(const St&)        -- staged struct and its stencil value
//   struct ERaw; ERaw efetch(size_t idx);                         -- epilogue loads
//   static constexpr int NV;                                      -- dot partials
//   void epilogue(size_t idx, const St& u, T Au, T kP, uint32_t inside,
//                 const ERaw&, double (&acc)[NV]);                -- stores + dots
template <int RY>
struct TileShape {
  static constexpr int TY = kWaves * RY;
  static constexpr int LW = kTX + 2;
  static constexpr int LH = TY + 2;
  static constexpr int NHALO = 2 * kTX + 2 * TY;
  static_assert(NHALO <= kThreads, "halo must fit one cell per thread");
};

// Phases opt in to carrying the z face coefficient with a static member
// kCarryZ = true; the others do not.
template <class Ph, class = void>
struct carry_z { static constexpr bool value = false; };
template <class Ph>
struct carry_z<Ph, std::void_t<decltype(Ph::kCarryZ)>> {
  static constexpr bool value = Ph::kCarryZ;
};

template <typename T, bool CELL, int RY, class Ph, int FORM = kFormGeneral>
__device__ __forceinline__ void march_tile(const Geo& g, const Op<T>& op,
                                           const float* __restrict__ kappa, int tile,
                                           Ph& ph, double (&acc)[Ph::NV], T* su,
                                           float* sk) {
  using TS = TileShape<RY>;
  constexpr int TY = TS::TY, LW = TS::LW, LH = TS::LH;
  constexpr int PD = Ph::PD;  // planes of loads in flight ahead of the compute
  static_assert(PD == 1 || PD == 2, "prefetch depth 1 or 2");
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int tx = tile % g.tiles_x;
  const int rest = tile / g.tiles_x;
  const int ty = rest % g.tiles_y;
  const int tz = rest / g.tiles_y;
  const int x0 = tx * kTX, y0 = ty * TY;
  const int k0 = tz * g.zc;
  const int k1 = min(k0 + g.zc, g.nz);
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const size_t plane = (size_t)g.plane;

  // own cells
  const int i = x0 + lane;
  bool own[RY];
  int poff[RY];      // offset inside a plane
  int lidx[RY];      // LDS index
  uint32_t ins_xy[RY];
#pragma unroll
  for (int r = 0; r < RY; ++r) {
    const int j = y0 + wave * RY + r;
    own[r] = (i < nx) && (j < ny);
    poff[r] = own[r] ? i + nx * j : 0;
    lidx[r] = (wave * RY + r + 1) * LW + lane + 1;
    ins_xy[r] = (i > 0 ? 1u : 0u) | (i < nx - 1 ? 2u : 0u) | (j > 0 ? 4u : 0u) |
                (j < ny - 1 ? 8u : 0u);
  }
  // halo cell of this thread
  int hl = -1, hoff = 0;
  bool hval = false;
  {
    const int hs = threadIdx.x;
    int hi = 0, hj = 0;
    if (hs < kTX) { hi = x0 + hs; hj = y0 - 1; hl = hs + 1; }
    else if (hs < 2 * kTX) { hi = x0 + hs - kTX; hj = y0 + TY; hl = (LH - 1) * LW + hs - kTX + 1; }
    else if (hs < 2 * kTX + TY) { hi = x0 - 1; hj = y0 + hs - 2 * kTX; hl = (hs - 2 * kTX + 1) * LW; }
    else if (hs < TS::NHALO) { hi = x0 + kTX; hj = y0 + hs - 2 * kTX - TY; hl = (hs - 2 * kTX - TY + 1) * LW + LW - 1; }
    if (hl >= 0) {
      hval = hi >= 0 && hi < nx && hj >= 0 && hj < ny;
      hoff = hval ? hi + nx * hj : 0;
    }
  }

  using Raw = typename Ph::Raw;
  using ORaw = typename Ph::ORaw;
  using ERaw = typename Ph::ERaw;
  // Loads of one plane that are in flight: own cells' stage inputs and
  // diffusivity, the halo cell's, and the epilogue's inputs.
  struct PlaneLoads {
    ORaw o[RY];
    float ko[RY];
    Raw h;
    float kh;
    ERaw e[RY];
  };
  // Issue the loads of plane kp (stage inputs up to the z-halo plane k1,
  // halo and epilogue inputs for output planes only).
  auto issue = [&](PlaneLoads& S, int kp) {
    const bool stage = (kp <= k1) && (kp < nz);
#pragma unroll
    for (int r = 0; r < RY; ++r) {
      if (stage && own[r]) {
        const size_t idx = (size_t)kp * plane + poff[r];
        S.o[r] = ph.fetch_own(idx);
        if (CELL) S.ko[r] = kappa[idx];
      }
      if (kp < k1 && own[r]) S.e[r] = ph.efetch((size_t)kp * plane + poff[r]);
    }
    if (hval && kp < k1) {
      const size_t idx = (size_t)kp * plane + hoff;
      S.h = ph.fetch(idx);
      if (CELL) S.kh = kappa[idx];
    }
  };

  using St = typename Ph::St;  // staged value (and what the epilogue needs of it)
  T up[RY];
  St uc[RY];
  float kpv[RY], kcv[RY];   // diffusivity stays FP32 (as stored) until used
  T hc = T(0);
  float kh = 1.f;
  ERaw ec[RY];
  // A phase that opts in (kCarryZ) carries each cell's z+ face coefficient
  // to the next plane's z- face: one harmonic mean less per cell, the same
  // value bit for bit.  It pays in the passes with few streams; in the
  // fused update pass the extra registers cost more than it saves.
  constexpr bool CZ = carry_z<Ph>::value;
  T kz[RY];                 // z+ face coefficient of the plane just computed
  bool carry = false;       // kz holds the next plane's z- face
#pragma unroll
  for (int r = 0; r < RY; ++r) kz[r] = T(0);

  // plane k0 - 1 (own cells only) and plane k0 (own + halo), staged directly
#pragma unroll
  for (int r = 0; r < RY; ++r) {
    up[r] = T(0);
    kpv[r] = 1.f;
    if (k0 > 0 && own[r]) {
      const size_t idx = (size_t)(k0 - 1) * plane + poff[r];
      up[r] = Ph::val(ph.combine(ph.fetch(idx)));
      if (CELL) kpv[r] = kappa[idx];
    }
    uc[r] = St{};
    kcv[r] = 1.f;
    if (own[r]) {
      const size_t idx = (size_t)k0 * plane + poff[r];
      uc[r] = ph.combine_own(ph.fetch_own(idx), idx, acc);
      if (CELL) kcv[r] = kappa[idx];
      ec[r] = ph.efetch(idx);
    }
  }
  if (hval) {
    const size_t idx = (size_t)k0 * plane + hoff;
    hc = Ph::val(ph.combine(ph.fetch(idx)));
    if (CELL) kh = kappa[idx];
  }
  PlaneLoads L0, L1;
  issue(L0, k0 + 1);
  if (PD == 2) issue(L1, k0 + 2);

  int buf = 0;
  // One output plane k; S holds the loads of plane k+1 and is refilled
  // with plane k+1+PD.
  auto step = [&](int k, PlaneLoads& S) {
    T* Lu = su + buf * (LH * LW);
    float* Lk = CELL ? sk + buf * (LH * LW) : nullptr;
#pragma unroll
    for (int r = 0; r < RY; ++r) {
      Lu[lidx[r]] = Ph::val(uc[r]);
      if (CELL) Lk[lidx[r]] = kcv[r];
    }
    if (hl >= 0) {
      Lu[hl] = hval ? hc : T(0);
      if (CELL) Lk[hl] = hval ? kh : 1.f;
    }
    __syncthreads();

    // stage plane k + 1 from its (now due) loads; an output plane's own
    // cells go through combine_own (which may store and accumulate), the
    // z-halo plane k1 only yields the stencil value
    const bool has_n = (k + 1 <= k1) && (k + 1 < nz);
    const bool out_n = k + 1 < k1;
    St un[RY];
    T unv[RY];
    float knv[RY];
    ERaw en[RY];
#pragma unroll
    for (int r = 0; r < RY; ++r) {
      un[r] = St{};
      unv[r] = T(0);
      knv[r] = 1.f;
      if (has_n && own[r]) {
        if (out_n) {
          un[r] = ph.combine_own(S.o[r], (size_t)(k + 1) * plane + poff[r], acc);
          unv[r] = Ph::val(un[r]);
        } else {
          unv[r] = ph.value_own(S.o[r]);
        }
        if (CELL) knv[r] = S.ko[r];
      }
      en[r] = S.e[r];
    }
    T hn = T(0);
    float khn = 1.f;
    if (hval && k + 1 < k1) {
      hn = Ph::val(ph.combine(S.h));
      if (CELL) khn = S.kh;
    }
    issue(S, k + 1 + PD);

    // compute plane k
    const uint32_t ins_z = (k > 0 ? 16u : 0u) | (k < nz - 1 ? 32u : 0u);
#pragma unroll
    for (int r = 0; r < RY; ++r) {
      if (own[r]) {
        const int l = lidx[r];
        T nb[6] = {Lu[l - 1], Lu[l + 1], Lu[l - LW], Lu[l + LW], up[r], unv[r]};
        T kn6[6];
        if (CELL) {
          kn6[0] = (T)Lk[l - 1]; kn6[1] = (T)Lk[l + 1]; kn6[2] = (T)Lk[l - LW];
          kn6[3] = (T)Lk[l + LW]; kn6[4] = (T)kpv[r]; kn6[5] = (T)knv[r];
        } else {
#pragma unroll
          for (int f = 0; f < 6; ++f) kn6[f] = T(1);
        }
        const uint32_t ins = ins_xy[r] | ins_z;
        T dg;
        T Au;
        if constexpr (CZ)
          Au = cell_apply<T, CELL, FORM>(op, Ph::val(uc[r]), nb, (T)kcv[r], kn6, ins, dg, kz[r],
                                         carry);
        else
          Au = cell_apply<T, CELL, FORM>(op, Ph::val(uc[r]), nb, (T)kcv[r], kn6, ins, dg);
        ph.epilogue((size_t)k * plane + poff[r], uc[r], Au, (T)kcv[r], ins, ec[r], dg, acc);
      }
    }
    // rotate
#pragma unroll
    for (int r = 0; r < RY; ++r) {
      up[r] = Ph::val(uc[r]); uc[r] = un[r];
      kpv[r] = kcv[r]; kcv[r] = knv[r];
      ec[r] = en[r];
    }
    hc = hn; kh = khn;
    carry = true;
    buf ^= 1;
  };

  for (int k = k0; k < k1;) {
    step(k, L0);
    ++k;
    if (PD == 2 && k < k1) {
      step(k, L1);
      ++k;
    }
  }
  __syncthreads();  // LDS planes are reused by the next tile of this workgroup
}

}  // namespace wfa
