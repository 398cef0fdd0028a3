// Pass AC of the two-reduction BiCGStab with t = A s formed again instead of
// read back.
//
// Pass B2 forms t = A s (s = r - alpha v) for its reductions (t,s), (t,t),
// (rh,s), (rh,t); the usual pass AC reads that t back to apply the update
// r' = s - omega t.  Here pass B2 stores nothing and this pass forms t again
// from r and v.  t at a cell needs s on the cell's six neighbours, and
// v' = A p' needs p' = r' + beta (p - omega v) on the tile's one-cell halo,
// so s is staged on a two-cell halo (the ring at distance two and its four
// diagonal corners), t, r' and p' are formed on the one-cell halo too, and
// v' on the tile.  Two levels march along z: level 1 (t, r', p', x') runs
// one plane ahead of level 2 (v' = A p').  s is staged with the operations
// pass B2 uses and the operator is cell_apply, so t is bitwise the value
// pass B2 reduced; every store and every partial sum, accumulated in the
// same order, is bitwise that of the pass that reads t.  Per cell and
// iteration two vector streams fewer cross HBM (t written by pass B2, read
// by pass AC).
//
// Tile: kTX x TY cells of a plane (4 waves, RY rows each, one column per
// lane) times the zc planes [k0, k1).  s is staged on planes [k0-2, k1+1]
// for the tile's own cells, [k0-1, k1] for the one-cell halo and [k0, k1-1]
// for the distance-two ring.  Level 1 runs on planes [k0-1, k1] for own
// cells (stores on output planes only) and on the output planes for the
// one-cell halo; level 2 on the output planes.  LDS holds s in a ring of 3
// planes, the diffusivity in a ring of 4 and p' in a ring of 2, each with a
// two-cell halo: with these depths one barrier per plane orders every write
// after the last read of its slot.
//
// With the diffusion-only operator the two products on an own cell share
// their coefficients: level 1 forms each face's coefficient and the
// diagonal once (diffusion_coefs, the z- face carried from the plane below)
// for t, keeps them, and level 2 applies them to p' a plane later
// (apply_coefs) -- the same values bit for bit, and no harmonic mean in
// level 2.
#include <hip/hip_runtime.h>

#include "device.hpp"
#include "internal.hpp"
#include "phases.hpp"

namespace wfa {

template <typename T>
struct ActArgs {
  const T* __restrict__ r;
  const T* __restrict__ v;
  const T* __restrict__ p;
  const T* __restrict__ rh;   // stored shadow residual (unused when hashed)
  T* __restrict__ x;
  T* __restrict__ r_out;
  T* __restrict__ p_out;
  T* __restrict__ v_out;
  int hashed;
};

template <int RY>
struct ActShape {
  static constexpr int TY = kWaves * RY;
  static constexpr int SW = kTX + 4;              // plane row with a two-cell halo
  static constexpr int SH = TY + 4;
  static constexpr int SP = SW * SH;
  static constexpr int NH1 = 2 * kTX + 2 * TY;     // one-cell halo
  static constexpr int NH2 = NH1 + 4;              // distance-two ring and corners
  static_assert(NH2 <= kThreads, "each thread takes at most one cell of each ring");
};

// Local coordinates (lx, ly) of ring cell `hs`; lx in [-2, kTX+1], ly in
// [-2, TY+1].
template <int RY>
__device__ __forceinline__ bool ring1_cell(int hs, int& lx, int& ly) {
  using S = ActShape<RY>;
  if (hs < kTX) { lx = hs; ly = -1; return true; }
  if (hs < 2 * kTX) { lx = hs - kTX; ly = S::TY; return true; }
  if (hs < 2 * kTX + S::TY) { lx = -1; ly = hs - 2 * kTX; return true; }
  if (hs < S::NH1) { lx = kTX; ly = hs - 2 * kTX - S::TY; return true; }
  return false;
}
template <int RY>
__device__ __forceinline__ bool ring2_cell(int hs, int& lx, int& ly) {
  using S = ActShape<RY>;
  if (hs < kTX) { lx = hs; ly = -2; return true; }
  if (hs < 2 * kTX) { lx = hs - kTX; ly = S::TY + 1; return true; }
  if (hs < 2 * kTX + S::TY) { lx = -2; ly = hs - 2 * kTX; return true; }
  if (hs < S::NH1) { lx = kTX + 1; ly = hs - 2 * kTX - S::TY; return true; }
  if (hs < S::NH2) {
    const int c = hs - S::NH1;
    lx = (c & 1) ? kTX : -1;
    ly = (c & 2) ? S::TY : -1;
    return true;
  }
  return false;
}

template <typename T, bool CELL, int RY, int FORM>
__global__ void __launch_bounds__(kThreads)
k_phase_act(Geo g, Op<T> op, const float* __restrict__ kappa, ActArgs<T> a, double* partials,
            Scalars* sc) {
  using AS = ActShape<RY>;
  constexpr int TY = AS::TY, SW = AS::SW, SP = AS::SP;
  __shared__ T sS[3 * SP];
  __shared__ float sK[CELL ? 4 * SP : 1];
  __shared__ T sP[2 * SP];
  __shared__ double red[kWaves * 3];
  // an iteration pass: skipped once its solve has stopped or awaits a restart
  if (sc->status != ST_RUN || sc->restart) return;
  const T alpha = (T)sc->alpha, omega = (T)sc->omega, beta = (T)sc->beta;
  const bool first = sc->first != 0;   // (re)start: p' = r' = r, nothing else read
  const bool xzero = sc->x_zero != 0;  // x is still the zero initial guess

  const int tile = xcd_tile(blockIdx.x, gridDim.x);
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

  // ---- the cells of this thread: RY own cells, one cell of each ring ----
  bool own[RY];
  int poff[RY], lo[RY];
  uint32_t mo[RY];
  {
    const int i = x0 + lane;
#pragma unroll
    for (int r = 0; r < RY; ++r) {
      const int j = y0 + wave * RY + r;
      own[r] = i < nx && j < ny;
      poff[r] = own[r] ? i + nx * j : 0;
      lo[r] = (wave * RY + r + 2) * SW + lane + 2;
      mo[r] = (i > 0 ? 1u : 0u) | (i < nx - 1 ? 2u : 0u) | (j > 0 ? 4u : 0u) |
              (j < ny - 1 ? 8u : 0u);
    }
  }
  int l1 = -1, off1 = 0, l2 = -1, off2 = 0;
  bool v1 = false, v2 = false;
  uint32_t m1 = 0;
  {
    int lx = 0, ly = 0;
    if (ring1_cell<RY>(threadIdx.x, lx, ly)) {
      const int i = x0 + lx, j = y0 + ly;
      l1 = (ly + 2) * SW + lx + 2;
      v1 = i >= 0 && i < nx && j >= 0 && j < ny;
      off1 = v1 ? i + nx * j : 0;
      m1 = (i > 0 ? 1u : 0u) | (i < nx - 1 ? 2u : 0u) | (j > 0 ? 4u : 0u) |
           (j < ny - 1 ? 8u : 0u);
    }
    if (ring2_cell<RY>(threadIdx.x, lx, ly)) {
      const int i = x0 + lx, j = y0 + ly;
      l2 = (ly + 2) * SW + lx + 2;
      v2 = i >= 0 && i < nx && j >= 0 && j < ny;
      off2 = v2 ? i + nx * j : 0;
    }
  }

  // ---- the loads of one plane q ----
  // own cells: r, v and kappa where s is staged ([k0-2, k1+1]), p on the
  // level-1 planes [k0-1, k1], x and a stored r^ on output planes; one-cell
  // halo: r, v, kappa on [k0-1, k1], p on output planes; distance-two ring:
  // r, v, kappa on output planes.  On a (re)start only r is read.
  struct Loads {
    T r[RY], v[RY], p[RY], x[RY], rh[RY];
    float k[RY];
    T hr, hv, hp;
    float hk;
    T qr, qv;
    float qk;
  };
  auto load = [&](Loads& L, int q) {
    const bool in = q >= 0 && q < nz;
    const bool s_own = in && q >= k0 - 2 && q <= k1 + 1;
    const bool lvl1 = in && q >= k0 - 1 && q <= k1;
    const bool outp = in && q >= k0 && q < k1;
    const size_t base = (size_t)(in ? q : 0) * plane;
#pragma unroll
    for (int r = 0; r < RY; ++r) {
      L.r[r] = T(0); L.v[r] = T(0); L.p[r] = T(0); L.x[r] = T(0); L.rh[r] = T(0);
      L.k[r] = 1.f;
      if (own[r] && s_own) {
        const size_t idx = base + poff[r];
        L.r[r] = a.r[idx];
        if (!first) L.v[r] = a.v[idx];
        if (CELL) L.k[r] = kappa[idx];
        if (lvl1 && !first) L.p[r] = a.p[idx];
        if (outp && !first && !xzero) L.x[r] = ld_once(a.x + idx);
        if (outp && !a.hashed) L.rh[r] = ld_once(a.rh + idx);
      }
    }
    L.hr = T(0); L.hv = T(0); L.hp = T(0); L.hk = 1.f;
    if (v1 && lvl1) {
      const size_t idx = base + off1;
      L.hr = a.r[idx];
      if (!first) L.hv = a.v[idx];
      if (CELL) L.hk = kappa[idx];
      if (outp && !first) L.hp = a.p[idx];
    }
    L.qr = T(0); L.qv = T(0); L.qk = 1.f;
    if (v2 && outp) {
      const size_t idx = base + off2;
      L.qr = a.r[idx];
      if (!first) L.qv = a.v[idx];
      if (CELL) L.qk = kappa[idx];
    }
  };

  // ---- register state, named relative to the output plane k of a step ----
  // (level 1 runs on k + 1, staging on k + 2)
  T s0[RY], s1[RY], s2[RY];                  // s on own cells at k, k+1, k+2
  float km[RY], kk0[RY], kk1[RY], kk2[RY];    // kappa at k-1 .. k+2
  T p1[RY], v1r[RY], x1[RY], rh1[RY];         // p, v, x, r^ at k+1
  T p2[RY], v2r[RY], x2[RY], rh2[RY];         // ... at k+2
  T rh0[RY];                                   // r^ at k
  T ppm[RY], pp0[RY], pp1[RY];                 // p' at k-1, k, k+1
  T hs0 = T(0), hs1 = T(0), hs2 = T(0);       // one-cell halo: s at k .. k+2
  float hk0 = 1.f, hk1 = 1.f, hk2 = 1.f;
  T hp1 = T(0), hv1 = T(0), hp2 = T(0), hv2 = T(0);
#pragma unroll
  for (int r = 0; r < RY; ++r) {
    s0[r] = s1[r] = s2[r] = T(0);
    km[r] = kk0[r] = kk1[r] = kk2[r] = 1.f;
    p1[r] = v1r[r] = x1[r] = rh1[r] = T(0);
    p2[r] = v2r[r] = x2[r] = rh2[r] = T(0);
    rh0[r] = ppm[r] = pp0[r] = pp1[r] = T(0);
  }
  double acc[3] = {0.0, 0.0, 0.0};  // (rh, v'), (rh, r'), (r', r')
  // shared coefficients of own cells (diffusion-only operator): those of
  // the plane level 1 just formed (n) and of the plane level 2 applies (o)
  constexpr bool SHARE = CELL && FORM == kFormDiffusion;
  T Dn[RY][6], dgn[RY], Do[RY][6], dgo[RY], dzc[RY];
  bool zcar = false;   // dzc holds the z+ coefficients of the last level-1 plane
#pragma unroll
  for (int r = 0; r < RY; ++r) {
    dgn[r] = dgo[r] = T(1);
    dzc[r] = T(0);
#pragma unroll
    for (int f = 0; f < 6; ++f) Dn[r][f] = Do[r][f] = T(0);
  }

  // stage plane q: s into LDS slot q and the "k+2" registers
  auto stage = [&](const Loads& L, int q) {
    T* S = sS + ((q + 3) % 3) * SP;
    float* K = CELL ? sK + ((q + 4) % 4) * SP : nullptr;
    const bool in = q >= 0 && q < nz;
#pragma unroll
    for (int r = 0; r < RY; ++r) {
      const bool ok = own[r] && in && q >= k0 - 2 && q <= k1 + 1;
      const T s = ok ? minus_ax(L.r[r], alpha, L.v[r]) : T(0);
      s2[r] = s;
      kk2[r] = L.k[r];
      p2[r] = L.p[r];
      v2r[r] = L.v[r];
      x2[r] = L.x[r];
      rh2[r] = (a.hashed && ok) ? hashed_shadow<T>((size_t)q * plane + poff[r]) : L.rh[r];
      S[lo[r]] = s;
      if (CELL) K[lo[r]] = L.k[r];
    }
    if (l1 >= 0) {
      const bool ok = v1 && in && q >= k0 - 1 && q <= k1;
      hs2 = ok ? minus_ax(L.hr, alpha, L.hv) : T(0);
      hk2 = L.hk;
      hp2 = L.hp;
      hv2 = L.hv;
      S[l1] = hs2;
      if (CELL) K[l1] = L.hk;
    }
    if (l2 >= 0) {
      const bool ok = v2 && in && q >= k0 && q < k1;
      S[l2] = ok ? minus_ax(L.qr, alpha, L.qv) : T(0);
      if (CELL) K[l2] = L.qk;
    }
  };
  // advance the output plane by one
  auto rotate = [&]() {
#pragma unroll
    for (int r = 0; r < RY; ++r) {
      s0[r] = s1[r]; s1[r] = s2[r];
      km[r] = kk0[r]; kk0[r] = kk1[r]; kk1[r] = kk2[r];
      p1[r] = p2[r]; v1r[r] = v2r[r]; x1[r] = x2[r];
      rh0[r] = rh1[r]; rh1[r] = rh2[r];
      ppm[r] = pp0[r]; pp0[r] = pp1[r];
      if (SHARE) {
        dgo[r] = dgn[r];
#pragma unroll
        for (int f = 0; f < 6; ++f) Do[r][f] = Dn[r][f];
      }
    }
    hs0 = hs1; hs1 = hs2;
    hk0 = hk1; hk1 = hk2;
    hp1 = hp2; hv1 = hv2;
  };
  // t = A s at LDS cell l of plane q (x, y neighbours from LDS slot q, z
  // neighbours from registers)
  auto form_t = [&](int l, const T* S, const float* K, T sc_, T sm, T sp, float kc, float kzm,
                    float kzp, uint32_t mask) -> T {
    T nb[6] = {S[l - 1], S[l + 1], S[l - SW], S[l + SW], sm, sp};
    T kn[6];
    if (CELL) {
      kn[0] = (T)K[l - 1]; kn[1] = (T)K[l + 1]; kn[2] = (T)K[l - SW]; kn[3] = (T)K[l + SW];
      kn[4] = (T)kzm; kn[5] = (T)kzp;
    } else {
#pragma unroll
      for (int f = 0; f < 6; ++f) kn[f] = T(1);
    }
    T dg;
    return cell_apply<T, CELL, FORM>(op, sc_, nb, (T)kc, kn, mask, dg);
  };
  // level 1 on plane q = k + 1: t, r', p' on own cells (stored with x' on
  // output planes) and on the one-cell halo of output planes; p' into LDS
  // slot q and pp1
  auto level1 = [&](int q) {
    if (q < 0 || q >= nz) {
#pragma unroll
      for (int r = 0; r < RY; ++r) pp1[r] = T(0);
      zcar = false;
      return;
    }
    const T* S = sS + (q % 3) * SP;
    const float* K = CELL ? sK + (q % 4) * SP : nullptr;
    T* P = sP + (q % 2) * SP;
    const bool outp = q >= k0 && q < k1;
    const uint32_t mz = (q > 0 ? 16u : 0u) | (q < nz - 1 ? 32u : 0u);
#pragma unroll
    for (int r = 0; r < RY; ++r) {
      T pn = T(0);
      if (own[r]) {
        T t;
        if constexpr (SHARE) {
          // this plane's coefficients, for t now and for v' a plane later
          const int l = lo[r];
          const T kn[6] = {(T)K[l - 1], (T)K[l + 1], (T)K[l - SW], (T)K[l + SW], (T)kk0[r],
                           (T)kk2[r]};
          dgn[r] = diffusion_coefs<T>(op, (T)kk1[r], kn, mo[r] | mz, Dn[r], dzc[r], zcar);
          if (first) {
            t = T(0);
          } else {
            const T nb[6] = {S[l - 1], S[l + 1], S[l - SW], S[l + SW], s0[r], s2[r]};
            t = apply_coefs<T>(Dn[r], dgn[r], s1[r], nb);
          }
        } else {
          t = first ? T(0)
                    : form_t(lo[r], S, K, s1[r], s0[r], s2[r], kk1[r], kk0[r], kk2[r],
                             mo[r] | mz);
        }
        const T rn = minus_ax(s1[r], omega, t);
        pn = next_p(rn, p1[r], v1r[r], beta, omega);
        if (outp) {
          const size_t idx = (size_t)q * plane + poff[r];
          if (!first) st_once(a.x + idx, next_x(x1[r], p1[r], s1[r], alpha, omega));
          st_once(a.r_out + idx, rn);
          st_once(a.p_out + idx, pn);
          dot_acc(acc[1], (double)rh1[r], (double)rn);
          dot_acc(acc[2], (double)rn, (double)rn);
        }
      }
      P[lo[r]] = pn;
      pp1[r] = pn;
    }
    zcar = SHARE;
    if (l1 >= 0 && outp) {
      T pn = T(0);
      if (v1) {
        const T t = first ? T(0) : form_t(l1, S, K, hs1, hs0, hs2, hk1, hk0, hk2, m1 | mz);
        const T rn = minus_ax(hs1, omega, t);
        pn = next_p(rn, hp1, hv1, beta, omega);
      }
      P[l1] = pn;
    }
  };
  // level 2 on output plane k: v' = A p' (x, y neighbours from LDS slot k,
  // z neighbours p' at k-1 and k+1 from registers)
  auto level2 = [&](int k) {
    const T* P = sP + (k % 2) * SP;
    const float* K = CELL ? sK + (k % 4) * SP : nullptr;
    const uint32_t mz = (k > 0 ? 16u : 0u) | (k < nz - 1 ? 32u : 0u);
#pragma unroll
    for (int r = 0; r < RY; ++r) {
      if (!own[r]) continue;
      const int l = lo[r];
      T nb[6] = {P[l - 1], P[l + 1], P[l - SW], P[l + SW], ppm[r], pp1[r]};
      T Av;
      if constexpr (SHARE) {
        Av = apply_coefs<T>(Do[r], dgo[r], pp0[r], nb);
      } else {
        T kn[6];
        if (CELL) {
          kn[0] = (T)K[l - 1]; kn[1] = (T)K[l + 1]; kn[2] = (T)K[l - SW]; kn[3] = (T)K[l + SW];
          kn[4] = (T)km[r]; kn[5] = (T)kk1[r];
        } else {
#pragma unroll
          for (int f = 0; f < 6; ++f) kn[f] = T(1);
        }
        T dg;
        Av = cell_apply<T, CELL, FORM>(op, pp0[r], nb, (T)kk0[r], kn, mo[r] | mz, dg);
      }
      st_once(a.v_out + (size_t)k * plane + poff[r], Av);
      dot_acc(acc[0], (double)rh0[r], (double)Av);
    }
  };

  // ---- prologue: stage k0-2 .. k0+1, level 1 on k0-1 and k0 ----
  // Two planes of loads are kept in flight (L0, L1): a step's loads are
  // issued two steps before they are staged.
  Loads L0, L1;
  load(L0, k0 - 2); load(L1, k0 - 1);
  stage(L0, k0 - 2); rotate();
  load(L0, k0);
  stage(L1, k0 - 1); rotate();
  load(L1, k0 + 1);
  stage(L0, k0);                          // registers now: k = k0-2
  load(L0, k0 + 2);
  __syncthreads();
  level1(k0 - 1);                         // own cells only (not an output plane)
  rotate();                               // k = k0-1
  stage(L1, k0 + 1);
  load(L1, k0 + 3);
  __syncthreads();
  level1(k0);
  rotate();                               // k = k0
  __syncthreads();                        // slot (k0-1) of s is free again

  // ---- march: stage k+2, level 1 on k+1, level 2 on k ----
  // plane k+2's loads are in L0 when k - k0 is even, in L1 when odd
  auto step = [&](int k, Loads& Lk) {
    stage(Lk, k + 2);
    load(Lk, k + 4);
    __syncthreads();
    level1(k + 1);
    level2(k);
    rotate();
  };
  for (int k = k0; k < k1; k += 2) {
    step(k, L0);
    if (k + 1 < k1) step(k + 1, L1);
  }
  publish_and_finalize<3>(acc, tile, g.ntiles, partials, sc, red, FinAC{sc});
}

template <typename T>
void launch_phase_act(const Launch<T>& L, const T* r, const T* v, const T* p, const T* rh, T* x,
                      T* r_out, T* p_out, T* v_out) {
  const Geo g = L.tl.geo;
  ActArgs<T> a{r, v, p, rh, x, r_out, p_out, v_out, L.shadow};
  dim3 grid(g.ntiles), block(kThreads);
#define WFA_ACT(CELLV, RYV, FV)                                                           \
  hipLaunchKernelGGL((k_phase_act<T, CELLV, RYV, FV>), grid, block, 0, L.stream, g, L.op,  \
                     L.kappa, a, L.partials, L.sc)
#define WFA_ACT_RY(CELLV, FV)                      \
  switch (L.tl.ry) {                               \
    case 1: WFA_ACT(CELLV, 1, FV); break;          \
    case 4: WFA_ACT(CELLV, 4, FV); break;          \
    default: WFA_ACT(CELLV, 2, FV); break;         \
  }
  if (L.cell && op_form(L.op) == kFormDiffusion) {
    WFA_ACT_RY(true, kFormDiffusion);
  } else if (L.cell) {
    WFA_ACT_RY(true, kFormGeneral);
  } else {
    WFA_ACT_RY(false, kFormGeneral);
  }
#undef WFA_ACT_RY
#undef WFA_ACT
}

template void launch_phase_act<double>(const Launch<double>&, const double*, const double*,
                                       const double*, const double*, double*, double*, double*,
                                       double*);
template void launch_phase_act<float>(const Launch<float>&, const float*, const float*,
                                      const float*, const float*, float*, float*, float*, float*);

}  // namespace wfa
