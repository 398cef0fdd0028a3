// Persistent BiCGStab: one cooperative launch runs up to `iters` full
// iterations of one solve, with a grid barrier in place of each of the three
// kernel boundaries per iteration.  For small grids, where an iteration is a
// few microseconds of memory traffic, launch and dependency latency would
// otherwise dominate (the paper makes the same observation for its
// reduction-bound CG on the wafer, section 3.2.2).
//
// Every workgroup runs the tiles blockIdx.x, blockIdx.x + gridDim.x, ... of
// each phase, stores one partial sum per tile (the same partials a
// single-phase launch produces), meets the others at a grid barrier, then
// reduces all partials in the same fixed order and applies the same
// finalizer to a private copy of the scalars.  The iterates are therefore
// bitwise those of the one-launch-per-phase path.
#include "device.hpp"
#include "internal.hpp"
#include "phases.hpp"

namespace wfa {

template <typename T>
struct PersistArgs {
  Geo geo;
  Op<T> op;
  const float* kappa;
  T *x, *r, *rh, *t, *p0, *p1, *v0, *v1;
  double* partials;  // regions: A [ntiles], B [2 ntiles], C [2 pw_blocks]
  Scalars* sc;
  GridBarrier* bar;
  size_t n;
  int pw_blocks;
  int iters;
  int parity;
  int spin_limit;
};

template <typename T, bool CELL, int RY>
__global__ void __launch_bounds__(kThreads) k_persistent_bicgstab(PersistArgs<T> a) {
  using TS = TileShape<RY>;
  __shared__ T su[2 * TS::LH * TS::LW];
  __shared__ float sk[CELL ? 2 * TS::LH * TS::LW : 1];
  __shared__ double red[kWaves * 2];
  __shared__ Scalars ls;
  if (threadIdx.x == 0) ls = *a.sc;
  __syncthreads();
  const Geo g = a.geo;
  const int nt = g.ntiles, pw = a.pw_blocks;
  double* partA = a.partials;
  double* partB = a.partials + nt;
  double* partC = a.partials + 3 * (size_t)nt;
  const uint32_t nb = gridDim.x;
  bool alive = true;
  for (int it = 0; it < a.iters && alive; ++it) {
    if (ls.status != ST_RUN || ls.restart) break;
    const int par = (a.parity + it) & 1;
    T* p_in = par ? a.p1 : a.p0;
    T* p_out = par ? a.p0 : a.p1;
    T* v_in = par ? a.v1 : a.v0;
    T* v_out = par ? a.v0 : a.v1;
    // ---- phase A: p' = r + beta (p - omega v), v' = A p', sigma
    {
      PhA<T> ph{};
      ph.r = a.r; ph.p = p_in; ph.v = v_in; ph.p_out = p_out; ph.v_out = v_out; ph.rh = a.rh;
      ph.bind(&ls);
      for (int tile = blockIdx.x; tile < nt; tile += nb) {
        double acc[1] = {0.0};
        march_tile<T, CELL, RY>(g, a.op, a.kappa, tile, ph, acc, su, sk);
        block_sum<1>(acc, red);
        store_partial<1>(partA, nt, tile, acc);
      }
      if (!(alive = grid_sync(a.bar, nb, a.spin_limit))) break;
      double s[1];
      reduce_partials<1>(partA, nt, s, red);
      if (threadIdx.x == 0) FinA{&ls}(s);
      __syncthreads();
      if (ls.status != ST_RUN || ls.restart) break;
    }
    // ---- phase B: s = r - alpha v', t = A s, (t,s), (t,t)
    {
      PhB<T> ph{};
      ph.r = a.r; ph.v = v_out; ph.t = a.t;
      ph.bind(&ls);
      for (int tile = blockIdx.x; tile < nt; tile += nb) {
        double acc[2] = {0.0, 0.0};
        march_tile<T, CELL, RY>(g, a.op, a.kappa, tile, ph, acc, su, sk);
        block_sum<2>(acc, red);
        store_partial<2>(partB, nt, tile, acc);
      }
      if (!(alive = grid_sync(a.bar, nb, a.spin_limit))) break;
      double s[2];
      reduce_partials<2>(partB, nt, s, red);
      if (threadIdx.x == 0) FinB{&ls}(s);
      __syncthreads();
      if (ls.status != ST_RUN) break;
    }
    // ---- phase C: x += alpha p' + omega s, r = s - omega t, rho', ||r||^2
    {
      for (int blk = blockIdx.x; blk < pw; blk += nb) {
        double acc[2] = {0.0, 0.0};
        phase_c_range<T>(a.n, blk, pw, a.x, p_out, a.r, v_out, a.t, a.rh, &ls, acc);
        block_sum<2>(acc, red);
        store_partial<2>(partC, pw, blk, acc);
      }
      if (!(alive = grid_sync(a.bar, nb, a.spin_limit))) break;
      double s[2];
      reduce_partials<2>(partC, pw, s, red);
      if (threadIdx.x == 0) FinC{&ls}(s);
      __syncthreads();
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ls.counter = 0;
    *a.sc = ls;
  }
}

template <typename T, bool CELL, int RY>
static hipError_t launch_one(const Launch<T>& L, const PersistArgs<T>& a, int blocks) {
  void* args[] = {(void*)&a};
  return hipLaunchCooperativeKernel((const void*)k_persistent_bicgstab<T, CELL, RY>, dim3(blocks),
                                    dim3(kThreads), args, 0, L.stream);
}

template <typename T, bool CELL, int RY>
static int max_coresident() {
  static int cached = -1;
  if (cached < 0) {
    int per_cu = 0, dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu, (const void*)k_persistent_bicgstab<T, CELL, RY>, kThreads, 0) != hipSuccess)
      return 0;
    cached = per_cu * cus;
  }
  return cached;
}

template <typename T>
hipError_t launch_persistent_bicgstab(const Launch<T>& L, T* x, T* r, const T* rh, T* p0, T* p1,
                                      T* v0, T* v1, T* t, int iters, int parity,
                                      GridBarrier* bar) {
  PersistArgs<T> a{};
  a.geo = L.tl.geo;
  a.op = L.op;
  a.kappa = L.kappa;
  a.x = x; a.r = r; a.rh = (T*)rh; a.t = t; a.p0 = p0; a.p1 = p1; a.v0 = v0; a.v1 = v1;
  a.partials = L.partials;
  a.sc = L.sc;
  a.bar = bar;
  a.n = (size_t)L.tl.geo.plane * L.tl.geo.nz;
  a.pw_blocks = L.tl.pw_blocks;
  a.iters = iters;
  a.parity = parity;
  a.spin_limit = 1 << 22;
  const int want = a.geo.ntiles > a.pw_blocks ? a.geo.ntiles : a.pw_blocks;
#define WFA_PERSIST(CELLV, RYV)                                            \
  {                                                                         \
    const int cap = max_coresident<T, CELLV, RYV>();                        \
    if (cap <= 0) return hipErrorInvalidConfiguration;                      \
    return launch_one<T, CELLV, RYV>(L, a, want < cap ? want : cap);        \
  }
  if (L.cell) {
    switch (L.tl.ry) {
      case 1: WFA_PERSIST(true, 1);
      case 4: WFA_PERSIST(true, 4);
      default: WFA_PERSIST(true, 2);
    }
  } else {
    switch (L.tl.ry) {
      case 1: WFA_PERSIST(false, 1);
      case 4: WFA_PERSIST(false, 4);
      default: WFA_PERSIST(false, 2);
    }
  }
#undef WFA_PERSIST
}

template hipError_t launch_persistent_bicgstab<double>(const Launch<double>&, double*, double*,
                                                       const double*, double*, double*, double*,
                                                       double*, double*, int, int, GridBarrier*);
template hipError_t launch_persistent_bicgstab<float>(const Launch<float>&, float*, float*,
                                                      const float*, float*, float*, float*,
                                                      float*, float*, int, int, GridBarrier*);

}  // namespace wfa
