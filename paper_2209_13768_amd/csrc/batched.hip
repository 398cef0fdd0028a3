// Batched two-reduction BiCGStab passes for serving: one launch advances
// every resident solve by one pass.  Work item i of a launch belongs to the
// solve s with bases[s] <= i < bases[s+1]; within its solve it is the tile of
// the same index a single-solve launch would give it.  Per-tile partial
// sums, their fixed-order reduction and the finalizers are the single-solve
// ones, so a solve's iterates are bitwise the same alone and batched with
// any other solves.
#include "batched.hpp"
#include "phases.hpp"

namespace wfa {

__device__ __forceinline__ int find_solve(const int* __restrict__ bases, int nsolves, int item) {
  int lo = 0, hi = nsolves - 1;  // largest s with bases[s] <= item
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (bases[mid] <= item) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// PASS 0: AC (update, p' and v' = A p'); PASS 1: B2 (t = A s).  r, p and v
// are double-buffered; `parity` selects the buffers of this iteration.
template <typename T, int RY, int PASS>
__global__ void __launch_bounds__(kThreads)
k_batch_march(const SolveDesc<T>* __restrict__ descs, const int* __restrict__ bases,
              int nsolves, int parity) {
  using TS = TileShape<RY>;
  __shared__ T su[2 * TS::LH * TS::LW];
  __shared__ float sk[2 * TS::LH * TS::LW];
  __shared__ double red[kWaves * kMaxReduce];
  const int s = find_solve(bases, nsolves, blockIdx.x);
  const SolveDesc<T> d = descs[s];
  Scalars* sc = d.sc;
  if (sc->status != ST_RUN || sc->restart) return;
  const int tile = blockIdx.x - bases[s];
  if (d.cg1) {
    // two CG iterations per launch pair: the pair returns the buffers to
    // where they started, whatever the launch's place in a round
    const int pp = PASS ^ d.par;
    PhCg1<T> ph{};
    ph.r = pp ? d.r1 : d.r; ph.w = pp ? d.v1 : d.v0; ph.s = pp ? d.p1 : d.p0;
    ph.p = d.t; ph.x = d.x;
    ph.r_out = pp ? d.r : d.r1; ph.w_out = pp ? d.v0 : d.v1; ph.s_out = pp ? d.p0 : d.p1;
    ph.bind(sc);
    double acc[2] = {0.0, 0.0};
    if (d.cell) march_tile<T, true, RY>(d.geo, d.op, d.kappa, tile, ph, acc, su, sk);
    else march_tile<T, false, RY>(d.geo, d.op, d.kappa, tile, ph, acc, su, sk);
    publish_and_finalize<2>(acc, tile, d.geo.ntiles, d.partials, sc, red, FinCg1{sc});
    return;
  }
  parity ^= d.par;
  T* r_in = parity ? d.r1 : d.r;
  T* r_out = parity ? d.r : d.r1;
  T* p_in = parity ? d.p1 : d.p0;
  T* p_out = parity ? d.p0 : d.p1;
  T* v_in = parity ? d.v1 : d.v0;
  T* v_out = parity ? d.v0 : d.v1;
  if (PASS == 0) {
    PhAC<T> ph{};
    ph.r = r_in; ph.v = v_in; ph.t = d.t; ph.p = p_in; ph.rh = d.rh; ph.x = d.x;
    ph.r_out = r_out; ph.p_out = p_out; ph.v_out = v_out;
    ph.hashed = d.hashed;
    ph.bind(sc);
    double acc[3] = {0.0, 0.0, 0.0};
    if (d.cell) march_tile<T, true, RY>(d.geo, d.op, d.kappa, tile, ph, acc, su, sk);
    else march_tile<T, false, RY>(d.geo, d.op, d.kappa, tile, ph, acc, su, sk);
    publish_and_finalize<3>(acc, tile, d.geo.ntiles, d.partials, sc, red, FinAC{sc});
  } else {
    PhB2<T> ph{};
    ph.r = r_out; ph.v = v_out; ph.rh = d.rh; ph.t = d.t;
    ph.hashed = d.hashed;
    ph.bind(sc);
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    if (d.cell) march_tile<T, true, RY>(d.geo, d.op, d.kappa, tile, ph, acc, su, sk);
    else march_tile<T, false, RY>(d.geo, d.op, d.kappa, tile, ph, acc, su, sk);
    publish_and_finalize<4>(acc, tile, d.geo.ntiles, d.partials, sc, red, FinB2{sc});
  }
}

template <typename T, int RY>
static void batch_iteration2(const SolveDesc<T>* descs, const int* tile_bases, int tiles_total,
                             int nsolves, int q, hipStream_t s) {
  hipLaunchKernelGGL((k_batch_march<T, RY, 0>), dim3(tiles_total), dim3(kThreads), 0, s, descs,
                     tile_bases, nsolves, q & 1);
  hipLaunchKernelGGL((k_batch_march<T, RY, 1>), dim3(tiles_total), dim3(kThreads), 0, s, descs,
                     tile_bases, nsolves, q & 1);
}

template <typename T>
void launch_batch_iteration2(const SolveDesc<T>* descs, const int* tile_bases, int tiles_total,
                             int nsolves, int q, int ry, hipStream_t s) {
  switch (ry) {
    case 1: batch_iteration2<T, 1>(descs, tile_bases, tiles_total, nsolves, q, s); break;
    case 4: batch_iteration2<T, 4>(descs, tile_bases, tiles_total, nsolves, q, s); break;
    default: batch_iteration2<T, 2>(descs, tile_bases, tiles_total, nsolves, q, s); break;
  }
}

// Persistent form of a serving round: one cooperative launch runs `iters`
// two-reduction iterations of every resident solve, with grid barriers in
// place of the kernel boundaries.  Each pass stores the per-tile partial
// sums of the one-launch-per-pass form; after a barrier, every running
// solve's finalizer runs once (solve s on workgroup s mod gridDim) over
// those partials in the same fixed order.  The iterates are therefore
// bitwise those of the per-pass launches.  A solve that has stopped, or
// awaits a restart, is skipped as the per-pass kernels skip it.
template <typename T, int RY>
__global__ void __launch_bounds__(kThreads)
k_batch_persistent(const SolveDesc<T>* __restrict__ descs, const int* __restrict__ bases,
                   int nsolves, int tiles_total, int iters, GridBarrier* bar, int spin_limit) {
  using TS = TileShape<RY>;
  __shared__ T su[2 * TS::LH * TS::LW];
  __shared__ float sk[2 * TS::LH * TS::LW];
  __shared__ double red[kWaves * kMaxReduce];
  const uint32_t nb = gridDim.x;
  for (int q = 0; q < iters; ++q) {
    // ---- pass AC of every solve
    for (int item = blockIdx.x; item < tiles_total; item += (int)nb) {
      const int s = find_solve(bases, nsolves, item);
      const SolveDesc<T> d = descs[s];
      Scalars* sc = d.sc;
      if (sc->status != ST_RUN || sc->restart) continue;
      const int tile = item - bases[s];
      const int parity = (q & 1) ^ d.par;
      PhAC<T> ph{};
      ph.r = parity ? d.r1 : d.r; ph.v = parity ? d.v1 : d.v0; ph.t = d.t;
      ph.p = parity ? d.p1 : d.p0; ph.rh = d.rh; ph.x = d.x;
      ph.r_out = parity ? d.r : d.r1; ph.p_out = parity ? d.p0 : d.p1;
      ph.v_out = parity ? d.v0 : d.v1;
      ph.hashed = d.hashed;
      ph.bind(sc);
      double acc[3] = {0.0, 0.0, 0.0};
      if (d.cell) march_tile<T, true, RY>(d.geo, d.op, d.kappa, tile, ph, acc, su, sk);
      else march_tile<T, false, RY>(d.geo, d.op, d.kappa, tile, ph, acc, su, sk);
      block_sum<3>(acc, red);
      store_partial<3>(d.partials, d.geo.ntiles, tile, acc);
    }
    if (!grid_sync(bar, nb, spin_limit)) return;
    for (int s = blockIdx.x; s < nsolves; s += (int)nb) {
      const SolveDesc<T> d = descs[s];
      Scalars* sc = d.sc;
      if (sc->status != ST_RUN || sc->restart) continue;
      double sums[3];
      reduce_partials<3>(d.partials, d.geo.ntiles, sums, red);
      if (threadIdx.x == 0) FinAC{sc}(sums);
      __syncthreads();
    }
    if (!grid_sync(bar, nb, spin_limit)) return;
    // ---- pass B2 of every solve
    for (int item = blockIdx.x; item < tiles_total; item += (int)nb) {
      const int s = find_solve(bases, nsolves, item);
      const SolveDesc<T> d = descs[s];
      Scalars* sc = d.sc;
      if (sc->status != ST_RUN || sc->restart) continue;
      const int tile = item - bases[s];
      const int parity = (q & 1) ^ d.par;
      PhB2<T> ph{};
      ph.r = parity ? d.r : d.r1; ph.v = parity ? d.v0 : d.v1; ph.rh = d.rh; ph.t = d.t;
      ph.hashed = d.hashed;
      ph.bind(sc);
      double acc[4] = {0.0, 0.0, 0.0, 0.0};
      if (d.cell) march_tile<T, true, RY>(d.geo, d.op, d.kappa, tile, ph, acc, su, sk);
      else march_tile<T, false, RY>(d.geo, d.op, d.kappa, tile, ph, acc, su, sk);
      block_sum<4>(acc, red);
      store_partial<4>(d.partials, d.geo.ntiles, tile, acc);
    }
    if (!grid_sync(bar, nb, spin_limit)) return;
    for (int s = blockIdx.x; s < nsolves; s += (int)nb) {
      const SolveDesc<T> d = descs[s];
      Scalars* sc = d.sc;
      if (sc->status != ST_RUN || sc->restart) continue;
      double sums[4];
      reduce_partials<4>(d.partials, d.geo.ntiles, sums, red);
      if (threadIdx.x == 0) FinB2{sc}(sums);
      __syncthreads();
    }
    if (!grid_sync(bar, nb, spin_limit)) return;
  }
}

template <typename T, int RY>
static hipError_t batch_persistent(const SolveDesc<T>* descs, const int* tile_bases,
                                   int tiles_total, int nsolves, int iters, GridBarrier* bar,
                                   int spin_limit, hipStream_t s) {
  static int cap = -1;  // workgroups that fit on the device at once
  if (cap < 0) {
    int per_cu = 0, dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess)
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &per_cu, (const void*)k_batch_persistent<T, RY>, kThreads, 0);
    if (e != hipSuccess) return e;
    cap = per_cu * cus;
  }
  if (cap <= 0) return hipErrorInvalidConfiguration;
  const int blocks = tiles_total < cap ? tiles_total : cap;
  void* args[] = {(void*)&descs, (void*)&tile_bases, (void*)&nsolves, (void*)&tiles_total,
                  (void*)&iters, (void*)&bar, (void*)&spin_limit};
  return hipLaunchCooperativeKernel((const void*)k_batch_persistent<T, RY>, dim3(blocks),
                                    dim3(kThreads), args, 0, s);
}

template <typename T>
hipError_t launch_batch_persistent(const SolveDesc<T>* descs, const int* tile_bases,
                                   int tiles_total, int nsolves, int iters, int ry,
                                   GridBarrier* bar, int spin_limit, hipStream_t s) {
  switch (ry) {
    case 1: return batch_persistent<T, 1>(descs, tile_bases, tiles_total, nsolves, iters, bar, spin_limit, s);
    case 4: return batch_persistent<T, 4>(descs, tile_bases, tiles_total, nsolves, iters, bar, spin_limit, s);
    default: return batch_persistent<T, 2>(descs, tile_bases, tiles_total, nsolves, iters, bar, spin_limit, s);
  }
}

template void launch_batch_iteration2<float>(const SolveDesc<float>*, const int*, int, int, int,
                                             int, hipStream_t);
template void launch_batch_iteration2<double>(const SolveDesc<double>*, const int*, int, int,
                                              int, int, hipStream_t);

template hipError_t launch_batch_persistent<float>(const SolveDesc<float>*, const int*, int, int,
                                                   int, int, GridBarrier*, int, hipStream_t);
template hipError_t launch_batch_persistent<double>(const SolveDesc<double>*, const int*, int, int,
                                                    int, int, GridBarrier*, int, hipStream_t);

}  // namespace wfa
