// Batched BiCGStab passes for serving: one launch advances every resident
// solve by one phase.  Work item i of a launch belongs to the solve s with
// bases[s] <= i < bases[s+1]; within its solve it is the tile (stencil
// passes) or the pointwise block (phase C) of the same index a single-solve
// launch would give it.  Per-tile partial sums, their fixed-order reduction
// and the finalizers are the single-solve ones, so a solve's iterates are
// bitwise the same alone and batched with any other solves.
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

template <typename T, int RY, int KIND>
__global__ void __launch_bounds__(kThreads)
k_batch_march(const SolveDesc<T>* __restrict__ descs, const int* __restrict__ bases,
              int nsolves, int parity) {
  using TS = TileShape<RY>;
  __shared__ T su[2 * TS::LH * TS::LW];
  __shared__ float sk[2 * TS::LH * TS::LW];
  __shared__ double red[kWaves * 2];
  const int s = find_solve(bases, nsolves, blockIdx.x);
  const SolveDesc<T> d = descs[s];
  Scalars* sc = d.sc;
  if (sc->status != ST_RUN || sc->restart) return;
  const int tile = blockIdx.x - bases[s];
  T* p_in = parity ? d.p1 : d.p0;
  T* p_out = parity ? d.p0 : d.p1;
  T* v_in = parity ? d.v1 : d.v0;
  T* v_out = parity ? d.v0 : d.v1;
  if (KIND == 0) {
    PhA<T> ph{};
    ph.r = d.r; ph.p = p_in; ph.v = v_in; ph.p_out = p_out; ph.v_out = v_out; ph.rh = d.rh;
    ph.bind(sc);
    double acc[1] = {0.0};
    if (d.cell) march_tile<T, true, RY>(d.geo, d.op, d.kappa, tile, ph, acc, su, sk);
    else march_tile<T, false, RY>(d.geo, d.op, d.kappa, tile, ph, acc, su, sk);
    publish_and_finalize<1>(acc, tile, d.geo.ntiles, d.partials, sc, red, FinA{sc});
  } else {
    PhB<T> ph{};
    ph.r = d.r; ph.v = v_out; ph.t = d.t;
    ph.bind(sc);
    double acc[2] = {0.0, 0.0};
    if (d.cell) march_tile<T, true, RY>(d.geo, d.op, d.kappa, tile, ph, acc, su, sk);
    else march_tile<T, false, RY>(d.geo, d.op, d.kappa, tile, ph, acc, su, sk);
    publish_and_finalize<2>(acc, tile, d.geo.ntiles, d.partials, sc, red, FinB{sc});
  }
}

template <typename T>
__global__ void __launch_bounds__(kThreads)
k_batch_phase_c(const SolveDesc<T>* __restrict__ descs, const int* __restrict__ bases,
                int nsolves, int parity) {
  __shared__ double red[kWaves * 2];
  const int s = find_solve(bases, nsolves, blockIdx.x);
  const SolveDesc<T> d = descs[s];
  Scalars* sc = d.sc;
  if (sc->status != ST_RUN || sc->restart) return;
  const int blk = blockIdx.x - bases[s];
  const T* p_new = parity ? d.p0 : d.p1;
  const T* v_new = parity ? d.v0 : d.v1;
  double acc[2] = {0.0, 0.0};
  phase_c_range<T>(d.n, blk, d.pw_blocks, d.x, p_new, d.r, v_new, d.t, d.rh, sc, acc);
  publish_and_finalize<2>(acc, blk, d.pw_blocks, d.partials, sc, red, FinC{sc});
}

template <typename T, int RY>
static void batch_iteration(const SolveDesc<T>* descs, const int* tile_bases, int tiles_total,
                            const int* pw_bases, int pw_total, int nsolves, int parity,
                            hipStream_t s) {
  hipLaunchKernelGGL((k_batch_march<T, RY, 0>), dim3(tiles_total), dim3(kThreads), 0, s, descs,
                     tile_bases, nsolves, parity);
  hipLaunchKernelGGL((k_batch_march<T, RY, 1>), dim3(tiles_total), dim3(kThreads), 0, s, descs,
                     tile_bases, nsolves, parity);
  hipLaunchKernelGGL((k_batch_phase_c<T>), dim3(pw_total), dim3(kThreads), 0, s, descs, pw_bases,
                     nsolves, parity);
}

template <typename T>
void launch_batch_iteration(const SolveDesc<T>* descs, const int* tile_bases, int tiles_total,
                            const int* pw_bases, int pw_total, int nsolves, int parity, int ry,
                            hipStream_t s) {
  switch (ry) {
    case 1: batch_iteration<T, 1>(descs, tile_bases, tiles_total, pw_bases, pw_total, nsolves, parity, s); break;
    case 4: batch_iteration<T, 4>(descs, tile_bases, tiles_total, pw_bases, pw_total, nsolves, parity, s); break;
    default: batch_iteration<T, 2>(descs, tile_bases, tiles_total, pw_bases, pw_total, nsolves, parity, s); break;
  }
}

template void launch_batch_iteration<float>(const SolveDesc<float>*, const int*, int, const int*,
                                            int, int, int, int, hipStream_t);
template void launch_batch_iteration<double>(const SolveDesc<double>*, const int*, int,
                                             const int*, int, int, int, int, hipStream_t);

}  // namespace wfa
