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

template void launch_batch_iteration2<float>(const SolveDesc<float>*, const int*, int, int, int,
                                             int, hipStream_t);
template void launch_batch_iteration2<double>(const SolveDesc<double>*, const int*, int, int,
                                              int, int, hipStream_t);

}  // namespace wfa
