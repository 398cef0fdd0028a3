// Descriptor of one resident solve in a batched launch (device memory).
#pragma once
#include <hip/hip_runtime.h>

#include "device.hpp"

namespace wfa {

template <typename T>
struct SolveDesc {
  Geo geo;
  Op<T> op;
  const float* kappa;
  T* x;                 // iterate of the Krylov solve (IR: the FP32 correction)
  T *r, *rh, *t, *p0, *p1, *v0, *v1;
  T* r1;                // second residual buffer of the two-reduction BiCGStab
  int par;              // buffer parity of the solve at the first iteration of the launch
  int hashed;           // shadow residual hashed from the cell index (not stored)
  int cg1;              // 1: CG with one reduction (symmetric A): each of the two passes
                        // is one CG iteration; r (r, r1), w (v0, v1) and s (p0, p1)
                        // alternate per pass, p in t; parity 0 at the first pass
  double* partials;
  Scalars* sc;
  size_t n;
  int cell;
  int pw_blocks;
};

// One two-reduction BiCGStab iteration (passes AC and B2) of every solve in
// descs[0..nsolves), or two iterations of a solve marked cg1.  tile_bases: prefix sums of the solves' tile counts
// (nsolves + 1 entries, device memory); every solve's tiling must use `ry`
// rows per wave.  Solve s uses the buffers of parity descs[s].par ^ (q & 1),
// q = the index of this iteration among the launches made since the
// descriptors were written.
template <typename T>
void launch_batch_iteration2(const SolveDesc<T>* descs, const int* tile_bases, int tiles_total,
                             int nsolves, int q, int ry, hipStream_t s);

// `iters` such iterations in one cooperative launch, with grid barriers in
// place of the kernel boundaries (bitwise the same iterates).  `bar` is a
// barrier in device memory whose count and timeout start at zero; the
// launch leaves them so unless a wait timed out: then bar->timeout is set,
// the waves have left early and the solves' state is undefined.  Returns
// the launch's error code.
template <typename T>
hipError_t launch_batch_persistent(const SolveDesc<T>* descs, const int* tile_bases,
                                   int tiles_total, int nsolves, int iters, int ry,
                                   GridBarrier* bar, int spin_limit, hipStream_t s);

}  // namespace wfa
