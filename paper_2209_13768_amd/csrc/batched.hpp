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
  double* partials;
  Scalars* sc;
  size_t n;
  int cell;
  int pw_blocks;
};

// One BiCGStab iteration (phases A, B, C) of every solve in descs[0..nsolves).
// tile_bases / pw_bases: prefix sums of the solves' tile and pointwise-block
// counts (nsolves + 1 entries each, device memory).  Every solve's tiling
// must use `ry` rows per wave.
template <typename T>
void launch_batch_iteration(const SolveDesc<T>* descs, const int* tile_bases, int tiles_total,
                            const int* pw_bases, int pw_total, int nsolves, int parity, int ry,
                            hipStream_t s);

}  // namespace wfa
