// HBM bandwidth probes (wfa_bandwidth_probe): streaming kernels of known
// traffic that measure the part's achievable bandwidth -- copies, read only,
// write only, and the stream mixes of the two-reduction BiCGStab's passes --
// and calibrate the hardware byte counters.  No part of a solve runs here.
#include <hip/hip_runtime.h>

#include "device.hpp"
#include "wfa.h"
#include "internal.hpp"

namespace wfa {

// Device copy with the streaming (nontemporal) hints the stencil passes use:
// four 16-byte loads in flight per thread before their stores.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x8 __attribute__((ext_vector_type(8)));

// HBM bandwidth probes: grid-stride loops, four independent lanes' worth of
// loads in flight per thread.  k_copy (nontemporal loads and stores, 16 B per
// lane) is also the dispatch of known traffic that calibrates the hardware
// byte counters.
__global__ void __launch_bounds__(kThreads)
k_copy(size_t n16, const u32x4* __restrict__ src, u32x4* __restrict__ dst) {
  const size_t stride = (size_t)gridDim.x * kThreads;
  size_t e = (size_t)blockIdx.x * kThreads + threadIdx.x;
  for (; e + 3 * stride < n16; e += 4 * stride) {
    const u32x4 a = __builtin_nontemporal_load(src + e);
    const u32x4 b = __builtin_nontemporal_load(src + e + stride);
    const u32x4 c = __builtin_nontemporal_load(src + e + 2 * stride);
    const u32x4 d = __builtin_nontemporal_load(src + e + 3 * stride);
    __builtin_nontemporal_store(a, dst + e);
    __builtin_nontemporal_store(b, dst + e + stride);
    __builtin_nontemporal_store(c, dst + e + 2 * stride);
    __builtin_nontemporal_store(d, dst + e + 3 * stride);
  }
  for (; e < n16; e += stride) __builtin_nontemporal_store(__builtin_nontemporal_load(src + e), dst + e);
}

// The same copy with plain (cached) loads and stores.
__global__ void __launch_bounds__(kThreads)
k_copy_plain(size_t n16, const u32x4* __restrict__ src, u32x4* __restrict__ dst) {
  const size_t stride = (size_t)gridDim.x * kThreads;
  size_t e = (size_t)blockIdx.x * kThreads + threadIdx.x;
  for (; e + 3 * stride < n16; e += 4 * stride) {
    const u32x4 a = src[e], b = src[e + stride], c = src[e + 2 * stride], d = src[e + 3 * stride];
    dst[e] = a;
    dst[e + stride] = b;
    dst[e + 2 * stride] = c;
    dst[e + 3 * stride] = d;
  }
  for (; e < n16; e += stride) dst[e] = src[e];
}

// Nontemporal copy with 32 contiguous bytes per lane.
__global__ void __launch_bounds__(kThreads)
k_copy32(size_t n32, const u32x8* __restrict__ src, u32x8* __restrict__ dst) {
  const size_t stride = (size_t)gridDim.x * kThreads;
  size_t e = (size_t)blockIdx.x * kThreads + threadIdx.x;
  for (; e + stride < n32; e += 2 * stride) {
    const u32x8 a = __builtin_nontemporal_load(src + e);
    const u32x8 b = __builtin_nontemporal_load(src + e + stride);
    __builtin_nontemporal_store(a, dst + e);
    __builtin_nontemporal_store(b, dst + e + stride);
  }
  for (; e < n32; e += stride) __builtin_nontemporal_store(__builtin_nontemporal_load(src + e), dst + e);
}

// Read only: nontemporal loads folded into one value per lane, which is
// stored (into the first kThreads * 16 bytes of dst) only when it equals
// `key`, so that the loads cannot be dropped.
__global__ void __launch_bounds__(kThreads)
k_read(size_t n16, const u32x4* __restrict__ src, u32x4* __restrict__ dst, unsigned key) {
  const size_t stride = (size_t)gridDim.x * kThreads;
  size_t e = (size_t)blockIdx.x * kThreads + threadIdx.x;
  u32x4 acc = {0u, 0u, 0u, 0u};
  for (; e + 3 * stride < n16; e += 4 * stride) {
    acc ^= __builtin_nontemporal_load(src + e);
    acc ^= __builtin_nontemporal_load(src + e + stride);
    acc ^= __builtin_nontemporal_load(src + e + 2 * stride);
    acc ^= __builtin_nontemporal_load(src + e + 3 * stride);
  }
  for (; e < n16; e += stride) acc ^= __builtin_nontemporal_load(src + e);
  if ((acc.x ^ acc.y ^ acc.z ^ acc.w) == key) dst[threadIdx.x] = acc;
}

// Write only: nontemporal stores of one value.
__global__ void __launch_bounds__(kThreads)
k_write(size_t n16, u32x4* __restrict__ dst, unsigned value) {
  const size_t stride = (size_t)gridDim.x * kThreads;
  const u32x4 v = {value, value, value, value};
  for (size_t e = (size_t)blockIdx.x * kThreads + threadIdx.x; e < n16; e += stride)
    __builtin_nontemporal_store(v, dst + e);
}

// A pass's stream mix: NR streams read and NW written, all of n16 16-byte
// elements, back to back in src (NR streams) and dst (NW streams); written
// stream k is the xor of the read streams j with j % NW == k, so that no
// load can be dropped.  Nontemporal loads and stores, the NR loads of one
// element in flight together.
template <int NR, int NW>
__global__ void __launch_bounds__(kThreads)
k_mix(size_t n16, const u32x4* __restrict__ src, u32x4* __restrict__ dst) {
  static_assert(NW >= 1 && NR >= NW, "every written stream takes at least one read stream");
  const size_t stride = (size_t)gridDim.x * kThreads;
  for (size_t e = (size_t)blockIdx.x * kThreads + threadIdx.x; e < n16; e += stride) {
    u32x4 a[NR];
#pragma unroll
    for (int j = 0; j < NR; ++j) a[j] = __builtin_nontemporal_load(src + (size_t)j * n16 + e);
#pragma unroll
    for (int k = 0; k < NW; ++k) {
      u32x4 w = a[k];
#pragma unroll
      for (int j = k + NW; j < NR; j += NW) w ^= a[j];
      __builtin_nontemporal_store(w, dst + (size_t)k * n16 + e);
    }
  }
}

static void launch_probe(int kind, int blocks, const void* src, void* dst, size_t bytes,
                         hipStream_t s) {
  const size_t n16 = bytes / 16;
  switch (kind) {
    case WFA_PROBE_COPY:
      hipLaunchKernelGGL(k_copy, dim3(blocks), dim3(kThreads), 0, s, n16, (const u32x4*)src,
                         (u32x4*)dst);
      break;
    case WFA_PROBE_COPY_PLAIN:
      hipLaunchKernelGGL(k_copy_plain, dim3(blocks), dim3(kThreads), 0, s, n16,
                         (const u32x4*)src, (u32x4*)dst);
      break;
    case WFA_PROBE_COPY32:
      hipLaunchKernelGGL(k_copy32, dim3(blocks), dim3(kThreads), 0, s, bytes / 32,
                         (const u32x8*)src, (u32x8*)dst);
      break;
    case WFA_PROBE_READ:
      hipLaunchKernelGGL(k_read, dim3(blocks), dim3(kThreads), 0, s, n16, (const u32x4*)src,
                         (u32x4*)dst, 0x9e3779b9u);
      break;
    case WFA_PROBE_MIX_6R4W:
      hipLaunchKernelGGL((k_mix<6, 4>), dim3(blocks), dim3(kThreads), 0, s, n16,
                         (const u32x4*)src, (u32x4*)dst);
      break;
    case WFA_PROBE_MIX_3R1W:
      hipLaunchKernelGGL((k_mix<3, 1>), dim3(blocks), dim3(kThreads), 0, s, n16,
                         (const u32x4*)src, (u32x4*)dst);
      break;
    default:
      hipLaunchKernelGGL(k_write, dim3(blocks), dim3(kThreads), 0, s, n16, (u32x4*)dst, 0u);
      break;
  }
}

// One untimed launch, then `reps` launches between two events; GB/s of the
// bytes the kind moves (a copy reads and writes `bytes`, a stream mix moves
// `bytes` per stream).
double bandwidth_probe(int kind, int blocks, const void* src, void* dst, size_t bytes, int reps,
                       hipStream_t s, hipError_t* err) {
  hipEvent_t e0, e1;
  *err = hipEventCreate(&e0);
  if (*err != hipSuccess) return 0.0;
  *err = hipEventCreate(&e1);
  if (*err != hipSuccess) { (void)hipEventDestroy(e0); return 0.0; }
  launch_probe(kind, blocks, src, dst, bytes, s);
  *err = hipEventRecord(e0, s);
  for (int i = 0; *err == hipSuccess && i < reps; ++i) launch_probe(kind, blocks, src, dst, bytes, s);
  if (*err == hipSuccess) *err = hipGetLastError();
  if (*err == hipSuccess) *err = hipEventRecord(e1, s);
  if (*err == hipSuccess) *err = hipEventSynchronize(e1);
  float ms = 0.f;
  if (*err == hipSuccess) *err = hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (*err != hipSuccess || ms <= 0.f) return 0.0;
  const double moved = probe_streams(kind);
  return moved * (double)bytes * reps / (ms * 1e-3) / 1e9;
}

}  // namespace wfa
