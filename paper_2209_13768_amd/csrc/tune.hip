// Tile-shape autotuner and the process-wide tuning table.
//
// The z-march's two shape parameters -- rows per wave (tile height 4, 8 or
// 16 rows) and z planes per workgroup -- trade halo re-reads against
// parallelism and register pressure, and the best pair depends on the grid
// shape and precision.  wfa_autotune times a short solve for each candidate
// pair on the caller's grid and keeps the fastest.  The result is recorded
// under (nx, ny, nz, precision, coefficient mode), so every grid created
// later with the same key gets the same tiling: the tiling (and with it the
// order of every reduction) is a function of the grid's key alone.
#include <hip/hip_runtime.h>
#include <stdio.h>
#include <string.h>

#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "wfa.h"
#include "host.hpp"
#include "internal.hpp"

namespace wfa {
namespace {

struct TuneKey {
  int nx, ny, nz, prec, mode;
  bool operator<(const TuneKey& o) const {
    return std::tie(nx, ny, nz, prec, mode) < std::tie(o.nx, o.ny, o.nz, o.prec, o.mode);
  }
};
struct TuneVal {
  int ry, zc;
  double us;
};

std::mutex g_mu;
std::map<TuneKey, TuneVal>& table() {
  static std::map<TuneKey, TuneVal> t;
  return t;
}

// A fixed pattern in [0.5, 1.5) as the right-hand side of the timed solves
// (an integer hash of the index; the timing needs no particular values,
// only ones that keep BiCGStab iterating).
template <typename T>
__global__ void k_pattern(size_t n, T* b) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    uint32_t h = (uint32_t)i * 2654435761u;
    h ^= h >> 15;
    h *= 2246822519u;
    h ^= h >> 13;
    b[i] = T(0.5) + T(h >> 8) * T(1.0 / 16777216.0);
  }
}

template <typename T>
__global__ void k_zero(size_t n, T* x) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) x[i] = T(0);
}

unsigned blocks_for(size_t n) {
  size_t b = (n + kThreads - 1) / kThreads;
  return (unsigned)(b > 2048 ? 2048 : (b < 1 ? 1 : b));
}

}  // namespace

bool tuned_tiling(int nx, int ny, int nz, int precision, int mode, int* ry, int* zc) {
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = table().find(TuneKey{nx, ny, nz, precision, mode});
  if (it == table().end()) return false;
  *ry = it->second.ry;
  *zc = it->second.zc;
  return true;
}

}  // namespace wfa

using namespace wfa;

namespace {

struct OptionGuard {
  wfa_grid* g;
  int method, check_every, profile, ry, zc;
  explicit OptionGuard(wfa_grid* grid)
      : g(grid), method(grid->method), check_every(grid->check_every), profile(grid->profile),
        ry(grid->ry), zc(grid->zchunk) {}
  void restore_all() {
    g->method = method;
    g->check_every = check_every;
    g->profile = profile;
    apply_tiling(g, ry, zc);
  }
  void restore_options() {  // everything but the tiling
    g->method = method;
    g->check_every = check_every;
    g->profile = profile;
  }
};

// Milliseconds of one solve of up to `iters` iterations from x = 0, and the
// iterations it ran.  The timing needs no particular numerics: a solve that
// the numbers stop early (non-finite values, or breakdown, e.g. a diverging
// FP32 solve) is still a timing of the iterations it ran, so every solver
// outcome is accepted; only HIP and argument errors end the tuning.
int time_solve(wfa_grid* g, void* x, const void* b, int iters, hipStream_t s, hipEvent_t e0,
               hipEvent_t e1, double* ms, int* its) {
  const bool f32 = g->prec == WFA_F32;
  if (f32) hipLaunchKernelGGL(k_zero<float>, dim3(blocks_for(g->n)), dim3(kThreads), 0, s, g->n, (float*)x);
  else hipLaunchKernelGGL(k_zero<double>, dim3(blocks_for(g->n)), dim3(kThreads), 0, s, g->n, (double*)x);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_error(WFA_ERR_HIP, "autotune: %s", hipGetErrorString(e));
  if ((e = hipEventRecord(e0, s)) != hipSuccess)
    return set_error(WFA_ERR_HIP, "autotune: %s", hipGetErrorString(e));
  wfa_solve_info info{};
  const int rc = solve_any(g, b, x, false, 1e-300, iters, &info, s);
  if (rc != WFA_OK && rc != WFA_ERR_NOCONV && rc != WFA_ERR_NONFINITE && rc != WFA_ERR_BREAKDOWN)
    return rc;
  *its = info.iterations;
  if ((e = hipEventRecord(e1, s)) != hipSuccess || (e = hipEventSynchronize(e1)) != hipSuccess)
    return set_error(WFA_ERR_HIP, "autotune: %s", hipGetErrorString(e));
  float t = 0.f;
  if ((e = hipEventElapsedTime(&t, e0, e1)) != hipSuccess)
    return set_error(WFA_ERR_HIP, "autotune: %s", hipGetErrorString(e));
  *ms = t;
  return WFA_OK;
}

int autotune_impl(wfa_grid* g, int method, void* x, void* b, int iters, wfa_tune_result* out,
                  hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  const bool f32 = g->prec == WFA_F32;
  if (f32) hipLaunchKernelGGL(k_pattern<float>, dim3(blocks_for(g->n)), dim3(kThreads), 0, s, g->n, (float*)b);
  else hipLaunchKernelGGL(k_pattern<double>, dim3(blocks_for(g->n)), dim3(kThreads), 0, s, g->n, (double*)b);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_error(WFA_ERR_HIP, "autotune: %s", hipGetErrorString(e));
  g->method = method;
  g->check_every = 2 * iters;
  g->profile = 0;
  // the default rule first: a candidate must beat it to be chosen
  std::vector<std::pair<int, int>> cands = {{0, 0}};
  for (int ry : {1, 2, 4})
    for (int zc : {1, 2, 4, 8, 16, 32, 64})
      if (zc <= g->nz) cands.push_back({ry, zc});
  int best = -1;
  double best_us = 0.0, default_us = 0.0;
  std::vector<std::pair<int, int>> seen;  // resolved (rows per wave, planes) already timed
  for (size_t q = 0; q < cands.size(); ++q) {
    apply_tiling(g, cands[q].first, cands[q].second);
    const std::pair<int, int> shape{g->tl.ry, g->tl.geo.zc};
    bool dup = false;
    for (const auto& p : seen) dup = dup || p == shape;
    if (dup) continue;
    seen.push_back(shape);
    double t1 = 0.0, t2 = 0.0;
    int i1 = 0, i2 = 0;
    int rc = time_solve(g, x, b, iters, s, e0, e1, &t1, &i1);  // also warms the kernels
    if (!rc) rc = time_solve(g, x, b, iters, s, e0, e1, &t1, &i1);
    if (!rc) rc = time_solve(g, x, b, 2 * iters, s, e0, e1, &t2, &i2);
    if (rc) return rc;
    // cost per iteration without the set-up passes: the difference of the
    // two solves over the iterations they differ by; if the numbers stopped
    // both at the same iteration, the longer solve's mean instead
    double us;
    if (i2 > i1) us = (t2 - t1) * 1e3 / (i2 - i1);
    else if (i2 > 0) us = t2 * 1e3 / i2;
    else continue;                      // nothing ran (b = 0 or x already converged)
    if (q == 0) default_us = us;
    if (best < 0 || us < best_us) {
      best = (int)q;
      best_us = us;
    }
  }
  if (best < 0) return set_error(WFA_ERR_INVALID, "autotune: no candidate ran an iteration");
  // record the tile shape itself (the default rule resolved to numbers)
  apply_tiling(g, cands[best].first, cands[best].second);
  const int ry = g->tl.ry, zc = g->tl.geo.zc;
  apply_tiling(g, ry, zc);
  {
    std::lock_guard<std::mutex> lk(g_mu);
    table()[TuneKey{g->nx, g->ny, g->nz, g->prec, g->c.mode}] = TuneVal{ry, zc, best_us};
  }
  out->ry = ry;
  out->zc = zc;
  out->candidates = (int)seen.size();
  out->pad = 0;
  out->us_per_iter = best_us;
  out->us_per_iter_default = default_us;
  return WFA_OK;
}

}  // namespace

extern "C" int wfa_autotune(wfa_grid* g, int method, void* x, void* b, int iters,
                            wfa_tune_result* out, void* stream) {
  if (!g || !x || !b || !out) return set_error(WFA_ERR_INVALID, "NULL argument");
  if (iters < 1 || iters > 10000) return set_error(WFA_ERR_INVALID, "iters must be 1..10000");
  if (method != WFA_METHOD_BICGSTAB && method != WFA_METHOD_CG && method != WFA_METHOD_BICGSTAB2 &&
      method != WFA_METHOD_CG1)
    return set_error(WFA_ERR_INVALID, "bad method %d", method);
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return set_error(WFA_ERR_HIP, "autotune: event creation failed");
  }
  OptionGuard guard(g);
  const int rc = autotune_impl(g, method, x, b, iters, out, s, e0, e1);
  if (rc) guard.restore_all();
  else guard.restore_options();
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return rc;
}

extern "C" int wfa_tune_save(const char* path) {
  if (!path) return set_error(WFA_ERR_INVALID, "path is NULL");
  FILE* f = fopen(path, "w");
  if (!f) return set_error(WFA_ERR_INVALID, "cannot write %s", path);
  std::lock_guard<std::mutex> lk(g_mu);
  fprintf(f, "# wfa tuning table: nx ny nz precision mode rows_per_wave z_planes us_per_iter\n");
  for (const auto& kv : table())
    fprintf(f, "%d %d %d %d %d %d %d %.3f\n", kv.first.nx, kv.first.ny, kv.first.nz,
            kv.first.prec, kv.first.mode, kv.second.ry, kv.second.zc, kv.second.us);
  const bool ok = fclose(f) == 0;
  return ok ? WFA_OK : set_error(WFA_ERR_INVALID, "error writing %s", path);
}

extern "C" int wfa_tune_load(const char* path) {
  if (!path) return set_error(WFA_ERR_INVALID, "path is NULL");
  FILE* f = fopen(path, "r");
  if (!f) return set_error(WFA_ERR_INVALID, "cannot read %s", path);
  std::map<TuneKey, TuneVal> add;
  char line[512];
  int lineno = 0, bad = 0;
  while (fgets(line, sizeof line, f)) {
    ++lineno;
    if (line[0] == '#' || line[0] == '\n') continue;
    TuneKey k{};
    TuneVal v{};
    if (sscanf(line, "%d %d %d %d %d %d %d %lf", &k.nx, &k.ny, &k.nz, &k.prec, &k.mode, &v.ry,
               &v.zc, &v.us) != 8 ||
        k.nx < 1 || k.ny < 1 || k.nz < 1 || k.prec < WFA_F64 || k.prec > WFA_F32_IR64 ||
        (k.mode != WFA_COEF_CONST && k.mode != WFA_COEF_CELL) ||
        (v.ry != 1 && v.ry != 2 && v.ry != 4) || v.zc < 1 || v.zc > k.nz) {
      bad = lineno;
      break;
    }
    add[k] = v;
  }
  fclose(f);
  if (bad) return set_error(WFA_ERR_INVALID, "%s: malformed entry on line %d", path, bad);
  std::lock_guard<std::mutex> lk(g_mu);
  for (const auto& kv : add) table()[kv.first] = kv.second;
  return WFA_OK;
}

extern "C" int wfa_tune_clear(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  table().clear();
  return WFA_OK;
}
