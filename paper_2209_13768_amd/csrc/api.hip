// Host side of libwfa: grid descriptors, the Krylov drivers (BiCGStab, CG,
// FP32-in-FP64 iterative refinement), backward-Euler time stepping, launch
// profiling, and the C-ABI declared in include/wfa.h.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdlib.h>
#include <stdio.h>
#include <string.h>

#include <chrono>
#include <functional>
#include <initializer_list>
#include <new>
#include <vector>

#include "wfa.h"
#include "internal.hpp"
#include "host.hpp"

using namespace wfa;

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local char g_err[512] = "";

namespace wfa {
int set_error(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
  return code;
}
}  // namespace wfa

#define HIP_TRY(expr)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      return set_error(WFA_ERR_HIP, "%s: %s (%s:%d)", #expr, hipGetErrorString(e_),     \
                       __FILE__, __LINE__);                                            \
  } while (0)

extern "C" const char* wfa_last_error(void) { return g_err; }
extern "C" const char* wfa_version(void) { return "wfa 0.1 (gfx950)"; }

// ---------------------------------------------------------------------------
// workspace layout
// ---------------------------------------------------------------------------
static size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

namespace wfa {

size_t partial_slots(int nx, int ny, int nz) {
  // worst case over the tile shapes the library may choose (ry >= 1, zc >= 1)
  const size_t tx = (size_t)(nx + kTX - 1) / kTX;
  const size_t ty = (size_t)(ny + kWaves - 1) / kWaves;
  size_t s = tx * ty * (size_t)nz;
  if (s < 2048) s = 2048;
  return s;
}

Layout layout_for(int nx, int ny, int nz, int precision) {
  Layout L{};
  const size_t n = (size_t)nx * ny * nz;
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off += align256(bytes); return o; };
  L.scalars = take(sizeof(Scalars) * 4);
  // one launch per pass: up to kMaxReduce values per tile slot (the
  // two-reduction BiCGStab's second pass reduces four); persistent launches
  // keep the three phases' partials apart (3 x tiles + 2 x pointwise blocks)
  L.partials = take(sizeof(double) * (kMaxReduce * partial_slots(nx, ny, nz) + 2 * 2048));
  if (precision == WFA_F32_IR64) {
    L.b64 = take(8 * n);
    for (int q = 0; q < kVecs; ++q) L.vec[q] = take(4 * n);
    L.d32 = take(4 * n);
  } else {
    const size_t w = precision == WFA_F32 ? 4 : 8;
    for (int q = 0; q < kVecs; ++q) L.vec[q] = take(w * n);
  }
  L.total = off;
  return L;
}

}  // namespace wfa

extern "C" size_t wfa_workspace_bytes(int nx, int ny, int nz, int precision) {
  if (nx < 1 || ny < 1 || nz < 1) return 0;
  if (precision < WFA_F64 || precision > WFA_F32_IR64) return 0;
  return layout_for(nx, ny, nz, precision).total;
}

// ---------------------------------------------------------------------------
// grid
// ---------------------------------------------------------------------------
namespace wfa {

template <typename T>
static Op<T> make_op(const wfa_coeffs& c) {
  Op<T> op{};
  const double cD = c.mode == WFA_COEF_CELL ? c.dt / (c.h * c.h) : c.dt * c.alpha / (c.h * c.h);
  op.cD = (T)cD;
  for (int f = 0; f < 6; ++f) {
    const int axis = f / 2;
    const double normal = (f % 2 == 0) ? -1.0 : 1.0;
    const double F = c.dt * (c.u[axis] * normal) / c.h;
    op.in[f] = (T)fmax(-F, 0.0);
    op.out[f] = (T)fmax(F, 0.0);
    op.bval[f] = (T)c.bc_value[f];
    if (c.bc[f] == WFA_BC_DIRICHLET) op.dir |= 1u << f;
    if (op.in[f] != T(0) || op.out[f] != T(0)) op.conv = 1;
  }
  return op;
}

int validate_coeffs(int nx, int ny, int nz, const wfa_coeffs* c) {
  if (!c) return set_error(WFA_ERR_INVALID, "coeffs is NULL");
  if (nx < 1 || ny < 1 || nz < 1)
    return set_error(WFA_ERR_INVALID, "grid dimensions must be >= 1 (got %d x %d x %d)", nx, ny, nz);
  if ((long long)nx * ny > 0x7fffffffLL)
    return set_error(WFA_ERR_INVALID, "nx*ny must fit in 31 bits");
  if (c->mode != WFA_COEF_CONST && c->mode != WFA_COEF_CELL)
    return set_error(WFA_ERR_INVALID, "bad coefficient mode %d", c->mode);
  if (c->precision < WFA_F64 || c->precision > WFA_F32_IR64)
    return set_error(WFA_ERR_INVALID, "bad precision %d", c->precision);
  if (!(c->h > 0.0) || !(c->dt > 0.0) || !isfinite(c->h) || !isfinite(c->dt))
    return set_error(WFA_ERR_INVALID, "h and dt must be finite and > 0");
  if (c->mode == WFA_COEF_CONST && !(c->alpha >= 0.0 && isfinite(c->alpha)))
    return set_error(WFA_ERR_INVALID, "alpha must be finite and >= 0");
  if (c->mode == WFA_COEF_CELL && !c->kappa)
    return set_error(WFA_ERR_INVALID, "CELL mode needs a kappa pointer");
  for (int a = 0; a < 3; ++a)
    if (!isfinite(c->u[a])) return set_error(WFA_ERR_INVALID, "velocity must be finite");
  for (int f = 0; f < 6; ++f) {
    if (c->bc[f] != WFA_BC_DIRICHLET && c->bc[f] != WFA_BC_ZEROFLUX)
      return set_error(WFA_ERR_INVALID, "bad boundary kind %d on face %d", c->bc[f], f);
    if (!isfinite(c->bc_value[f])) return set_error(WFA_ERR_INVALID, "boundary value not finite");
  }
  return WFA_OK;
}

void grid_setup(wfa_grid* g, int nx, int ny, int nz, const wfa_coeffs* c, char* ws) {
  g->nx = nx; g->ny = ny; g->nz = nz;
  g->n = (size_t)nx * ny * nz;
  g->c = *c;
  g->prec = c->precision;
  g->ws = ws;
  g->lay = layout_for(nx, ny, nz, c->precision);
  g->sc = (Scalars*)(ws + g->lay.scalars);
  g->sc_in = g->sc + 1;
  g->sc_aux = g->sc + 2;
  g->partials = (double*)(ws + g->lay.partials);
  for (int q = 0; q < kVecs; ++q) g->vec[q] = ws + g->lay.vec[q];
  g->b64 = g->prec == WFA_F32_IR64 ? (double*)(ws + g->lay.b64) : nullptr;
  g->d32 = g->prec == WFA_F32_IR64 ? (float*)(ws + g->lay.d32) : nullptr;
  g->op64 = make_op<double>(*c);
  g->op32 = make_op<float>(*c);
  g->method = WFA_METHOD_BICGSTAB;
  g->persistent = 0;
  g->profile = 0;
  g->force_bd = 0;
  g->check_every = 0;
  g->zchunk = 0;
  g->ir_inner_tol = 1e-4;
  g->force_div = 0;
  g->hint_iters = 0;
  const int w = g->prec == WFA_F32 ? 4 : 8;
  g->ry = 0;
  g->jacobi = 0;
  g->graph = 0;
  g->fuse = 0;
  g->shadow = 0;
  g->recompute_t = 0;
  g->tl = make_tiling(nx, ny, nz, w, 0, 0);
  g->tl32 = make_tiling(nx, ny, nz, 4, 0, 0);
}

// Rows per wave and z planes per workgroup (0 = default rule) of every
// stencil pass of the grid.
void apply_tiling(wfa_grid* g, int ry, int zc) {
  g->ry = ry;
  g->zchunk = zc;
  const int w = g->prec == WFA_F32 ? 4 : 8;
  g->tl = make_tiling(g->nx, g->ny, g->nz, w, zc, ry);
  g->tl32 = make_tiling(g->nx, g->ny, g->nz, 4, zc, ry);
  ++g->graphs.generation;
}

}  // namespace wfa

extern "C" int wfa_grid_create(int nx, int ny, int nz, const wfa_coeffs* c, void* workspace,
                               size_t workspace_bytes, wfa_grid** out) {
  if (!out) return set_error(WFA_ERR_INVALID, "out is NULL");
  *out = nullptr;
  int rc = validate_coeffs(nx, ny, nz, c);
  if (rc) return rc;
  if (!workspace) return set_error(WFA_ERR_INVALID, "workspace is NULL");
  if (((uintptr_t)workspace & 255) != 0)
    return set_error(WFA_ERR_INVALID, "workspace must be 256-byte aligned");
  const size_t need = wfa_workspace_bytes(nx, ny, nz, c->precision);
  if (workspace_bytes < need)
    return set_error(WFA_ERR_NOMEM, "workspace too small: %zu < %zu bytes", workspace_bytes, need);
  wfa_grid* g = new (std::nothrow) wfa_grid();
  if (!g) return set_error(WFA_ERR_NOMEM, "host allocation failed");
  grid_setup(g, nx, ny, nz, c, (char*)workspace);
  int ry = 0, zc = 0;
  if (tuned_tiling(nx, ny, nz, c->precision, c->mode, &ry, &zc)) apply_tiling(g, ry, zc);
  *out = g;
  return WFA_OK;
}

extern "C" int wfa_grid_destroy(wfa_grid* g) {
  if (!g) return set_error(WFA_ERR_INVALID, "grid is NULL");
  g->prof.clear();
  g->graphs.clear();
  g->rb.clear();
  delete g;
  return WFA_OK;
}

extern "C" int wfa_grid_set_option(wfa_grid* g, int option, int64_t value) {
  if (!g) return set_error(WFA_ERR_INVALID, "grid is NULL");
  switch (option) {
    case WFA_OPT_METHOD:
      if (value != WFA_METHOD_BICGSTAB && value != WFA_METHOD_CG &&
          value != WFA_METHOD_BICGSTAB2 && value != WFA_METHOD_CG1)
        return set_error(WFA_ERR_INVALID, "bad method %lld", (long long)value);
      g->method = (int)value;
      return WFA_OK;
    case WFA_OPT_PERSISTENT:
      if (value < -1 || value > 1) return set_error(WFA_ERR_INVALID, "bad persistent mode");
      g->persistent = (int)value;
      return WFA_OK;
    case WFA_OPT_PROFILE:
      if (value < 0 || value > (1 << 20)) return set_error(WFA_ERR_INVALID, "bad profile interval");
      g->profile = (int)value;
      for (auto& c : g->prof.seen) c = 0;
      return WFA_OK;
    case WFA_OPT_FORCE_BREAKDOWN:
      if (value < 0) return set_error(WFA_ERR_INVALID, "bad breakdown iteration");
      g->force_bd = (int)value;
      return WFA_OK;
    case WFA_OPT_CHECK_EVERY:
      if (value < 0 || value > 100000) return set_error(WFA_ERR_INVALID, "bad check interval");
      g->check_every = (int)value;
      return WFA_OK;
    case WFA_OPT_FORCE_DIVERGE:
      if (value < 0) return set_error(WFA_ERR_INVALID, "bad divergence iteration");
      g->force_div = (int)value;
      return WFA_OK;
    case WFA_OPT_IR_INNER_TOL:
      if (value <= 0) return set_error(WFA_ERR_INVALID, "bad inner tolerance");
      g->ir_inner_tol = (double)value * 1e-12;
      return WFA_OK;
    case WFA_OPT_JACOBI:
      if (value != 0 && value != 1) return set_error(WFA_ERR_INVALID, "Jacobi flag must be 0 or 1");
      g->jacobi = (int)value;
      ++g->graphs.generation;
      return WFA_OK;
    case WFA_OPT_EXPLICIT_FUSE:
      if (value < 0 || value > 4) return set_error(WFA_ERR_INVALID, "explicit fusion must be 0 to 4");
      if (value > 1 && g->c.mode != WFA_COEF_CONST)
        return set_error(WFA_ERR_INVALID, "fused explicit steps need a constant diffusivity");
      g->fuse = (int)value;
      return WFA_OK;
    case WFA_OPT_SHADOW:
      if (value != 0 && value != 1) return set_error(WFA_ERR_INVALID, "shadow mode must be 0 or 1");
      g->shadow = (int)value;
      return WFA_OK;
    case WFA_OPT_RECOMPUTE_T:
      if (value != 0 && value != 1) return set_error(WFA_ERR_INVALID, "recompute flag must be 0 or 1");
      g->recompute_t = (int)value;
      return WFA_OK;
    case WFA_OPT_GRAPH:
      if (value < -1 || value > 1) return set_error(WFA_ERR_INVALID, "graph mode must be -1, 0 or 1");
      g->graph = (int)value;
      return WFA_OK;
    case WFA_OPT_ZCHUNK:
    case WFA_OPT_RY: {
      if (option == WFA_OPT_ZCHUNK) {
        if (value < 0 || value > g->nz) return set_error(WFA_ERR_INVALID, "bad z chunk");
        g->zchunk = (int)value;
      } else {
        if (value != 0 && value != 1 && value != 2 && value != 4)
          return set_error(WFA_ERR_INVALID, "rows per wave must be 0, 1, 2 or 4");
        g->ry = (int)value;
      }
      apply_tiling(g, g->ry, g->zchunk);
      return WFA_OK;
    }
    default:
      return set_error(WFA_ERR_INVALID, "unknown option %d", option);
  }
}

extern "C" int wfa_grid_tiling(wfa_grid* g, int* tx, int* ty, int* zc, int* blocks) {
  if (!g) return set_error(WFA_ERR_INVALID, "grid is NULL");
  if (tx) *tx = kTX;
  if (ty) *ty = kWaves * g->tl.ry;
  if (zc) *zc = g->tl.geo.zc;
  if (blocks) *blocks = g->tl.geo.ntiles;
  return WFA_OK;
}

extern "C" int wfa_grid_vector(wfa_grid* g, int which, void** ptr) {
  if (!g || !ptr) return set_error(WFA_ERR_INVALID, "grid or ptr is NULL");
  if (which < 0 || which >= kVecs) return set_error(WFA_ERR_INVALID, "no vector %d", which);
  *ptr = g->vec[which];
  return WFA_OK;
}

// ---------------------------------------------------------------------------
// profiling
// ---------------------------------------------------------------------------
namespace wfa {

void Profiler::clear() {
  for (auto& p : pending) {
    (void)hipEventDestroy(p.e0);   // teardown: nothing to report a failure to
    (void)hipEventDestroy(p.e1);
  }
  pending.clear();
  for (auto e : pool) (void)hipEventDestroy(e);
  pool.clear();
}

hipEvent_t Profiler::get() {
  if (!pool.empty()) {
    hipEvent_t e = pool.back();
    pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

void Profiler::drain() {
  for (auto& p : pending) {
    float ms = 0.f;
    if (hipEventSynchronize(p.e1) == hipSuccess && hipEventElapsedTime(&ms, p.e0, p.e1) == hipSuccess) {
      launches[p.kernel] += 1;
      total_ms[p.kernel] += ms;
    }
    pool.push_back(p.e0);
    pool.push_back(p.e1);
  }
  pending.clear();
}

}  // namespace wfa

// Bracket one launch with events when profiling: every launch, or every
// profile-th launch of each kernel (the first, then one in profile).  A
// launch whose events could not be created or recorded is simply not
// counted.
struct ProfScope {
  wfa_grid* g;
  int kernel;
  hipStream_t s;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  bool armed = false;
  ProfScope(wfa_grid* g_, int k, hipStream_t s_) : g(g_), kernel(k), s(s_) {
    if (g->profile && (g->prof.seen[kernel]++ % g->profile) == 0) {
      e0 = g->prof.get();
      e1 = g->prof.get();
      armed = e0 && e1 && hipEventRecord(e0, s) == hipSuccess;
      if (!armed) {
        if (e0) g->prof.pool.push_back(e0);
        if (e1) g->prof.pool.push_back(e1);
      }
    }
  }
  ~ProfScope() {
    if (!armed) return;
    if (hipEventRecord(e1, s) == hipSuccess) {
      g->prof.pending.push_back({kernel, e0, e1});
    } else {
      g->prof.pool.push_back(e0);
      g->prof.pool.push_back(e1);
    }
  }
};

static double bytes_per_cell(const wfa_grid* g, int kernel) {
  const double w = g->prec == WFA_F32 ? 4.0 : 8.0;
  const double wi = g->prec == WFA_F32_IR64 ? 4.0 : w;  // inner vectors
  const double k = g->c.mode == WFA_COEF_CELL ? 4.0 : 0.0;
  switch (kernel) {
    case WFA_K_APPLY: return 2 * w + k;
    case WFA_K_INIT: return 4 * w + k;
    case WFA_K_PHASE_A: return 6 * wi + k;
    case WFA_K_PHASE_B: return 3 * wi + k;
    case WFA_K_PHASE_C: return 8 * wi;
    case WFA_K_RESIDUAL: return 2 * w + k + (g->prec == WFA_F32_IR64 ? 8.0 : 0.0);
    case WFA_K_PROMOTE: return 20.0;
    case WFA_K_CG_A: return 4 * wi + k;
    case WFA_K_CG_B: return 6 * wi;
    case WFA_K_PERSISTENT: return 17 * wi + 2 * k;
    // pass 1 reads r, v, t, p, x (+ r^) and writes x, r', p', v'; with
    // recompute_t it forms t instead of reading it
    case WFA_K_PHASE_AC: return ((g->shadow ? 9 : 10) - (g->recompute_t ? 1 : 0)) * wi + k;
    case WFA_K_EXPLICIT: return 2 * w + k;
    case WFA_K_EXPLICIT_FUSED: return 2 * w;  // one read, one write per pass
    // pass 2 reads r', v' (+ r^) and writes t, unless pass 1 forms t again
    case WFA_K_PHASE_B2: return ((g->shadow ? 3 : 4) - (g->recompute_t ? 1 : 0)) * wi + k;
    case WFA_K_CG1: return 10 * wi + k;  // r w s p x read; r' w' s' p x written
    default: return 0.0;
  }
}

extern "C" int wfa_kernel_stats(wfa_grid* g, int kernel, int64_t* launches, double* ms,
                                double* bytes_per_launch, int reset) {
  if (!g) return set_error(WFA_ERR_INVALID, "grid is NULL");
  if (kernel < 0 || kernel >= WFA_K_COUNT) return set_error(WFA_ERR_INVALID, "bad kernel id");
  g->prof.drain();
  if (launches) *launches = g->prof.launches[kernel];
  if (ms) *ms = g->prof.total_ms[kernel];
  if (bytes_per_launch) *bytes_per_launch = bytes_per_cell(g, kernel) * (double)g->n;
  if (reset) {
    for (int q = 0; q < WFA_K_COUNT; ++q) {
      g->prof.launches[q] = 0;
      g->prof.total_ms[q] = 0.0;
    }
  }
  return WFA_OK;
}

// ---------------------------------------------------------------------------
// launch contexts
// ---------------------------------------------------------------------------
template <typename T>
static Launch<T> ctx(wfa_grid* g, Scalars* sc, hipStream_t s);

template <>
Launch<double> ctx<double>(wfa_grid* g, Scalars* sc, hipStream_t s) {
  Launch<double> L{};
  L.tl = g->tl;
  L.op = g->op64;
  L.op.jac = (uint32_t)g->jacobi;
  L.cell = g->c.mode == WFA_COEF_CELL;
  L.kappa = (const float*)g->c.kappa;
  L.partials = g->partials;
  L.sc = sc;
  L.stream = s;
  return L;
}

template <>
Launch<float> ctx<float>(wfa_grid* g, Scalars* sc, hipStream_t s) {
  Launch<float> L{};
  L.tl = g->prec == WFA_F32 ? g->tl : g->tl32;
  L.op = g->op32;
  L.op.jac = (uint32_t)g->jacobi;
  L.cell = g->c.mode == WFA_COEF_CELL;
  L.kappa = (const float*)g->c.kappa;
  L.partials = g->partials;
  L.sc = sc;
  L.stream = s;
  return L;
}

// Launch context of the operator itself (no Jacobi scaling): true
// residuals, wfa_stencil_apply, wfa_rhs.
template <typename T>
static Launch<T> plain_ctx(wfa_grid* g, Scalars* sc, hipStream_t s) {
  Launch<T> L = ctx<T>(g, sc, s);
  L.op.jac = 0;
  return L;
}

static int check_launch(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_error(WFA_ERR_HIP, "%s launch: %s", what, hipGetErrorString(e));
  return WFA_OK;
}

namespace wfa {

int Readback::init() {
  if (host) return WFA_OK;
  if (sync) {
    host = local;
    return WFA_OK;
  }
  Scalars* h = nullptr;
  HIP_TRY(hipHostMalloc((void**)&h, kSlots * sizeof(Scalars), hipHostMallocDefault));
  hipEvent_t e = nullptr;
  const hipError_t ee = hipEventCreateWithFlags(&e, hipEventDisableTiming);
  if (ee != hipSuccess) {
    (void)hipHostFree(h);
    return set_error(WFA_ERR_HIP, "readback event: %s", hipGetErrorString(ee));
  }
  host = h;
  done = e;
  return WFA_OK;
}

void Readback::clear() {
  if (done) (void)hipEventDestroy(done);   // teardown: nothing to report a failure to
  if (host && !sync) (void)hipHostFree(host);
  done = nullptr;
  host = nullptr;
}

}  // namespace wfa

namespace wfa {

// Polls the event for up to 2 ms (the common wait on small grids is tens of
// microseconds), then blocks on it.
hipError_t wait_event(hipEvent_t e) {
  const auto t0 = std::chrono::steady_clock::now();
  hipError_t q;
  while ((q = hipEventQuery(e)) == hipErrorNotReady) {
    if (std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(2)) {
      q = hipEventSynchronize(e);
      break;
    }
  }
  // "not ready" is an answer, not a failure: leave no trace of it for the
  // calling thread's next hipGetLastError
  (void)hipGetLastError();
  return q;
}

}  // namespace wfa

static int wait_readback(wfa_grid* g) {
  const hipError_t e = wait_event(g->rb.done);
  if (e != hipSuccess) return set_error(WFA_ERR_HIP, "readback: %s", hipGetErrorString(e));
  if (g->profile) g->prof.drain();
  return WFA_OK;
}

// Host copies of one or two device scalar blocks, read together.
static int read_scalars(wfa_grid* g, const Scalars* dev, Scalars* host, hipStream_t s,
                        const Scalars* dev2 = nullptr, Scalars* host2 = nullptr) {
  int rc = g->rb.init();
  if (rc) return rc;
  HIP_TRY(hipMemcpyAsync(g->rb.host, dev, sizeof(Scalars), hipMemcpyDeviceToHost, s));
  if (dev2)
    HIP_TRY(hipMemcpyAsync(g->rb.host + 1, dev2, sizeof(Scalars), hipMemcpyDeviceToHost, s));
  if (g->rb.sync) {
    HIP_TRY(hipStreamSynchronize(s));
  } else {
    HIP_TRY(hipEventRecord(g->rb.done, s));
    if ((rc = wait_readback(g))) return rc;
  }
  *host = g->rb.host[0];
  if (dev2) *host2 = g->rb.host[1];
  return WFA_OK;
}

static int write_scalars(const Scalars* host, Scalars* dev, hipStream_t s) {
  launch_set_scalars(dev, *host, s);
  return check_launch("set scalars");
}

static int status_code(int dev_status) {
  switch (dev_status) {
    case ST_CONV: case ST_BZERO: return WFA_OK;
    case ST_NOCONV: return WFA_ERR_NOCONV;
    case ST_NONFINITE: return WFA_ERR_NONFINITE;
    case ST_BREAKDOWN: return WFA_ERR_BREAKDOWN;
    default: return WFA_ERR_NOCONV;
  }
}

// Iterations to launch before the next host check: an estimate of what
// remains from the residual history, bounded by the iteration budget.  The
// first chunk of a solve takes `hint` iterations when given (the count the
// grid's previous solve of the same kind converged in: successive time steps
// and refinements take similar counts, so most solves end in one chunk).
static int next_chunk(const wfa_grid* g, const Scalars& h, int budget, int hint) {
  int m;
  if (g->check_every > 0) {
    m = g->check_every;
  } else if (h.iter == 0 && hint > 0) {
    m = hint;
  } else if (h.iter == 0 || !(h.rr > 0.0) || !(h.rr0 > 0.0) || h.rr >= h.rr0) {
    m = 8;
  } else {
    const double rate = log(h.rr / h.rr0) / (double)h.iter;  // < 0
    const double target = log(h.tol * h.tol * h.bb);
    double rem = (target - log(h.rr)) / rate;
    if (!(rem > 0.0)) rem = 1.0;
    m = (int)ceil(rem * 1.05) + 1;
    if (m > 512) m = 512;
  }
  if (m > budget) m = budget;
  if (m < 1) m = 1;
  return m;
}

// ---------------------------------------------------------------------------
// persistent launches
// ---------------------------------------------------------------------------
// Grids up to this many cells iterate in one cooperative launch per chunk by
// default: below it, launch and dependency latency outweighs the three
// kernel boundaries' cache effects.
static const size_t kPersistentCells = (size_t)1 << 21;

static bool use_persistent(const wfa_grid* g, const Tiling& tl) {
  (void)tl;
  if (g->persistent == 1) return true;
  if (g->persistent == 0) return false;
  return g->n <= kPersistentCells;
}

static GridBarrier* barrier_of(wfa_grid* g) { return (GridBarrier*)(g->sc + 3); }

static int reset_barrier(wfa_grid* g, hipStream_t s) {
  static const GridBarrier zero{};
  HIP_TRY(hipMemcpyAsync(barrier_of(g), &zero, sizeof zero, hipMemcpyHostToDevice, s));
  return WFA_OK;
}

static int check_barrier(wfa_grid* g, hipStream_t s) {
  GridBarrier b{};
  HIP_TRY(hipMemcpyAsync(&b, barrier_of(g), sizeof b, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (b.timeout) return set_error(WFA_ERR_HIP, "persistent launch: grid barrier timed out");
  return WFA_OK;
}

// ---------------------------------------------------------------------------
// graph replay of iteration chunks
// ---------------------------------------------------------------------------
// A chunk of iterations is a fixed sequence of launches whose arguments do
// not change from one chunk to the next (the kernels read every Krylov
// scalar from the device).  Captured once as a graph of kGraphIters
// iterations, it is replayed with one launch instead of 2-3 per iteration;
// the kernels are the same, so the results are bitwise those of plain
// launches.  Off by default: measured on 32^3 to 256^3 grids it changes
// the time per iteration by under 2%, because what bounds a small grid's
// iteration is the GPU-side latency of each kernel (its dependent memory
// round trips and the cache maintenance between kernels), not the rate at
// which the host submits launches.  Option -1 selects it for grids up to
// kGraphCells cells.
static const int kGraphIters = 8;  // even: the double-buffer parity returns
static const size_t kGraphCells = (size_t)1 << 23;

void GraphCache::clear() {
  for (auto& e : entries) (void)hipGraphExecDestroy(e.exec);
  entries.clear();
  if (cap) (void)hipStreamDestroy(cap);
  cap = nullptr;
}

static bool use_graph(const wfa_grid* g) {
  if (g->profile) return false;  // per-launch events need plain launches
  if (g->graph == 1) return true;
  if (g->graph == 0) return false;
  return g->n <= kGraphCells;
}

// Launches the sequence `body` issues `reps` times, from a cached graph.
// `key` names the sequence: the method, the parity it starts at, the
// vectors it touches, the scalar block and the option generation.
template <typename T, typename Body>
static int replay(wfa_grid* g, const Launch<T>& L, const uint64_t (&key)[GraphCache::kKey],
                  int reps, Body&& body) {
  GraphCache& gc = g->graphs;
  hipGraphExec_t exec = nullptr;
  for (auto& e : gc.entries)
    if (memcmp(e.key, key, sizeof key) == 0) { exec = e.exec; break; }
  if (!exec) {
    if (!gc.cap) HIP_TRY(hipStreamCreateWithFlags(&gc.cap, hipStreamNonBlocking));
    Launch<T> Lc = L;
    Lc.stream = gc.cap;
    HIP_TRY(hipStreamBeginCapture(gc.cap, hipStreamCaptureModeThreadLocal));
    body(Lc);
    const hipError_t le = hipGetLastError();
    hipGraph_t graph = nullptr;
    const hipError_t ee = hipStreamEndCapture(gc.cap, &graph);
    if (le != hipSuccess || ee != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      return set_error(WFA_ERR_HIP, "graph capture: %s",
                       hipGetErrorString(le != hipSuccess ? le : ee));
    }
    const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ie != hipSuccess) return set_error(WFA_ERR_HIP, "graph instantiate: %s", hipGetErrorString(ie));
    if (gc.entries.size() >= GraphCache::kMaxEntries) {
      (void)hipGraphExecDestroy(gc.entries.front().exec);
      gc.entries.erase(gc.entries.begin());
    }
    GraphCache::Entry e;
    memcpy(e.key, key, sizeof key);
    e.exec = exec;
    gc.entries.push_back(e);
  }
  for (int i = 0; i < reps; ++i) HIP_TRY(hipGraphLaunch(exec, L.stream));
  return WFA_OK;
}

template <typename T>
static void graph_key(uint64_t (&k)[GraphCache::kKey], const wfa_grid* g, const Launch<T>& L,
                      int kind, int par, std::initializer_list<const void*> ptrs) {
  memset(k, 0, sizeof k);
  k[0] = (uint64_t)kind;
  k[1] = sizeof(T);
  k[2] = (uint64_t)par;
  k[3] = g->graphs.generation;
  k[4] = (uint64_t)(uintptr_t)L.sc;
  k[5] = (uint64_t)L.op.jac | ((uint64_t)L.shadow << 1);
  int q = 6;
  for (const void* p : ptrs) k[q++] = (uint64_t)(uintptr_t)p;
}

// ---------------------------------------------------------------------------
// BiCGStab (and CG) iteration loops on an initialised scalar block
// ---------------------------------------------------------------------------
// Runs iterations until the device status leaves ST_RUN.  A breakdown
// restarts from the true residual b - A x when `restartable`; otherwise the
// loop returns with h->restart set (the caller restarts at a higher level).
//
// The caller has queued the pass that initialises the scalar block; h holds
// the host's values for the block from before that pass (iteration count,
// limits).  The first chunk is queued behind that pass without reading it
// back (if it ended the solve, every pass of the chunk exits at its first
// instruction).  The same holds after a restart.
// Each chunk's scalars are read back once, together with the optional
// `tail`: a second scalar block, and a pass queued behind every chunk.

// Queued behind every chunk of iterations and read back with it.
struct ChunkTail {
  std::function<void()> launch;  // may be empty
  const Scalars* dev = nullptr;  // block read back with the solve's own
  Scalars* host = nullptr;
};

static int read_chunk(wfa_grid* g, const Scalars* dev, Scalars* h, hipStream_t s,
                      ChunkTail* tail) {
  if (tail && tail->launch) {
    tail->launch();
    int rc = check_launch("tail");
    if (rc) return rc;
  }
  return read_scalars(g, dev, h, s, tail ? tail->dev : nullptr, tail ? tail->host : nullptr);
}

template <typename T>
static int iterate_bicgstab(wfa_grid* g, const Launch<T>& L, T* x, T* r, T* rh, T** p, T** v,
                            T* t, const T* b, Scalars* h, int* restarts, bool restartable,
                            ChunkTail* tail, int hint) {
  int par = 0;
  int rc = WFA_OK;
  if (use_persistent(g, L.tl)) {
    if ((rc = reset_barrier(g, L.stream))) return rc;
    if ((rc = read_chunk(g, L.sc, h, L.stream, tail))) return rc;
  }
  while (h->status == ST_RUN) {
    if (h->restart) {
      if (!restartable) return WFA_OK;
      if (++*restarts > WFA_MAX_RESTARTS) { h->status = -1; return WFA_OK; }
      {
        ProfScope ps(g, WFA_K_INIT, L.stream);
        launch_init<T>(L, false, x, b, nullptr, r, rh);
      }
      if ((rc = check_launch("init"))) return rc;
      h->restart = 0;
      if (use_persistent(g, L.tl) && (rc = read_chunk(g, L.sc, h, L.stream, tail))) return rc;
      continue;
    }
    const int m = next_chunk(g, *h, h->maxit - h->iter, hint);
    if (use_persistent(g, L.tl)) {
      hipError_t e;
      {
        ProfScope ps(g, WFA_K_PERSISTENT, L.stream);
        e = launch_persistent_bicgstab<T>(L, x, r, rh, p[0], p[1], v[0], v[1], t, m, par,
                                          barrier_of(g));
      }
      if (e != hipSuccess)
        return set_error(WFA_ERR_HIP, "persistent launch: %s", hipGetErrorString(e));
      par ^= (m & 1);
      if ((rc = read_chunk(g, L.sc, h, L.stream, tail))) return rc;
      if ((rc = check_barrier(g, L.stream))) return rc;
      continue;
    }
    int q = 0;
    if (use_graph(g) && m >= kGraphIters) {
      uint64_t key[GraphCache::kKey];
      graph_key<T>(key, g, L, 0, par, {x, r, rh, p[0], p[1], v[0], v[1], t});
      const int p0 = par;
      rc = replay<T>(g, L, key, m / kGraphIters, [&](const Launch<T>& Lc) {
        int pp = p0;
        for (int k = 0; k < kGraphIters; ++k, pp ^= 1) {
          launch_phase_a<T>(Lc, r, p[pp], v[pp], p[pp ^ 1], v[pp ^ 1], rh);
          launch_phase_b<T>(Lc, r, v[pp ^ 1], t);
          launch_phase_c<T>(Lc, x, p[pp ^ 1], r, v[pp ^ 1], t, rh);
        }
      });
      if (rc) return rc;
      q = m - m % kGraphIters;
    }
    for (; q < m; ++q) {
      {
        ProfScope ps(g, WFA_K_PHASE_A, L.stream);
        launch_phase_a<T>(L, r, p[par], v[par], p[par ^ 1], v[par ^ 1], rh);
      }
      {
        ProfScope ps(g, WFA_K_PHASE_B, L.stream);
        launch_phase_b<T>(L, r, v[par ^ 1], t);
      }
      {
        ProfScope ps(g, WFA_K_PHASE_C, L.stream);
        launch_phase_c<T>(L, x, p[par ^ 1], r, v[par ^ 1], t, rh);
      }
      par ^= 1;
    }
    if ((rc = check_launch("phase"))) return rc;
    if ((rc = read_chunk(g, L.sc, h, L.stream, tail))) return rc;
  }
  return WFA_OK;
}

// Two-reduction BiCGStab: pass 1 reads r[par], p[par], v[par] and writes
// the [par ^ 1] buffers (r too: neighbours read the old r on the halo).
template <typename T>
static int iterate_bicgstab2(wfa_grid* g, const Launch<T>& L, T* x, T** r, T* rh, T** p, T** v,
                             T* t, const T* b, Scalars* h, int* restarts, int* par_io,
                             bool restartable, ChunkTail* tail, int hint) {
  int par = *par_io;
  int rc = WFA_OK;
  // With recompute_t pass 1 forms t = A s again and pass 2 stores nothing:
  // bitwise the same iterates, two vector streams fewer per iteration.
  const bool recompute = g->recompute_t != 0;
  auto pass_pair = [&](const Launch<T>& Lp, int pp) {
    {
      ProfScope ps(g, WFA_K_PHASE_AC, Lp.stream);
      if (recompute)
        launch_phase_act<T>(Lp, r[pp], v[pp], p[pp], rh, x, r[pp ^ 1], p[pp ^ 1], v[pp ^ 1]);
      else
        launch_phase_ac<T>(Lp, r[pp], v[pp], t, p[pp], rh, x, r[pp ^ 1], p[pp ^ 1], v[pp ^ 1]);
    }
    {
      ProfScope ps(g, WFA_K_PHASE_B2, Lp.stream);
      launch_phase_b2<T>(Lp, r[pp ^ 1], v[pp ^ 1], rh, recompute ? nullptr : t);
    }
  };
  while (h->status == ST_RUN) {
    if (h->restart) {
      if (!restartable) break;
      if (++*restarts > WFA_MAX_RESTARTS) { h->status = -1; break; }
      {
        ProfScope ps(g, WFA_K_INIT, L.stream);
        launch_init<T>(L, false, x, b, nullptr, r[par], rh);
      }
      if ((rc = check_launch("init"))) return rc;
      h->restart = 0;
      continue;
    }
    // maxit iterations take maxit + 1 first passes (the last applies the update)
    const int m = next_chunk(g, *h, h->maxit - h->iter + 1, hint);
    int q = 0;
    if (use_graph(g) && m >= kGraphIters) {
      uint64_t key[GraphCache::kKey];
      graph_key<T>(key, g, L, recompute ? 4 : 1, par,
                   {x, r[0], r[1], rh, p[0], p[1], v[0], v[1], t});
      const int p0 = par;
      rc = replay<T>(g, L, key, m / kGraphIters, [&](const Launch<T>& Lc) {
        int pp = p0;
        for (int k = 0; k < kGraphIters; ++k, pp ^= 1) pass_pair(Lc, pp);
      });
      if (rc) return rc;
      q = m - m % kGraphIters;
    }
    for (; q < m; ++q) {
      pass_pair(L, par);
      par ^= 1;
    }
    if ((rc = check_launch("bicgstab2"))) return rc;
    if ((rc = read_chunk(g, L.sc, h, L.stream, tail))) return rc;
  }
  *par_io = par;
  return WFA_OK;
}

template <typename T>
static int iterate_cg(wfa_grid* g, const Launch<T>& L, T* x, T* r, T** d, T* q, Scalars* h,
                      ChunkTail* tail, int hint) {
  int par = 0;
  int rc = WFA_OK;
  while (h->status == ST_RUN) {
    const int m = next_chunk(g, *h, h->maxit - h->iter, hint);
    int k = 0;
    if (use_graph(g) && m >= kGraphIters) {
      uint64_t key[GraphCache::kKey];
      graph_key<T>(key, g, L, 2, par, {x, r, d[0], d[1], q});
      const int p0 = par;
      rc = replay<T>(g, L, key, m / kGraphIters, [&](const Launch<T>& Lc) {
        int pp = p0;
        for (int j = 0; j < kGraphIters; ++j, pp ^= 1) {
          launch_cg_a<T>(Lc, r, d[pp], d[pp ^ 1], q);
          launch_cg_b<T>(Lc, x, d[pp ^ 1], r, q);
        }
      });
      if (rc) return rc;
      k = m - m % kGraphIters;
    }
    for (; k < m; ++k) {
      {
        ProfScope ps(g, WFA_K_CG_A, L.stream);
        launch_cg_a<T>(L, r, d[par], d[par ^ 1], q);
      }
      {
        ProfScope ps(g, WFA_K_CG_B, L.stream);
        launch_cg_b<T>(L, x, d[par ^ 1], r, q);
      }
      par ^= 1;
    }
    if ((rc = check_launch("cg"))) return rc;
    if ((rc = read_chunk(g, L.sc, h, L.stream, tail))) return rc;
  }
  return WFA_OK;
}

// CG with one reduction per iteration: one pass per iteration.  r, w and s
// are read on the halo, so each is double-buffered ([par] in, [par ^ 1]
// out); p and x are only touched at the own cell and are updated in place.
// The first pass after init only forms w0 = A r0 (and copies r0 across), so
// maxit iterations take maxit + 1 passes.
template <typename T>
static int iterate_cg1(wfa_grid* g, const Launch<T>& L, T* x, T** r, T** w, T** sv, T* p,
                       Scalars* h, ChunkTail* tail, int hint) {
  int par = 0;
  int rc = WFA_OK;
  while (h->status == ST_RUN) {
    // passes still needed: the iterations left, and w0 = A r0 if not formed
    const int m = next_chunk(g, *h, h->maxit - h->iter + (h->stage == 0 ? 1 : 0), hint);
    int k = 0;
    if (use_graph(g) && m >= kGraphIters) {
      uint64_t key[GraphCache::kKey];
      graph_key<T>(key, g, L, 3, par, {x, r[0], r[1], w[0], w[1], sv[0], sv[1], p});
      const int p0 = par;
      rc = replay<T>(g, L, key, m / kGraphIters, [&](const Launch<T>& Lc) {
        int pp = p0;
        for (int j = 0; j < kGraphIters; ++j, pp ^= 1)
          launch_phase_cg1<T>(Lc, r[pp], w[pp], sv[pp], p, x, r[pp ^ 1], w[pp ^ 1], sv[pp ^ 1]);
      });
      if (rc) return rc;
      k = m - m % kGraphIters;
    }
    for (; k < m; ++k) {
      {
        ProfScope ps(g, WFA_K_CG1, L.stream);
        launch_phase_cg1<T>(L, r[par], w[par], sv[par], p, x, r[par ^ 1], w[par ^ 1],
                            sv[par ^ 1]);
      }
      par ^= 1;
    }
    if ((rc = check_launch("cg1"))) return rc;
    if ((rc = read_chunk(g, L.sc, h, L.stream, tail))) return rc;
  }
  return WFA_OK;
}

static Scalars fresh_scalars(double tol, int maxit, int force_bd) {
  Scalars h{};
  h.tol = tol;
  h.maxit = maxit;
  h.iter = 0;
  h.force_bd = force_bd;
  h.scale = 1.0;
  h.inv_scale = 1.0;
  h.status = ST_RUN;
  h.counter = 0;
  return h;
}

// FP64 true relative residual of Tin-typed x and b.
template <typename Tin>
static int true_residual(wfa_grid* g, const Tin* b, const Tin* x, double* rel, hipStream_t s) {
  Scalars h = fresh_scalars(1.0, 1, 0);
  int rc = write_scalars(&h, g->sc_aux, s);
  if (rc) return rc;
  Launch<double> L = plain_ctx<double>(g, g->sc_aux, s);
  {
    ProfScope ps(g, WFA_K_RESIDUAL, s);
    launch_residual<Tin>(L, x, b, nullptr, nullptr, nullptr, 0, 0);
  }
  if ((rc = check_launch("residual"))) return rc;
  if ((rc = read_scalars(g, g->sc_aux, &h, s))) return rc;
  *rel = h.bb > 0.0 ? sqrt(h.rr / h.bb) : sqrt(h.rr);
  return WFA_OK;
}

// One solve of A x = b in the grid's own vector type T.
template <typename T>
static int solve_plain(wfa_grid* g, const T* b_user, T* x, bool form_b, double tol, int maxit,
                       wfa_solve_info* info, hipStream_t s) {
  auto t0 = std::chrono::steady_clock::now();
  T** vec = (T**)g->vec;
  T *r = vec[0], *rh = vec[1], *t = vec[2];
  T* p[2] = {vec[3], vec[4]};
  T* v[2] = {vec[5], vec[6]};
  T* bw = vec[7];
  Scalars h = fresh_scalars(tol, maxit, g->force_bd);
  g->force_bd = 0;
  int rc = write_scalars(&h, g->sc, s);
  if (rc) return rc;
  Launch<T> L = ctx<T>(g, g->sc, s);
  L.shadow = g->method == WFA_METHOD_BICGSTAB2 ? g->shadow : 0;
  const T* b = form_b ? bw : b_user;
  {
    ProfScope ps(g, WFA_K_INIT, s);
    launch_init<T>(L, form_b, x, b_user, bw, r, rh);
  }
  if ((rc = check_launch("init"))) return rc;
  // The true residual pass is queued behind every chunk and runs once the
  // solve has converged or used its iterations, so the chunk that ends the
  // solve also brings its true residual back.  (Not when profiling: there
  // every launch that is timed is one that does its work.)
  ChunkTail tail;
  Scalars ha = fresh_scalars(1.0, 1, 0);
  const bool use_tail = !g->profile;
  const Launch<double> La = plain_ctx<double>(g, g->sc_aux, s);
  if (use_tail) {
    if ((rc = write_scalars(&ha, g->sc_aux, s))) return rc;
    tail.launch = [&]() {
      launch_residual<T>(La, x, b, nullptr, nullptr, nullptr, 0, 0, g->sc);
    };
    tail.dev = g->sc_aux;
    tail.host = &ha;
  }
  int restarts = 0;
  T* rbuf[2] = {r, vec[8]};
  int rpar = 0;
  ChunkTail* tp = use_tail ? &tail : nullptr;
  const int hint = g->hint_iters;
  if (g->method == WFA_METHOD_CG) {
    rc = iterate_cg<T>(g, L, x, r, p, t, &h, tp, hint);
  } else if (g->method == WFA_METHOD_CG1) {
    T* w[2] = {v[0], v[1]};
    rc = iterate_cg1<T>(g, L, x, rbuf, w, p, t, &h, tp, hint);
  }
  else if (g->method == WFA_METHOD_BICGSTAB2)
    rc = iterate_bicgstab2<T>(g, L, x, rbuf, rh, p, v, t, b, &h, &restarts, &rpar, true, tp, hint);
  else
    rc = iterate_bicgstab<T>(g, L, x, r, rh, p, v, t, b, &h, &restarts, true, tp, hint);
  if (rc) return rc;
  g->hint_iters = h.status == ST_CONV && restarts == 0 ? h.iter : 0;
  int status;
  if (h.status == -1) status = WFA_ERR_BREAKDOWN;
  else status = status_code(h.status);
  if (h.status == ST_BZERO) {
    launch_fill<T>(g->n, x, T(0), s);
    if ((rc = check_launch("fill"))) return rc;
  }
  double rel_true = 0.0;
  if (status == WFA_ERR_NONFINITE) {
    rel_true = NAN;
  } else if (use_tail && (h.status == ST_CONV || h.status == ST_NOCONV)) {
    // the tail ran behind the chunk that ended the solve
    rel_true = ha.bb > 0.0 ? sqrt(ha.rr / ha.bb) : sqrt(ha.rr);
  } else {
    if ((rc = true_residual<T>(g, b, x, &rel_true, s))) return rc;
  }
  if (status != WFA_OK)
    set_error(status, "solve ended with %s after %d iterations (%d restarts)",
              status == WFA_ERR_NOCONV ? "NOCONV" : status == WFA_ERR_NONFINITE ? "NONFINITE"
              : "BREAKDOWN", h.iter, restarts);
  if (info) {
    info->status = status;
    info->iterations = h.iter;
    info->refinements = 0;
    info->restarts = restarts;
    info->rel_res_recursive = h.bb > 0.0 ? sqrt(h.rr / h.bb) : 0.0;
    info->rel_res_true = rel_true;
    info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  return status;
}

// Inner iterations allowed per refinement: the remaining budget, capped so
// that a slowly converging FP32 solve still hands back a correction.
int wfa::ir_inner_maxit(int maxit, int used) {
  const int left = maxit - used;
  const int cap = maxit / 4 > 500 ? maxit / 4 : 500;
  return left < cap ? left : cap;
}

// FP32 BiCGStab inside FP64 iterative refinement.
static int solve_ir(wfa_grid* g, const double* b_user, double* x, bool form_b, double tol,
                    int maxit, wfa_solve_info* info, hipStream_t s) {
  auto t0 = std::chrono::steady_clock::now();
  float** vec = (float**)g->vec;
  float *r = vec[0], *rh = vec[1], *t = vec[2];
  float* rbuf[2] = {vec[0], vec[8]};
  float* p[2] = {vec[3], vec[4]};
  float* v[2] = {vec[5], vec[6]};
  float* d = g->d32;
  int rc;
  Launch<double> L64 = plain_ctx<double>(g, g->sc, s);
  // the inner FP32 BiCGStab iterates on the Jacobi-scaled system D^{-1} A d =
  // D^{-1} r: far better conditioned when the diffusivity varies by orders
  // of magnitude, which FP32 BiCGStab needs to make progress at all there.
  // The inner CG (one reduction) keeps the symmetric A d = r.
  const bool cg1 = g->method == WFA_METHOD_CG1;
  float* w[2] = {v[0], v[1]};
  Launch<float> L32 = ctx<float>(g, g->sc_in, s);
  L32.op.jac = cg1 ? 0 : 1;
  // the inner solve's shadow residual (as the residual pass writes it); a
  // refinement whose inner solve diverged without a usable iterate under the
  // hashed one is repeated with r^ = r0, kept for the rest of the solve
  int shadow = g->shadow;
  L32.shadow = shadow;
  const double* b = b_user;
  if (form_b) {
    launch_rhs<double>(L64, x, g->b64);
    if ((rc = check_launch("rhs"))) return rc;
    b = g->b64;
  }
  const int max_ref = 30;
  int total_it = 0, refinements = 0, restarts = 0;
  double scale = 1.0, rec = 0.0;
  Scalars ho{}, hi{};
  int status = WFA_ERR_NOCONV;
  const int force_bd = g->force_bd;
  g->force_bd = 0;
  const int force_div = g->force_div;
  g->force_div = 0;
  g->hint_iters = 0;
  // > 0: this refinement repeats one whose inner solve diverged, stopping it
  // at the iteration that had reached its smallest residual (the kernels are
  // deterministic, so the repeat retraces the same iterates)
  int inner_cap = 0;
  for (int ref = 0;; ++ref) {
    ho = fresh_scalars(tol, maxit, 0);
    ho.scale = scale;
    ho.inv_scale = 1.0 / scale;
    hi = fresh_scalars(g->ir_inner_tol, inner_cap > 0 ? inner_cap : ir_inner_maxit(maxit, total_it),
                       ref == 0 ? force_bd : 0);
    hi.scale = scale;
    hi.inv_scale = 1.0 / scale;
    hi.guard = inner_cap > 0 ? 0.0 : kIrGuard;
    hi.force_div = ref == 0 ? force_div : 0;
    if ((rc = write_scalars(&ho, g->sc, s))) return rc;
    if ((rc = write_scalars(&hi, g->sc_in, s))) return rc;
    {
      ProfScope ps(g, WFA_K_RESIDUAL, s);
      launch_residual<double>(L64, x, b, r, rh, g->sc_in, cg1 ? 1 : 2, shadow);
    }
    if ((rc = check_launch("residual"))) return rc;
    const bool last = ref >= max_ref || total_it >= maxit;
    int inner_restarts = 0, inner_par = 0;
    if (last) {
      if ((rc = read_scalars(g, g->sc, &ho, s))) return rc;
    } else {
      // inner FP32 solve of A d = r32 from d = 0 with the two-reduction
      // BiCGStab (r32 sits in r[0]; an inner breakdown ends the inner solve
      // and the next refinement restarts it from the FP64 true residual).
      // Its first chunk is queued behind the residual pass, whose outer
      // scalars come back with the chunk's: when the residual already meets
      // the tolerance, the pass marks the inner solve converged and the
      // chunk's passes exit at once.
      ChunkTail outer;
      outer.dev = g->sc;
      outer.host = &ho;
      if (cg1)
        rc = iterate_cg1<float>(g, L32, d, rbuf, w, p, t, &hi, &outer, g->hint_iters);
      else
        rc = iterate_bicgstab2<float>(g, L32, d, rbuf, rh, p, v, t, nullptr, &hi,
                                      &inner_restarts, &inner_par, false, &outer, g->hint_iters);
      if (rc) return rc;
      g->hint_iters = hi.status == ST_CONV && !hi.restart && hi.iter > 0 ? hi.iter : 0;
    }
    if (ho.status != ST_RUN) {
      status = status_code(ho.status);
      if (ho.status == ST_BZERO) {
        launch_fill<double>(g->n, x, 0.0, s);
        if ((rc = check_launch("fill"))) return rc;
      }
      break;
    }
    if (last) { status = WFA_ERR_NOCONV; break; }
    if (hi.status == ST_RUN && hi.restart) ++restarts;
    if (restarts > WFA_MAX_RESTARTS) { status = WFA_ERR_BREAKDOWN; break; }
    total_it += hi.iter;
    rec = hi.bb > 0.0 ? sqrt(hi.rr / hi.bb) : 0.0;
    if (hi.status == ST_NONFINITE) { status = WFA_ERR_NONFINITE; break; }
    if (hi.diverged) {
      if (inner_cap == 0 && hi.it_min > 0) {  // repeat it, stopped at its best iterate
        inner_cap = hi.it_min;
        continue;
      }
      if (shadow && !cg1) {  // repeat it with r^ = r0 stored
        shadow = 0;
        L32.shadow = 0;
        inner_cap = 0;
        continue;
      }
      status = WFA_ERR_NOCONV;  // no usable correction
      break;
    }
    inner_cap = 0;
    if (hi.iter > 0) {
      ProfScope ps(g, WFA_K_PROMOTE, s);
      launch_promote(g->n, g->tl.pw_blocks, x, d, g->sc_in, s);
      if ((rc = check_launch("promote"))) return rc;
      ++refinements;
    }
    // next residual scaled by 2^-e so that its entries are O(1) in FP32
    const double rms = sqrt(ho.rr / (double)g->n);
    scale = (rms > 0.0 && isfinite(rms)) ? ldexp(1.0, -(int)lround(log2(rms))) : 1.0;
    if (hi.iter == 0 && hi.status != ST_RUN && hi.status != ST_CONV) {
      status = status_code(hi.status);
      break;
    }
  }
  if (status != WFA_OK)
    set_error(status, "refinement ended with %s after %d refinements, %d inner iterations "
              "(outer status %d, inner status %d, inner rr %.3e, outer rr %.3e)",
              status == WFA_ERR_NOCONV ? "NOCONV" : status == WFA_ERR_NONFINITE ? "NONFINITE"
              : "BREAKDOWN", refinements, total_it, ho.status, hi.status, hi.rr, ho.rr);
  if (info) {
    info->status = status;
    info->iterations = total_it;
    info->refinements = refinements;
    info->restarts = restarts;
    info->rel_res_recursive = rec;
    info->rel_res_true = ho.bb > 0.0 ? sqrt(ho.rr / ho.bb) : 0.0;
    if (status == WFA_ERR_NONFINITE) info->rel_res_true = NAN;
    info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  return status;
}

static int validate_solve(wfa_grid* g, const void* b, void* x, double tol, int maxit) {
  if (!g) return set_error(WFA_ERR_INVALID, "grid is NULL");
  if (!x) return set_error(WFA_ERR_INVALID, "x is NULL");
  if (!b) return set_error(WFA_ERR_INVALID, "b is NULL");
  if (!(tol > 0.0) || !isfinite(tol)) return set_error(WFA_ERR_INVALID, "tol must be > 0");
  if (maxit < 1) return set_error(WFA_ERR_INVALID, "maxit must be >= 1");
  return WFA_OK;
}

namespace wfa {
int solve_any(wfa_grid* g, const void* b, void* x, bool form_b, double tol, int maxit,
              wfa_solve_info* info, hipStream_t s) {
  const bool cg = g->method == WFA_METHOD_CG || g->method == WFA_METHOD_CG1;
  if (cg && (g->c.u[0] != 0.0 || g->c.u[1] != 0.0 || g->c.u[2] != 0.0))
    return set_error(WFA_ERR_INVALID, "CG needs a symmetric operator (u == 0)");
  if (g->jacobi && (cg || g->prec == WFA_F32_IR64))
    return set_error(WFA_ERR_INVALID,
                     "Jacobi scaling is available for BiCGStab on WFA_F64 / WFA_F32 grids");
  switch (g->prec) {
    case WFA_F64: return solve_plain<double>(g, (const double*)b, (double*)x, form_b, tol, maxit, info, s);
    case WFA_F32: return solve_plain<float>(g, (const float*)b, (float*)x, form_b, tol, maxit, info, s);
    default:
      // the inner solve is the two-reduction BiCGStab, or CG with one reduction
      if (g->method == WFA_METHOD_CG)
        return set_error(WFA_ERR_INVALID,
                         "WFA_F32_IR64 grids iterate with BiCGStab or the one-reduction CG");
      return solve_ir(g, (const double*)b, (double*)x, form_b, tol, maxit, info, s);
  }
}
}  // namespace wfa

extern "C" int wfa_bicgstab_solve(wfa_grid* g, const void* b, void* x, double tol, int maxit,
                                  wfa_solve_info* info, void* stream) {
  int rc = validate_solve(g, b, x, tol, maxit);
  if (rc) return rc;
  const int saved = g->method;
  g->method = WFA_METHOD_BICGSTAB;
  rc = solve_any(g, b, x, false, tol, maxit, info, (hipStream_t)stream);
  g->method = saved;
  return rc;
}

extern "C" int wfa_bicgstab2_solve(wfa_grid* g, const void* b, void* x, double tol, int maxit,
                                   wfa_solve_info* info, void* stream) {
  int rc = validate_solve(g, b, x, tol, maxit);
  if (rc) return rc;
  const int saved = g->method;
  g->method = WFA_METHOD_BICGSTAB2;
  rc = solve_any(g, b, x, false, tol, maxit, info, (hipStream_t)stream);
  g->method = saved;
  return rc;
}

extern "C" int wfa_cg_solve(wfa_grid* g, const void* b, void* x, double tol, int maxit,
                            wfa_solve_info* info, void* stream) {
  int rc = validate_solve(g, b, x, tol, maxit);
  if (rc) return rc;
  const int saved = g->method;
  g->method = WFA_METHOD_CG;
  rc = solve_any(g, b, x, false, tol, maxit, info, (hipStream_t)stream);
  g->method = saved;
  return rc;
}

extern "C" int wfa_cg1_solve(wfa_grid* g, const void* b, void* x, double tol, int maxit,
                             wfa_solve_info* info, void* stream) {
  int rc = validate_solve(g, b, x, tol, maxit);
  if (rc) return rc;
  const int saved = g->method;
  g->method = WFA_METHOD_CG1;
  rc = solve_any(g, b, x, false, tol, maxit, info, (hipStream_t)stream);
  g->method = saved;
  return rc;
}

extern "C" int wfa_timestep(wfa_grid* g, void* T, int nsteps, double tol, int maxit,
                            wfa_solve_info* info, void* stream) {
  int rc = validate_solve(g, T, T, tol, maxit);
  if (rc) return rc;
  if (nsteps < 0) return set_error(WFA_ERR_INVALID, "nsteps must be >= 0");
  for (int k = 0; k < nsteps; ++k) {
    rc = solve_any(g, nullptr, T, true, tol, maxit, info ? info + k : nullptr, (hipStream_t)stream);
    if (rc) return rc;
  }
  return WFA_OK;
}

extern "C" int wfa_stencil_apply(wfa_grid* g, const void* x, void* y, void* stream) {
  if (!g) return set_error(WFA_ERR_INVALID, "grid is NULL");
  if (!x || !y) return set_error(WFA_ERR_INVALID, "x and y must be non-NULL");
  const size_t w = g->prec == WFA_F32 ? 4 : 8;
  const char* xb = (const char*)x;
  const char* yb = (const char*)y;
  if (xb < yb + w * g->n && yb < xb + w * g->n)
    return set_error(WFA_ERR_INVALID, "x and y overlap");
  hipStream_t s = (hipStream_t)stream;
  if (g->prec == WFA_F32) {
    ProfScope ps(g, WFA_K_APPLY, s);
    launch_apply<float>(plain_ctx<float>(g, g->sc, s), (const float*)x, (float*)y);
  } else {
    ProfScope ps(g, WFA_K_APPLY, s);
    launch_apply<double>(plain_ctx<double>(g, g->sc, s), (const double*)x, (double*)y);
  }
  return check_launch("apply");
}

extern "C" int wfa_rhs(wfa_grid* g, const void* T, void* b, void* stream) {
  if (!g) return set_error(WFA_ERR_INVALID, "grid is NULL");
  if (!T || !b) return set_error(WFA_ERR_INVALID, "T and b must be non-NULL");
  hipStream_t s = (hipStream_t)stream;
  if (g->prec == WFA_F32)
    launch_rhs<float>(plain_ctx<float>(g, g->sc, s), (const float*)T, (float*)b);
  else
    launch_rhs<double>(plain_ctx<double>(g, g->sc, s), (const double*)T, (double*)b);
  return check_launch("rhs");
}

extern "C" int wfa_explicit_step(wfa_grid* g, void* T, int nsteps, void* stream) {
  if (!g || !T) return set_error(WFA_ERR_INVALID, "NULL argument");
  if (nsteps < 0) return set_error(WFA_ERR_INVALID, "nsteps must be >= 0");
  if (g->prec == WFA_F32_IR64)
    return set_error(WFA_ERR_INVALID, "explicit steps need a WFA_F64 or WFA_F32 grid");
  hipStream_t s = (hipStream_t)stream;
  const size_t w = g->prec == WFA_F32 ? 4 : 8;
  void* bufs[2] = {T, g->vec[0]};
  // automatic: the fastest measured on 512x512x1024 (FP32 3 steps per pass,
  // 1.29x one step per pass; FP64 2 steps, 1.32x); one step with a per-cell
  // diffusivity
  const int fuse = g->fuse > 0 ? g->fuse
                   : (g->c.mode != WFA_COEF_CONST ? 1 : (g->prec == WFA_F32 ? 3 : 2));
  int pass = 0;
  for (int done = 0; done < nsteps; ++pass) {
    const int k = nsteps - done >= fuse ? fuse : 1;
    const void* in = bufs[pass & 1];
    void* out = bufs[(pass + 1) & 1];
    if (k > 1) {
      ProfScope ps(g, WFA_K_EXPLICIT_FUSED, s);
      if (g->prec == WFA_F32)
        launch_explicit_fused<float>(plain_ctx<float>(g, g->sc, s), (const float*)in, (float*)out,
                                     k, g->zchunk);
      else
        launch_explicit_fused<double>(plain_ctx<double>(g, g->sc, s), (const double*)in,
                                      (double*)out, k, g->zchunk);
    } else {
      ProfScope ps(g, WFA_K_EXPLICIT, s);
      if (g->prec == WFA_F32)
        launch_explicit<float>(plain_ctx<float>(g, g->sc, s), (const float*)in, (float*)out);
      else
        launch_explicit<double>(plain_ctx<double>(g, g->sc, s), (const double*)in, (double*)out);
    }
    done += k;
  }
  int rc = check_launch("explicit");
  if (rc) return rc;
  if (pass & 1) HIP_TRY(hipMemcpyAsync(T, bufs[1], w * g->n, hipMemcpyDeviceToDevice, s));
  return WFA_OK;
}

extern "C" int wfa_true_residual(wfa_grid* g, const void* b, const void* x, double* rel,
                                 void* stream) {
  if (!g || !b || !x || !rel) return set_error(WFA_ERR_INVALID, "NULL argument");
  if (g->prec == WFA_F32)
    return true_residual<float>(g, (const float*)b, (const float*)x, rel, (hipStream_t)stream);
  return true_residual<double>(g, (const double*)b, (const double*)x, rel, (hipStream_t)stream);
}

extern "C" int wfa_stream_probe(const void* src, void* dst, size_t bytes, int reps, double* gbps,
                                void* stream) {
  return wfa_bandwidth_probe(WFA_PROBE_COPY, 0, src, dst, bytes, reps, gbps, stream);
}

extern "C" int wfa_bandwidth_probe(int kind, int blocks, const void* src, void* dst, size_t bytes,
                                   int reps, double* gbps, void* stream) {
  if (kind < WFA_PROBE_COPY || kind > WFA_PROBE_MIX_3R1W)
    return set_error(WFA_ERR_INVALID, "unknown probe kind %d", kind);
  const bool reads = probe_reads(kind) > 0;
  const size_t unit = kind == WFA_PROBE_COPY32 ? 32 : 16;
  if ((reads && !src) || !dst || !gbps || reps < 1 || bytes < unit || (bytes % unit) != 0 ||
      blocks < 0 || blocks > (1 << 20))
    return set_error(WFA_ERR_INVALID, "bad bandwidth probe arguments");
  if (bytes > ((size_t)1 << 40))
    return set_error(WFA_ERR_INVALID, "probe streams of at most 1 TiB");
  if (kind == WFA_PROBE_READ && bytes < (size_t)kThreads * 16)
    return set_error(WFA_ERR_INVALID, "read probe needs at least %d bytes", kThreads * 16);
  if ((((uintptr_t)src) | ((uintptr_t)dst)) & (unit - 1))
    return set_error(WFA_ERR_INVALID, "probe buffers must be %zu-byte aligned", unit);
  // measured: 8192 workgroups the fastest of 2048, 4096 and 8192 for the copy
  const int nb = blocks ? blocks : 256 * 32;
  hipError_t e = hipSuccess;
  *gbps = bandwidth_probe(kind, nb, src, dst, bytes, reps, (hipStream_t)stream, &e);
  if (e != hipSuccess) return set_error(WFA_ERR_HIP, "probe: %s", hipGetErrorString(e));
  return WFA_OK;
}
