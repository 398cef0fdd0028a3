// Continuous-batching server: many backward-Euler solves resident in one
// caller-provided HBM arena, advanced together by batched launches.
//
// A host worker thread owns the GPU side.  Each round it
//   1. admits queued requests in arrival order while a slot is free and the
//      arena can hold the request's Krylov workspace (a request first in
//      line that does not fit lets later ones that fit go ahead, a bounded
//      number of times);
//   2. starts new requests (right-hand side + first residual) and refines
//      requests whose inner solve ended (FP64 update + FP64 residual);
//   3. launches `chunk` batched BiCGStab iterations over every resident
//      solve (finished or paused solves are skipped on the device);
//   4. reads all slots' device scalar blocks with one copy and retires,
//      refines or restarts requests.
// Requests are split into up to kMaxLanes size classes by their cell count
// (WFA_OPT_SIZE_CLASS_*), each served by its own worker thread, HIP stream,
// slots and tables: a small request's rounds do not wait for a large
// request's passes.  The arena, the options and the tickets are shared.
// A request's arithmetic never depends on its neighbours (tiles, partial
// sums, reduction order and decisions are per solve), so its result is the
// same alone, in any mix and in any class.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "batched.hpp"
#include "host.hpp"
#include "internal.hpp"
#include "wfa.h"

using namespace wfa;

namespace {

constexpr int kScalarsPerSlot = 4;
constexpr int kMaxLanes = 4;   // size classes, each with its own worker and stream
// Default upper bounds (cells) of the size classes: 96^3 and 152^3, i.e.
// three classes.  Measured on a 2000-request stream of 32^3..192^3 grids.
constexpr int64_t kDefaultClassBound[kMaxLanes - 1] = {884736, 3511808, 0};

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// First-fit allocator over [0, size) with coalescing free list.
struct Heap {
  std::map<size_t, size_t> free_;  // offset -> length
  size_t size = 0;
  void init(size_t n) { size = n; free_.clear(); if (n) free_[0] = n; }
  bool alloc(size_t n, size_t* off) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= n) {
        *off = it->first;
        const size_t rest = it->second - n;
        const size_t o = it->first + n;
        free_.erase(it);
        if (rest) free_[o] = rest;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t n) {
    auto it = free_.emplace(off, n).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
};

enum Phase { Q_QUEUED, R_START, R_ITER, R_REFINE, R_FINAL, R_DONE };

// Every served solve starts with the index-hashed shadow residual (one
// vector stream less per pass than storing r0), as a grid does with
// WFA_OPT_SHADOW; a refinement whose inner solve diverged without a usable
// iterate is repeated with r^ = r0 stored, and the request keeps it.
constexpr int kServerShadow = 1;

struct Request {
  uint64_t ticket;
  int nx, ny, nz;
  wfa_coeffs c;
  void* T;
  double tol;
  int maxit;
  Phase phase = Q_QUEUED;
  int slot = -1;
  size_t off = 0, bytes = 0;
  wfa_grid g{};
  int total_it = 0, refinements = 0, restarts = 0;
  int inner_cap = 0;  // > 0: repeating a diverged inner solve up to its best iterate
  int passed_over = 0;  // later requests admitted while this one, first in line, did not fit
  int lane = 0;         // size class serving the request
  int par = 0;        // buffer parity of the next iteration (0 after every (re)start)
  int cg1 = 0;        // 1: iterates with CG with one reduction (symmetric request)
  int shadow = kServerShadow;  // 1: hashed r^; 0: r^ = r0, stored
  double inner_tol = 1e-4;     // FP32 inner solve's relative tolerance (fixed at submission)
  double scale = 1.0;
  double last_rec = 0.0;
  double t_submit = 0.0, t_done = 0.0;
  wfa_solve_info info{};
  int code = WFA_PENDING;
};

}  // namespace

struct wfa_server {
  char* arena;
  size_t arena_bytes;
  int max_slots;               // resident solves per size class
  // One size class: its worker thread, stream, slots, device tables (inside
  // the arena) and their pinned host mirrors.  The tables are uploaded with
  // asynchronous copies, and the slot scalars written back into their mapped
  // mirror by a kernel at the end of each round; the worker rewrites a table
  // only after the round that uploaded it has been waited for.
  struct Lane {
    int id = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;         // created by the server (classes above the first)
    Scalars* slot_sc = nullptr;      // device: max_slots * kScalarsPerSlot
    SolveDesc<float>* d32 = nullptr;   // device: max_slots
    SolveDesc<double>* d64 = nullptr;  // device: max_slots
    int* bases = nullptr;            // device: 4 * (max_slots + 1)
    GridBarrier* bar = nullptr;      // device: grid barrier of a persistent round
    Scalars* h_sc = nullptr;         // pinned mirrors of the above
    uint32_t* h_sc_dev = nullptr;    // h_sc as the device addresses it
    uint32_t* flag = nullptr;        // pinned: number of the last round read back
    uint32_t* flag_dev = nullptr;    // the same word as the device addresses it
    uint32_t round_seq = 0;
    SolveDesc<float>* h_d32 = nullptr;
    SolveDesc<double>* h_d64 = nullptr;
    int* h_bases = nullptr;
    GridBarrier* h_bar = nullptr;
    hipEvent_t round_done = nullptr; // the round's scalar readback
    std::condition_variable cv_work;
    std::deque<Request*> queue;
    std::vector<Request*> slots;
    int ry = 0;                      // rows per wave of every resident solve's tiling
    std::vector<char> last_d32, last_d64, last_bases;  // bytes of the last table uploads
    std::thread worker;
  };
  Lane lanes[kMaxLanes];
  int64_t class_bound[kMaxLanes - 1];  // cell-count upper bounds of the classes (0: unused)
  size_t heap_base;
  Heap heap;
  void* pinned = nullptr;
  // requests
  std::mutex mu;
  std::condition_variable cv_done;
  std::map<uint64_t, Request*> reqs;
  uint64_t next_ticket = 1;
  int inflight = 0;  // queued + resident
  bool stop = false;
  std::atomic<int> worker_error{WFA_OK};
  std::mutex err_mu;
  char worker_msg[256] = "";
  int chunk = 4;      // iterations per round (WFA_OPT_CHECK_EVERY)
  double ir_inner_tol = 1e-4;  // WFA_OPT_IR_INNER_TOL for requests submitted from now on
  int persistent = 0; // 1: a round is one cooperative launch per precision (WFA_OPT_PERSISTENT)
  int method = WFA_METHOD_BICGSTAB2;  // WFA_OPT_METHOD: _CG1 for symmetric requests
  int64_t cg1_max_cells = 0;          // WFA_OPT_CG1_MAX_CELLS (0: no limit)
};

namespace {

bool is_f32_batch(const Request* r) { return r->c.precision != WFA_F64; }

// Workspace bytes one request needs from the heap.
size_t request_bytes(int nx, int ny, int nz, int precision) {
  return align256(wfa_workspace_bytes(nx, ny, nz, precision));
}

// Record a worker's failure (the first one's message is kept).
int fail_code(wfa_server* sv, int code, const char* msg) {
  std::lock_guard<std::mutex> lk(sv->err_mu);
  if (sv->worker_error.load() == WFA_OK) {
    snprintf(sv->worker_msg, sizeof sv->worker_msg, "%s", msg);
    sv->worker_error.store(code);
  }
  return code;
}

int fail(wfa_server* sv, const char* what, hipError_t e) {
  char msg[256];
  snprintf(msg, sizeof msg, "%s: %s", what, hipGetErrorString(e));
  return fail_code(sv, WFA_ERR_HIP, msg);
}

wfa_server::Lane& lane_of(wfa_server* sv, const Request* r) { return sv->lanes[r->lane]; }

// A persistent round's waits are bounded: a barrier wait that gives up (after
// about this many polls of a few cycles' sleep each) makes every wave leave,
// and the server reports the failure instead of hanging.
constexpr int kRoundSpinLimit = 1 << 22;

// Host-to-device copy of a table; remembers the first failure.
int put(wfa_server* sv, hipStream_t st, void* dst, const void* src, size_t bytes) {
  const hipError_t e = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st);
  return e == hipSuccess ? WFA_OK : fail(sv, "table upload", e);
}

// Upload a table only when its bytes differ from the last upload: between
// admissions, refinements and retirements the resident set's tables repeat
// from round to round, and each copy is a dependent step on the stream.
int put_changed(wfa_server* sv, hipStream_t st, void* dst, const void* src, size_t bytes,
                std::vector<char>* last) {
  if (last->size() == bytes && memcmp(last->data(), src, bytes) == 0) return WFA_OK;
  const int rc = put(sv, st, dst, src, bytes);
  if (rc == WFA_OK) last->assign((const char*)src, (const char*)src + bytes);
  else last->clear();
  return rc;
}

// Sets `count` consecutive device scalar blocks from kernel arguments.
int put_scalars(wfa_server* sv, hipStream_t st, Scalars* dst, const Scalars* h, int count) {
  for (int k = 0; k < count; ++k) launch_set_scalars(dst + k, h[k], st);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? WFA_OK : fail(sv, "scalar upload", e);
}

Scalars fresh(double tol, int maxit) {
  Scalars h{};
  h.tol = tol;
  h.maxit = maxit;
  h.scale = 1.0;
  h.inv_scale = 1.0;
  h.status = ST_RUN;
  return h;
}

template <typename T>
SolveDesc<T> make_desc(Request* r, T* x) {
  wfa_grid& g = r->g;
  SolveDesc<T> d{};
  const Tiling& tl = (sizeof(T) == 4 && g.prec == WFA_F32_IR64) ? g.tl32 : g.tl;
  d.geo = tl.geo;
  if constexpr (sizeof(T) == 4) d.op = g.op32; else d.op = g.op64;
  // the inner FP32 BiCGStab of refinement iterates on D^{-1} A (as
  // wfa_timestep); CG keeps the symmetric A
  d.op.jac = g.prec == WFA_F32_IR64 && !r->cg1 ? 1u : 0u;
  d.kappa = (const float*)g.c.kappa;
  T** v = (T**)g.vec;
  d.x = x;
  d.r = v[0]; d.rh = v[1]; d.t = v[2]; d.p0 = v[3]; d.p1 = v[4]; d.v0 = v[5]; d.v1 = v[6];
  d.r1 = v[8];
  d.par = r->par;
  d.hashed = r->shadow;
  d.cg1 = r->cg1;
  d.partials = g.partials;
  d.sc = g.prec == WFA_F32_IR64 ? g.sc_in : g.sc;
  d.n = g.n;
  d.cell = g.c.mode == WFA_COEF_CELL;
  d.pw_blocks = tl.pw_blocks;
  return d;
}

// Start a just-admitted request: right-hand side and first residual (IR)
// or the BiCGStab initialisation (plain).
int start_request(wfa_server* sv, Request* r) {
  wfa_grid& g = r->g;
  hipStream_t s = lane_of(sv, r).stream;
  r->par = 0;  // the first residual goes to the parity-0 buffer
  if (g.prec == WFA_F32_IR64) {
    Scalars h2[2] = {fresh(r->tol, r->maxit), fresh(r->inner_tol, ir_inner_maxit(r->maxit, 0))};
    h2[1].guard = kIrGuard;
    if (int rc = put_scalars(sv, s, g.sc, h2, 2)) return rc;
    Launch<double> L{g.tl, g.op64, g.c.mode == WFA_COEF_CELL, (const float*)g.c.kappa,
                     g.partials, g.sc, s};
    launch_rhs<double>(L, (const double*)r->T, g.b64);
    float** v = (float**)g.vec;
    launch_residual<double>(L, (const double*)r->T, g.b64, v[0], v[1], g.sc_in, r->cg1 ? 1 : 2,
                            r->shadow);
  } else {
    const Scalars h = fresh(r->tol, r->maxit);
    if (int rc = put_scalars(sv, s, g.sc, &h, 1)) return rc;
    if (g.prec == WFA_F64) {
      Launch<double> L{g.tl, g.op64, g.c.mode == WFA_COEF_CELL, (const float*)g.c.kappa,
                       g.partials, g.sc, s};
      double** v = (double**)g.vec;
      L.shadow = r->shadow;
      launch_init<double>(L, true, (double*)r->T, nullptr, v[7], v[0], v[1]);
    } else {
      Launch<float> L{g.tl, g.op32, g.c.mode == WFA_COEF_CELL, (const float*)g.c.kappa,
                      g.partials, g.sc, s};
      float** v = (float**)g.vec;
      L.shadow = r->shadow;
      launch_init<float>(L, true, (float*)r->T, nullptr, v[7], v[0], v[1]);
    }
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(sv, "start", e);
  r->phase = R_ITER;
  return WFA_OK;
}

// IR: apply the inner correction and compute the next FP64 residual.
int refine_request(wfa_server* sv, Request* r, double scale_next, bool promote) {
  wfa_grid& g = r->g;
  hipStream_t s = lane_of(sv, r).stream;
  if (promote) launch_promote(g.n, g.tl.pw_blocks, (double*)r->T, g.d32, g.sc_in, s);
  Scalars h2[2] = {fresh(r->tol, r->maxit),
                   fresh(r->inner_tol, r->inner_cap > 0 ? r->inner_cap : ir_inner_maxit(r->maxit, r->total_it))};
  Scalars& ho = h2[0];
  Scalars& hi = h2[1];
  ho.scale = scale_next; ho.inv_scale = 1.0 / scale_next;
  hi.scale = scale_next; hi.inv_scale = 1.0 / scale_next;
  hi.guard = r->inner_cap > 0 ? 0.0 : kIrGuard;
  if (int rc = put_scalars(sv, s, g.sc, h2, 2)) return rc;
  Launch<double> L{g.tl, g.op64, g.c.mode == WFA_COEF_CELL, (const float*)g.c.kappa,
                   g.partials, g.sc, s};
  float** v = (float**)g.vec;
  launch_residual<double>(L, (const double*)r->T, g.b64, v[0], v[1], g.sc_in, r->cg1 ? 1 : 2,
                          r->shadow);
  r->par = 0;
  r->scale = scale_next;
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(sv, "refine", e);
  r->phase = R_ITER;
  return WFA_OK;
}

// Plain precisions: FP64 true residual of the final iterate into sc_aux.
int final_residual(wfa_server* sv, Request* r) {
  wfa_grid& g = r->g;
  hipStream_t s = lane_of(sv, r).stream;
  const Scalars ha = fresh(1.0, 1);
  if (int rc = put_scalars(sv, s, g.sc_aux, &ha, 1)) return rc;
  Launch<double> L{g.tl, g.op64, g.c.mode == WFA_COEF_CELL, (const float*)g.c.kappa,
                   g.partials, g.sc_aux, s};
  void** v = g.vec;
  if (g.prec == WFA_F64)
    launch_residual<double>(L, (const double*)r->T, (const double*)v[7], nullptr, nullptr, nullptr,
                            0, 0);
  else
    launch_residual<float>(L, (const float*)r->T, (const float*)v[7], nullptr, nullptr, nullptr,
                           0, 0);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(sv, "final residual", e);
  r->phase = R_FINAL;
  return WFA_OK;
}

void retire(wfa_server* sv, Request* r, int code, double rel_true) {
  r->t_done = now_s();
  r->code = code;
  r->info.status = code;
  r->info.iterations = r->total_it;
  r->info.refinements = r->refinements;
  r->info.restarts = r->restarts;
  r->info.rel_res_recursive = r->last_rec;
  r->info.rel_res_true = rel_true;
  r->info.seconds = r->t_done - r->t_submit;
  r->phase = R_DONE;
  sv->heap.release(r->off, r->bytes);
  lane_of(sv, r).slots[r->slot] = nullptr;
  r->slot = -1;
  --sv->inflight;
}

int code_of(int st) {
  switch (st) {
    case ST_CONV: case ST_BZERO: return WFA_OK;
    case ST_NOCONV: return WFA_ERR_NOCONV;
    case ST_NONFINITE: return WFA_ERR_NONFINITE;
    case ST_BREAKDOWN: return WFA_ERR_BREAKDOWN;
    default: return WFA_ERR_NOCONV;
  }
}

// Inspect one resident request after a round (scalars already on the host).
int advance(wfa_server* sv, Request* r) {
  wfa_server::Lane& ln = lane_of(sv, r);
  const Scalars* hs = &ln.h_sc[r->slot * kScalarsPerSlot];
  wfa_grid& g = r->g;
  if (r->phase == R_FINAL) {
    // IR: the outer block holds the FP64 residual of the last refinement;
    // plain precisions: the true residual went to the aux block
    const Scalars& a = g.prec == WFA_F32_IR64 ? hs[0] : hs[2];
    // b = 0 under refinement: x = 0 was filled in, the residual is zero
    const double rel = g.prec == WFA_F32_IR64 && a.status == ST_BZERO ? 0.0
                       : a.bb > 0.0 ? sqrt(a.rr / a.bb) : sqrt(a.rr);
    int code = r->code;
    if (g.prec == WFA_F32_IR64 && a.status == ST_CONV) code = WFA_OK;
    retire(sv, r, code, rel);
    return WFA_OK;
  }
  if (g.prec == WFA_F32_IR64) {
    const Scalars& o = hs[0];
    const Scalars& in = hs[1];
    if (o.status == ST_BZERO) {
      // x = 0 solves A x = 0.  The fill runs on the server's stream; the
      // request retires when the next round's readback, queued behind it,
      // comes back, so a caller never sees T before the fill has run.
      launch_fill<double>(g.n, (double*)r->T, 0.0, ln.stream);
      hipError_t e = hipGetLastError();
      if (e != hipSuccess) return fail(sv, "fill", e);
      r->code = WFA_OK;
      r->phase = R_FINAL;
      return WFA_OK;
    }
    if (o.status != ST_RUN) {
      retire(sv, r, code_of(o.status), o.bb > 0.0 ? sqrt(o.rr / o.bb) : 0.0);
      return WFA_OK;
    }
    if (in.status == ST_RUN && !in.restart) return WFA_OK;  // still iterating
    r->total_it += in.iter;
    r->last_rec = in.bb > 0.0 ? sqrt(in.rr / in.bb) : 0.0;
    if (in.restart) ++r->restarts;
    if (in.status == ST_NONFINITE) {
      retire(sv, r, WFA_ERR_NONFINITE, NAN);
      return WFA_OK;
    }
    if (in.diverged) {
      if (r->inner_cap == 0 && in.it_min > 0) {
        // repeat this refinement, stopping the inner solve at the iteration
        // that had reached its smallest residual (deterministic kernels
        // retrace the same iterates); nothing is promoted
        r->inner_cap = in.it_min;
        r->phase = R_REFINE;
        return refine_request(sv, r, r->scale, false);
      }
      if (r->shadow && !r->cg1) {
        // no usable correction with the hashed shadow residual: repeat the
        // refinement with r^ = r0 (the residual pass stores it), nothing
        // promoted
        r->shadow = 0;
        r->inner_cap = 0;
        r->phase = R_REFINE;
        return refine_request(sv, r, r->scale, false);
      }
      retire(sv, r, WFA_ERR_NOCONV, sqrt(o.rr / o.bb));  // no usable correction
      return WFA_OK;
    }
    r->inner_cap = 0;
    if (r->restarts > WFA_MAX_RESTARTS) {
      retire(sv, r, WFA_ERR_BREAKDOWN, sqrt(o.rr / o.bb));
      return WFA_OK;
    }
    if (in.iter > 0) ++r->refinements;
    if (r->refinements >= 30 || r->total_it >= r->maxit) {
      // apply the last correction, then report the FP64 residual as NOCONV
      r->code = WFA_ERR_NOCONV;
    }
    const double rms = sqrt(o.rr / (double)g.n);
    const double scale = (rms > 0.0 && isfinite(rms)) ? ldexp(1.0, -(int)lround(log2(rms))) : 1.0;
    r->phase = R_REFINE;
    int rc = refine_request(sv, r, scale, true);
    if (rc) return rc;
    if (r->code == WFA_ERR_NOCONV) r->phase = R_FINAL;  // read the residual next round
    return WFA_OK;
  }
  // plain FP64 / FP32 BiCGStab
  const Scalars& h = hs[0];
  if (h.status == ST_RUN && !h.restart) return WFA_OK;
  if (h.status == ST_RUN && h.restart) {
    if (++r->restarts > WFA_MAX_RESTARTS) {
      r->total_it = h.iter;
      r->code = WFA_ERR_BREAKDOWN;
      return final_residual(sv, r);
    }
    r->par = 0;  // the restart's residual goes to the parity-0 buffer
    if (g.prec == WFA_F64) {
      Launch<double> L{g.tl, g.op64, g.c.mode == WFA_COEF_CELL, (const float*)g.c.kappa,
                       g.partials, g.sc, ln.stream};
      double** v = (double**)g.vec;
      L.shadow = r->shadow;
      launch_init<double>(L, false, (double*)r->T, v[7], nullptr, v[0], v[1]);
    } else {
      Launch<float> L{g.tl, g.op32, g.c.mode == WFA_COEF_CELL, (const float*)g.c.kappa,
                      g.partials, g.sc, ln.stream};
      float** v = (float**)g.vec;
      L.shadow = r->shadow;
      launch_init<float>(L, false, (float*)r->T, v[7], nullptr, v[0], v[1]);
    }
    return WFA_OK;
  }
  r->total_it = h.iter;
  r->last_rec = h.bb > 0.0 ? sqrt(h.rr / h.bb) : 0.0;
  r->code = code_of(h.status);
  if (h.status == ST_BZERO) {
    if (g.prec == WFA_F64) launch_fill<double>(g.n, (double*)r->T, 0.0, ln.stream);
    else launch_fill<float>(g.n, (float*)r->T, 0.0f, ln.stream);
  }
  return final_residual(sv, r);
}

// Rebuild the batched work tables of the resident set.
int build_tables(wfa_server* sv, wfa_server::Lane& ln, int* n32, int* tiles32, int* pw32,
                 int* n64, int* tiles64, int* pw64) {
  const int S = sv->max_slots;
  int a = 0, b = 0, t32 = 0, p32 = 0, t64 = 0, p64 = 0;
  int* tb32 = &ln.h_bases[0];
  int* pb32 = &ln.h_bases[S + 1];
  int* tb64 = &ln.h_bases[2 * (S + 1)];
  int* pb64 = &ln.h_bases[3 * (S + 1)];
  for (int s = 0; s < S; ++s) {
    Request* r = ln.slots[s];
    if (!r || (r->phase != R_ITER && r->phase != R_REFINE)) continue;
    const int ry = r->g.prec == WFA_F32_IR64 ? r->g.tl32.ry : r->g.tl.ry;
    if (ry != ln.ry) return fail_code(sv, WFA_ERR_INVALID, "tilings with different rows per wave");
    if (is_f32_batch(r)) {
      float* x = r->g.prec == WFA_F32_IR64 ? r->g.d32 : (float*)r->T;
      ln.h_d32[a] = make_desc<float>(r, x);
      tb32[a] = t32; pb32[a] = p32;
      t32 += ln.h_d32[a].geo.ntiles; p32 += ln.h_d32[a].pw_blocks;
      ++a;
    } else {
      ln.h_d64[b] = make_desc<double>(r, (double*)r->T);
      tb64[b] = t64; pb64[b] = p64;
      t64 += ln.h_d64[b].geo.ntiles; p64 += ln.h_d64[b].pw_blocks;
      ++b;
    }
  }
  tb32[a] = t32; pb32[a] = p32; tb64[b] = t64; pb64[b] = p64;
  *n32 = a; *tiles32 = t32; *pw32 = p32; *n64 = b; *tiles64 = t64; *pw64 = p64;
  return WFA_OK;
}

// Admission in arrival order while a slot and arena space are free.  A
// request first in line that does not fit lets later requests that fit go
// ahead, at most kMaxPassOver of them; then admission waits for it, so no
// request waits for ever behind smaller ones.
constexpr int kMaxPassOver = 16;
constexpr int kAdmitScan = 64;   // queued requests looked at per round

void admit(wfa_server* sv, wfa_server::Lane& ln, std::vector<Request*>* admitted) {
  Request* blocked = nullptr;  // the earliest request that did not fit
  int scanned = 0;
  for (auto it = ln.queue.begin(); it != ln.queue.end() && scanned < kAdmitScan; ++scanned) {
    Request* r = *it;
    if (blocked && blocked->passed_over >= kMaxPassOver) return;
    int slot = -1;
    for (int s = 0; s < sv->max_slots; ++s)
      if (!ln.slots[s]) { slot = s; break; }
    if (slot < 0) return;
    size_t off = 0;
    if (!sv->heap.alloc(r->bytes, &off)) {
      if (!blocked) blocked = r;
      ++it;
      continue;
    }
    if (blocked) ++blocked->passed_over;
    it = ln.queue.erase(it);
    r->slot = slot;
    r->off = off;
    ln.slots[slot] = r;
    admitted->push_back(r);
  }
}

// Fail every request of one class, resident or queued (under sv->mu).
void fail_lane(wfa_server* sv, wfa_server::Lane& ln, int rc) {
  for (auto*& r : ln.slots)
    if (r) { r->code = rc; r->phase = R_DONE; r->t_done = now_s(); r = nullptr; --sv->inflight; }
  for (auto* r : ln.queue) { r->code = rc; r->phase = R_DONE; r->t_done = now_s(); --sv->inflight; }
  ln.queue.clear();
  sv->cv_done.notify_all();
}

// Copies the slot scalar blocks of one class into their pinned host mirror
// (mapped, coherent), then writes the round's number into the mirror's flag
// word: every thread's stores are made visible at system scope before the
// workgroup barrier, and the flag is stored after it, so a host that sees
// the number sees the blocks.  One workgroup.
__global__ void __launch_bounds__(kThreads)
k_readback(const uint32_t* __restrict__ src, uint32_t* __restrict__ dst, size_t n,
           uint32_t* __restrict__ flag, uint32_t seq) {
  for (size_t e = threadIdx.x; e < n; e += kThreads) dst[e] = src[e];
  __threadfence_system();
  __syncthreads();
  if (threadIdx.x == 0)
    __hip_atomic_store(flag, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

void worker_main(wfa_server* sv, int lane) {
  wfa_server::Lane& ln = sv->lanes[lane];
  std::vector<Request*> admitted;
  while (true) {
    admitted.clear();
    int chunk = 0, persist = 0;  // this round's options
    {
      std::unique_lock<std::mutex> lk(sv->mu);
      if (const int err = sv->worker_error.load()) {
        // another class failed: the server stays unusable
        fail_lane(sv, ln, err);
        break;
      }
      chunk = sv->chunk;
      // only the first class runs cooperative rounds (while it is on, new
      // requests all go to that class)
      persist = lane == 0 ? sv->persistent : 0;
      admit(sv, ln, &admitted);
      bool any = false;
      for (auto* r : ln.slots) any = any || r != nullptr;
      if (!any && admitted.empty()) {
        if (sv->stop) break;
        ln.cv_work.wait(lk);
        continue;
      }
    }
    int rc = WFA_OK;
    for (Request* r : admitted) {
      char* ws = sv->arena + sv->heap_base + r->off;
      grid_setup(&r->g, r->nx, r->ny, r->nz, &r->c, ws);
      // a tuned plane depth for this grid key, where the tuned row count is
      // the one every resident solve shares (one launch covers them all)
      int t_ry = 0, t_zc = 0;
      const int shared_ry = r->g.prec == WFA_F32_IR64 ? r->g.tl32.ry : r->g.tl.ry;
      if (tuned_tiling(r->nx, r->ny, r->nz, r->c.precision, r->c.mode, &t_ry, &t_zc) &&
          t_ry == shared_ry)
        apply_tiling(&r->g, t_ry, t_zc);
      // the slot's scalar blocks live in the class's contiguous region
      r->g.sc = ln.slot_sc + r->slot * kScalarsPerSlot;
      r->g.sc_in = r->g.sc + 1;
      r->g.sc_aux = r->g.sc + 2;
      // every grid keeps the default rule's row count, so all share it
      ln.ry = r->g.prec == WFA_F32_IR64 ? r->g.tl32.ry : r->g.tl.ry;
      if ((rc = start_request(sv, r))) break;
    }
    int n32 = 0, t32 = 0, p32 = 0, n64 = 0, t64 = 0, p64 = 0;
    if (!rc) rc = build_tables(sv, ln, &n32, &t32, &p32, &n64, &t64, &p64);
    // persistent rounds carry two-reduction BiCGStab only: a round with a
    // CG1 solve resident makes one launch per pass
    for (Request* r : ln.slots)
      if (r && r->cg1) persist = 0;
    const int S = sv->max_slots;
    if (!rc) {
      rc = put_changed(sv, ln.stream, ln.d32, ln.h_d32,
                       sizeof(SolveDesc<float>) * std::max(n32, 1), &ln.last_d32);
      if (!rc)
        rc = put_changed(sv, ln.stream, ln.d64, ln.h_d64,
                         sizeof(SolveDesc<double>) * std::max(n64, 1), &ln.last_d64);
      if (!rc)
        rc = put_changed(sv, ln.stream, ln.bases, ln.h_bases, sizeof(int) * 4 * (S + 1),
                         &ln.last_bases);
    }
    if (!rc) {
      // two-reduction BiCGStab iterations of every resident solve: one
      // launch per pass, or the whole round in one cooperative launch per
      // precision (bitwise the same iterates)
      hipError_t e = hipSuccess;
      if (persist) {
        if (n32)
          e = launch_batch_persistent<float>(ln.d32, ln.bases, t32, n32, chunk, ln.ry, ln.bar,
                                             kRoundSpinLimit, ln.stream);
        if (e == hipSuccess && n64)
          e = launch_batch_persistent<double>(ln.d64, ln.bases + 2 * (S + 1), t64, n64, chunk,
                                              ln.ry, ln.bar, kRoundSpinLimit, ln.stream);
      } else {
        for (int q = 0; q < chunk; ++q) {
          if (n32)
            launch_batch_iteration2<float>(ln.d32, ln.bases, t32, n32, q, ln.ry, ln.stream);
          if (n64)
            launch_batch_iteration2<double>(ln.d64, ln.bases + 2 * (S + 1), t64, n64, q, ln.ry,
                                            ln.stream);
        }
        e = hipGetLastError();
      }
      // (a CG1 solve's buffers return to parity 0 after each pair of passes)
      for (Request* r : ln.slots)
        if (r && !r->cg1 && (r->phase == R_ITER || r->phase == R_REFINE)) r->par ^= (chunk & 1);
      if (e != hipSuccess) rc = fail(sv, "batched iteration", e);
    }
    if (!rc) {
      static_assert(sizeof(Scalars) % 4 == 0, "scalar blocks are copied as 32-bit words");
      // the blocks of the slots up to the last resident one (the host reads
      // only resident slots' blocks)
      int used = 1;
      for (int q = 0; q < sv->max_slots; ++q)
        if (ln.slots[q]) used = q + 1;
      const size_t words = sizeof(Scalars) * kScalarsPerSlot * (size_t)used / 4;
      const uint32_t seq = ++ln.round_seq;
      hipLaunchKernelGGL(k_readback, dim3(1), dim3(kThreads), 0, ln.stream,
                         (const uint32_t*)ln.slot_sc, ln.h_sc_dev, words, ln.flag_dev, seq);
      hipError_t e = hipGetLastError();
      if (e == hipSuccess && persist)
        e = hipMemcpyAsync(ln.h_bar, ln.bar, sizeof(GridBarrier), hipMemcpyDeviceToHost,
                           ln.stream);
      if (e == hipSuccess) e = hipEventRecord(ln.round_done, ln.stream);
      // the round's number in the flag word shows the blocks have landed,
      // a few microseconds before the event does; the event stays the
      // fallback that reports a failed round (and carries persistent
      // rounds, whose barrier block is copied after the kernel)
      bool seen = false;
      if (e == hipSuccess && !persist) {
        const auto t0 = std::chrono::steady_clock::now();
        while (!(seen = __atomic_load_n(ln.flag, __ATOMIC_ACQUIRE) == seq) &&
               std::chrono::steady_clock::now() - t0 < std::chrono::milliseconds(2)) {
        }
      }
      if (e == hipSuccess && !seen) {
        e = wait_event(ln.round_done);
        if (e == hipSuccess && !persist && __atomic_load_n(ln.flag, __ATOMIC_ACQUIRE) != seq)
          e = hipErrorUnknown;   // the round completed without its readback
      }
      if (e != hipSuccess)
        rc = fail(sv, "scalar readback", e);
      else if (persist && ln.h_bar->timeout)
        rc = fail_code(sv, WFA_ERR_HIP, "persistent round: a grid barrier wait timed out");
    }
    std::unique_lock<std::mutex> lk(sv->mu);
    if (rc) {
      // fail every request of this class; the other classes stop at their
      // next round and the server stays unusable
      fail_lane(sv, ln, rc);
      for (auto& other : sv->lanes) other.cv_work.notify_all();
      break;
    }
    for (int s = 0; s < sv->max_slots; ++s) {
      Request* r = ln.slots[s];
      if (!r || r->phase == R_START) continue;
      if ((rc = advance(sv, r))) break;
    }
    sv->cv_done.notify_all();
    if (rc) {
      fail_lane(sv, ln, rc);
      for (auto& other : sv->lanes) other.cv_work.notify_all();
      break;
    }
  }
}

// The class a request of `cells` cells goes to.
int lane_for(const wfa_server* sv, int64_t cells) {
  if (sv->persistent) return 0;
  int k = 0;
  while (k < kMaxLanes - 1 && sv->class_bound[k] > 0 && cells > sv->class_bound[k]) ++k;
  return k;
}

}  // namespace

extern "C" int wfa_server_create(void* arena, size_t arena_bytes, int max_slots, void* stream,
                                 wfa_server** out) {
  if (!out) return set_error(WFA_ERR_INVALID, "out is NULL");
  *out = nullptr;
  if (!arena || ((uintptr_t)arena & 255)) return set_error(WFA_ERR_INVALID, "arena must be non-NULL and 256-byte aligned");
  if (max_slots < 1 || max_slots > 4096) return set_error(WFA_ERR_INVALID, "max_slots must be in [1, 4096]");
  // per class: slot scalars, the two descriptor tables, tile bases, barrier
  const size_t sc_bytes = align256(sizeof(Scalars) * kScalarsPerSlot * max_slots);
  const size_t d32_bytes = align256(sizeof(SolveDesc<float>) * max_slots);
  const size_t d64_bytes = align256(sizeof(SolveDesc<double>) * max_slots);
  const size_t b_bytes = align256(sizeof(int) * 4 * (max_slots + 1));
  const size_t bar_bytes = align256(sizeof(GridBarrier));
  const size_t lane_bytes = sc_bytes + d32_bytes + d64_bytes + b_bytes + bar_bytes;
  const size_t meta = kMaxLanes * lane_bytes;
  if (arena_bytes <= meta) return set_error(WFA_ERR_NOMEM, "arena smaller than the slot tables");
  wfa_server* sv = new (std::nothrow) wfa_server();
  if (!sv) return set_error(WFA_ERR_NOMEM, "host allocation failed");
  sv->arena = (char*)arena;
  sv->arena_bytes = arena_bytes;
  sv->max_slots = max_slots;
  for (int k = 0; k < kMaxLanes - 1; ++k) sv->class_bound[k] = kDefaultClassBound[k];
  sv->heap_base = meta;
  sv->heap.init(arena_bytes - meta);
  auto teardown = [&](const char* what, hipError_t e) {
    for (auto& ln : sv->lanes) {
      if (ln.round_done) (void)hipEventDestroy(ln.round_done);
      if (ln.own_stream && ln.stream) (void)hipStreamDestroy(ln.stream);
    }
    if (sv->pinned) (void)hipHostFree(sv->pinned);
    delete sv;
    return set_error(WFA_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
  };
  hipError_t e = hipHostMalloc(&sv->pinned, meta, hipHostMallocMapped | hipHostMallocCoherent);
  if (e != hipSuccess) return teardown("server host tables", e);
  memset(sv->pinned, 0, meta);
  for (int k = 0; k < kMaxLanes; ++k) {
    wfa_server::Lane& ln = sv->lanes[k];
    ln.id = k;
    char* d = sv->arena + k * lane_bytes;
    char* h = (char*)sv->pinned + k * lane_bytes;
    ln.slot_sc = (Scalars*)d;
    ln.d32 = (SolveDesc<float>*)(d + sc_bytes);
    ln.d64 = (SolveDesc<double>*)(d + sc_bytes + d32_bytes);
    ln.bases = (int*)(d + sc_bytes + d32_bytes + d64_bytes);
    ln.bar = (GridBarrier*)(d + sc_bytes + d32_bytes + d64_bytes + b_bytes);
    ln.h_sc = (Scalars*)h;
    {
      void* hd = nullptr;
      e = hipHostGetDevicePointer(&hd, h, 0);
      if (e != hipSuccess) return teardown("server host tables", e);
      ln.h_sc_dev = (uint32_t*)hd;
    }
    ln.h_d32 = (SolveDesc<float>*)(h + sc_bytes);
    ln.h_d64 = (SolveDesc<double>*)(h + sc_bytes + d32_bytes);
    ln.h_bases = (int*)(h + sc_bytes + d32_bytes + d64_bytes);
    ln.h_bar = (GridBarrier*)(h + sc_bytes + d32_bytes + d64_bytes + b_bytes);
    // the flag word shares the barrier mirror's 256-byte piece, past it
    static_assert(sizeof(GridBarrier) + 64 + 4 <= 256, "flag word inside the barrier piece");
    ln.flag = (uint32_t*)((char*)ln.h_bar + 64);
    ln.flag_dev = (uint32_t*)((char*)ln.h_sc_dev + ((char*)ln.flag - h));
    ln.slots.assign(max_slots, nullptr);
    // the first class runs on the caller's stream, the others on streams of
    // their own (default priority)
    if (k == 0) {
      ln.stream = (hipStream_t)stream;
    } else {
      e = hipStreamCreateWithFlags(&ln.stream, hipStreamNonBlocking);
      if (e != hipSuccess) return teardown("server stream", e);
      ln.own_stream = true;
    }
    e = hipEventCreateWithFlags(&ln.round_done, hipEventDisableTiming);
    if (e != hipSuccess) return teardown("server event", e);
  }
  // the persistent rounds' barrier starts with no arrivals and no timeout
  e = hipMemsetAsync(sv->lanes[0].bar, 0, sizeof(GridBarrier), sv->lanes[0].stream);
  if (e != hipSuccess) return teardown("server barrier", e);
  int started = 0;
  try {
    for (; started < kMaxLanes; ++started)
      sv->lanes[started].worker = std::thread(worker_main, sv, started);
  } catch (...) {
    {
      std::lock_guard<std::mutex> lk(sv->mu);
      sv->stop = true;
    }
    for (int k = 0; k < started; ++k) {
      sv->lanes[k].cv_work.notify_all();
      sv->lanes[k].worker.join();
    }
    for (auto& ln : sv->lanes) {
      (void)hipEventDestroy(ln.round_done);
      if (ln.own_stream) (void)hipStreamDestroy(ln.stream);
    }
    (void)hipHostFree(sv->pinned);
    delete sv;
    return set_error(WFA_ERR_NOMEM, "could not start the server threads");
  }
  *out = sv;
  return WFA_OK;
}

extern "C" int wfa_server_set_option(wfa_server* sv, int option, int64_t value) {
  if (!sv) return set_error(WFA_ERR_INVALID, "server is NULL");
  std::lock_guard<std::mutex> lk(sv->mu);  // the worker reads them once per round
  switch (option) {
    case WFA_OPT_PERSISTENT:
      if (value != 0 && value != 1) return set_error(WFA_ERR_INVALID, "persistent must be 0 or 1");
      sv->persistent = (int)value;
      return WFA_OK;
    case WFA_OPT_METHOD:
      if (value != WFA_METHOD_BICGSTAB2 && value != WFA_METHOD_CG1)
        return set_error(WFA_ERR_INVALID, "server method must be WFA_METHOD_BICGSTAB2 or _CG1");
      sv->method = (int)value;
      return WFA_OK;
    case WFA_OPT_CG1_MAX_CELLS:
      if (value < 0) return set_error(WFA_ERR_INVALID, "cell limit must be >= 0");
      sv->cg1_max_cells = value;
      return WFA_OK;
    case WFA_OPT_CHECK_EVERY:
      if (value < 1 || value > 1024)
        return set_error(WFA_ERR_INVALID, "iterations per round must be in [1, 1024]");
      sv->chunk = (int)value;
      return WFA_OK;
    case WFA_OPT_IR_INNER_TOL:
      if (value <= 0 || value >= 1000000000000LL)
        return set_error(WFA_ERR_INVALID, "inner tolerance must be in (0, 1)");
      sv->ir_inner_tol = (double)value * 1e-12;
      return WFA_OK;
    case WFA_OPT_SIZE_CLASS_1:
    case WFA_OPT_SIZE_CLASS_2:
    case WFA_OPT_SIZE_CLASS_3: {
      if (value < 0) return set_error(WFA_ERR_INVALID, "size class bound must be >= 0");
      int64_t b[kMaxLanes - 1];
      for (int k = 0; k < kMaxLanes - 1; ++k) b[k] = sv->class_bound[k];
      b[option - WFA_OPT_SIZE_CLASS_1] = value;
      for (int k = 1; k < kMaxLanes - 1; ++k)
        if (b[k] > 0 && !(b[k - 1] > 0 && b[k] > b[k - 1]))
          return set_error(WFA_ERR_INVALID,
                           "size class bounds must increase, each after a non-zero one");
      for (int k = 0; k < kMaxLanes - 1; ++k) sv->class_bound[k] = b[k];
      return WFA_OK;
    }
    default:
      return set_error(WFA_ERR_INVALID, "option %d is not a server option", option);
  }
}

extern "C" int wfa_submit(wfa_server* sv, int nx, int ny, int nz, const wfa_coeffs* c, void* T,
                          double tol, int maxit, uint64_t* ticket) {
  if (!sv || !ticket) return set_error(WFA_ERR_INVALID, "NULL argument");
  int rc = validate_coeffs(nx, ny, nz, c);
  if (rc) return rc;
  if (!T) return set_error(WFA_ERR_INVALID, "T is NULL");
  if (!(tol > 0.0) || !isfinite(tol) || maxit < 1) return set_error(WFA_ERR_INVALID, "bad tol or maxit");
  const size_t bytes = request_bytes(nx, ny, nz, c->precision);
  if (bytes > sv->heap.size)
    return set_error(WFA_ERR_NOMEM, "request needs %zu bytes, arena holds %zu", bytes, sv->heap.size);
  Request* r = new (std::nothrow) Request();
  if (!r) return set_error(WFA_ERR_NOMEM, "host allocation failed");
  r->nx = nx; r->ny = ny; r->nz = nz;
  r->c = *c;
  r->T = T;
  r->tol = tol;
  r->maxit = maxit;
  r->bytes = bytes;
  r->t_submit = now_s();
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    if (const int err = sv->worker_error.load()) {
      delete r;
      return set_error(err, "server failed: %s", sv->worker_msg);
    }
    r->ticket = sv->next_ticket++;
    const int64_t cells = (int64_t)nx * ny * nz;
    r->cg1 = sv->method == WFA_METHOD_CG1 && c->u[0] == 0.0 && c->u[1] == 0.0 &&
             c->u[2] == 0.0 && (sv->cg1_max_cells == 0 || cells <= sv->cg1_max_cells);
    r->lane = lane_for(sv, cells);
    r->inner_tol = sv->ir_inner_tol;
    sv->reqs[r->ticket] = r;
    sv->lanes[r->lane].queue.push_back(r);
    ++sv->inflight;
  }
  sv->lanes[r->lane].cv_work.notify_one();
  *ticket = r->ticket;
  return WFA_OK;
}

extern "C" int wfa_poll(wfa_server* sv, uint64_t ticket, wfa_solve_info* info) {
  if (!sv) return set_error(WFA_ERR_INVALID, "server is NULL");
  std::lock_guard<std::mutex> lk(sv->mu);
  auto it = sv->reqs.find(ticket);
  if (it == sv->reqs.end()) return set_error(WFA_ERR_INVALID, "unknown ticket %llu", (unsigned long long)ticket);
  Request* r = it->second;
  if (r->phase != R_DONE) return WFA_PENDING;
  if (info) *info = r->info;
  if (r->code < 0 && r->code == sv->worker_error.load())
    set_error(r->code, "server failed: %s", sv->worker_msg);
  return r->code;
}

extern "C" int wfa_server_drain(wfa_server* sv) {
  if (!sv) return set_error(WFA_ERR_INVALID, "server is NULL");
  std::unique_lock<std::mutex> lk(sv->mu);
  sv->cv_done.wait(lk, [&] { return sv->inflight == 0 || sv->worker_error.load() != 0; });
  if (const int err = sv->worker_error.load())
    return set_error(err, "server failed: %s", sv->worker_msg);
  return WFA_OK;
}

extern "C" int wfa_server_destroy(wfa_server* sv) {
  if (!sv) return set_error(WFA_ERR_INVALID, "server is NULL");
  {
    std::unique_lock<std::mutex> lk(sv->mu);
    sv->cv_done.wait(lk, [&] { return sv->inflight == 0 || sv->worker_error.load() != 0; });
    sv->stop = true;
  }
  for (auto& ln : sv->lanes) ln.cv_work.notify_all();
  for (auto& ln : sv->lanes)
    if (ln.worker.joinable()) ln.worker.join();
  for (auto& kv : sv->reqs) delete kv.second;
  // teardown: nothing to report a failure to
  for (auto& ln : sv->lanes) {
    (void)hipEventDestroy(ln.round_done);
    if (ln.own_stream) {
      (void)hipStreamSynchronize(ln.stream);
      (void)hipStreamDestroy(ln.stream);
    }
  }
  (void)hipHostFree(sv->pinned);
  delete sv;
  return WFA_OK;
}
