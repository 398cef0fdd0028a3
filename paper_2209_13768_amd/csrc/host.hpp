// Host-side descriptor of a grid and helpers shared by the solver driver and
// the server.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <vector>

#include "wfa.h"
#include "internal.hpp"

namespace wfa {

constexpr int kVecs = 9;  // r, rh, t, p0, p1, v0, v1, b, r1 (b unused by the IR inner
                          // solve; r1 = second residual buffer of BiCGStab2)

// Byte offsets of the workspace sub-buffers (each 256-byte aligned).
struct Layout {
  size_t scalars;           // 4 Scalars blocks: solve, inner solve, aux, spare
  size_t partials;          // 3 x partial_slots doubles
  size_t vec[kVecs];        // Krylov vectors (FP64 or FP32; FP32 for IR)
  size_t b64, d32;          // IR only: FP64 right-hand side, FP32 correction
  size_t total;
};

Layout layout_for(int nx, int ny, int nz, int precision);
size_t partial_slots(int nx, int ny, int nz);

struct Profiler {
  struct Pending {
    int kernel;
    hipEvent_t e0, e1;
  };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> pool;
  int64_t launches[WFA_K_COUNT] = {};  // timed launches
  double total_ms[WFA_K_COUNT] = {};
  int64_t seen[WFA_K_COUNT] = {};      // launches since profiling was set (sampling)
  hipEvent_t get();
  void drain();
  void clear();
};

// Executable graphs of fixed launch sequences (a chunk of iterations),
// keyed by everything the captured launches depend on.
struct GraphCache {
  static constexpr int kKey = 16;
  static constexpr size_t kMaxEntries = 32;
  struct Entry {
    uint64_t key[kKey];
    hipGraphExec_t exec;
  };
  hipStream_t cap = nullptr;  // private stream the sequences are captured on
  std::vector<Entry> entries;
  uint64_t generation = 1;    // bumped whenever tiling or operator options change
  void clear();
};

// Pinned host copies of device scalar blocks: the host reads a solve's
// scalars with asynchronous copies into this block and one event, which it
// polls (a wait of a few tens of microseconds is common on small grids, and
// polling answers sooner than a blocking wait).
struct Readback {
  static constexpr int kSlots = 2;
  Scalars* host = nullptr;   // kSlots blocks (hipHostMalloc), or `local` in sync mode
  hipEvent_t done = nullptr;
  // sync mode: the copies land in `local` (pageable host memory) and the
  // stream is synchronised; no pinned block or event is ever created
  bool sync = false;
  Scalars local[kSlots];
  int init();                // 0 or a WFA_ERR_* code
  void clear();
};

// Waits for `e` (polling first); clears the thread's last-error state.
hipError_t wait_event(hipEvent_t e);

int set_error(int code, const char* fmt, ...);
int ir_inner_maxit(int maxit, int used);
// The inner FP32 solve of iterative refinement stops as diverged once its
// residual norm has grown 1000-fold (squared: 1e6).
constexpr double kIrGuard = 1e6;
int validate_coeffs(int nx, int ny, int nz, const wfa_coeffs* c);

}  // namespace wfa

struct wfa_grid {
  int nx, ny, nz;
  size_t n;
  wfa_coeffs c;
  int prec;
  char* ws;
  wfa::Layout lay;
  wfa::Scalars* sc;      // the solve
  wfa::Scalars* sc_in;   // inner solve of iterative refinement
  wfa::Scalars* sc_aux;  // true residual
  double* partials;
  void* vec[wfa::kVecs];
  double* b64;
  float* d32;
  wfa::Op<double> op64;
  wfa::Op<float> op32;
  wfa::Tiling tl;        // tiling of the grid's vector type
  wfa::Tiling tl32;      // tiling of FP32 inner vectors
  int method, persistent, profile, force_bd, check_every, zchunk, ry, jacobi, graph, fuse;
  int shadow;  // two-reduction BiCGStab: 0 r^ = r0 (stored), 1 index-hashed r^
  int recompute_t;  // two-reduction BiCGStab: pass 1 forms t = A s again (not stored)
  double ir_inner_tol;
  int force_div;         // n > 0: the next IR solve's first inner solve diverges at n
  int hint_iters;        // iterations of the last converged (inner) solve: first chunk size
  wfa::Profiler prof;
  wfa::GraphCache graphs;
  wfa::Readback rb;
};

namespace wfa {
void grid_setup(wfa_grid* g, int nx, int ny, int nz, const wfa_coeffs* c, char* ws);
void apply_tiling(wfa_grid* g, int ry, int zc);
// Tile shape the tuning table holds for this grid key, if any.
bool tuned_tiling(int nx, int ny, int nz, int precision, int mode, int* ry, int* zc);
int solve_any(wfa_grid* g, const void* b, void* x, bool form_b, double tol, int maxit,
              wfa_solve_info* info, hipStream_t s);
}  // namespace wfa
