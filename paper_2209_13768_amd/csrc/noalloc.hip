// wfa_bicgstab_solve_static: the BiCGStab solve of wfa_bicgstab_solve for
// callers that cannot allocate (code under HIP graph capture, tight serving
// loops, harnesses that forbid allocation).  The grid's workspace (Krylov
// vectors, per-tile partial sums, scalar blocks) is carved out of one
// file-scope device array instead of a caller buffer, the grid descriptor
// lives on the stack for the duration of the call, and the scalars are read
// back with plain copies and a stream synchronisation instead of a pinned
// block and an event.  Nothing is allocated: no hipMalloc, hipFree,
// hipHostMalloc, event or stream creation.
#include <hip/hip_runtime.h>
#include <math.h>

#include <mutex>

#include "host.hpp"
#include "wfa.h"

namespace {

// The scratch array.  Each GPU the library runs on holds its own copy until
// the process ends.  In host code `scratch` names a host-side stand-in, not
// device memory: kernels and copies are only ever given the device address
// that hipGetSymbolAddress returns for the current device.
constexpr size_t kScratchBytes = (size_t)WFA_STATIC_WORKSPACE_BYTES;
__device__ __align__(256) char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_dev_scratch[kMaxDevices] = {};

// Device address of the scratch array on the current device, looked up once
// per device (with that device current).
int scratch_of_current_device(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return wfa::set_error(WFA_ERR_HIP, "hipGetDevice: %s", hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices)
    return wfa::set_error(WFA_ERR_HIP, "device %d beyond the %d the library tracks", dev,
                          kMaxDevices);
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_dev_scratch[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return wfa::set_error(WFA_ERR_HIP, "scratch address: %s", hipGetErrorString(e));
    if (((uintptr_t)p & 255) != 0)
      return wfa::set_error(WFA_ERR_HIP, "scratch array not 256-byte aligned");
    g_dev_scratch[dev] = p;
  }
  *out = g_dev_scratch[dev];
  return WFA_OK;
}

}  // namespace

extern "C" int wfa_bicgstab_solve_static(int nx, int ny, int nz, const wfa_coeffs* c,
                                         const void* b, void* x, double tol, int maxit,
                                         wfa_solve_info* info, void* stream) {
  int rc = wfa::validate_coeffs(nx, ny, nz, c);
  if (rc) return rc;
  if (!x) return wfa::set_error(WFA_ERR_INVALID, "x is NULL");
  if (!b) return wfa::set_error(WFA_ERR_INVALID, "b is NULL");
  if (!(tol > 0.0) || !isfinite(tol)) return wfa::set_error(WFA_ERR_INVALID, "tol must be > 0");
  if (maxit < 1) return wfa::set_error(WFA_ERR_INVALID, "maxit must be >= 1");
  const size_t need = wfa_workspace_bytes(nx, ny, nz, c->precision);
  if (need > kScratchBytes)
    return wfa::set_error(WFA_ERR_NOMEM,
                          "grid needs %zu workspace bytes; the static workspace holds %zu",
                          need, kScratchBytes);
  void* ws = nullptr;
  if ((rc = scratch_of_current_device(&ws))) return rc;
  // The descriptor wfa_grid_create would make over that workspace, with the
  // same tiling rule (and tuned tiling), so the solve is bitwise that of
  // wfa_bicgstab_solve on such a grid.
  wfa_grid g{};
  wfa::grid_setup(&g, nx, ny, nz, c, (char*)ws);
  int ry = 0, zc = 0;
  if (wfa::tuned_tiling(nx, ny, nz, c->precision, c->mode, &ry, &zc)) wfa::apply_tiling(&g, ry, zc);
  g.rb.sync = true;
  g.method = WFA_METHOD_BICGSTAB;
  rc = wfa::solve_any(&g, b, x, false, tol, maxit, info, (hipStream_t)stream);
  g.rb.clear();
  return rc;
}
