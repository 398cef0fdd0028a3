// Explicit forward-time steps with temporal blocking: S steps of
//   T' = T - (A T - T) + boundary terms
// (the paper's explicit scheme, Eq. 2, with the operator's general faces)
// per pass over HBM.  The paper's wafer keeps the whole field in SRAM next
// to the processors, so each step costs no memory traffic at all (section
// 3.1); on a GPU a one-step pass reads and writes the field once, which
// bounds it at 2w bytes per cell-step.  Fusing S steps into one pass cuts
// that to about 2w / S plus the redundant halo reads below.
//
// A workgroup owns a column of 64 x TY cells (TY = 4 waves x RY rows; lane =
// x, so each row is one contiguous load) and marches it along z.  Step level
// s (s = 1..S) of a plane m needs level s-1 on the planes m-1, m, m+1 and on
// the x/y neighbours, so the levels run as a pipeline behind the loads: when
// level 0 (the input) of plane j arrives, level s is computed on plane
// j - s.  Each thread keeps the last three planes of every level for its
// own cells in registers (the z neighbours).  The x neighbours are the
// adjacent lanes of the same wave, read with DPP lane shifts; the y
// neighbours are the thread's own rows, except across the boundary between
// two waves, whose first and last rows of every level go through a small
// double-buffered LDS exchange (one barrier per plane).  Level s is correct on the
// column shrunk by s cells on each side, so a tile's output is the inner
// (64 - 2S) x (TY - 2S) cells; neighbouring tiles overlap by 2S cells and
// recompute the overlap.  Along z a tile covers zc output planes and reads
// S more on each side.
//
// Each level applies exactly the arithmetic of a one-step pass to the same
// values, so the result is bitwise that of S one-step passes.
#include "device.hpp"
#include "internal.hpp"

namespace wfa {

struct TbGeo {
  int nx, ny, nz;
  int tiles_x, tiles_y, zchunks, zc;
  int ntiles;
  long long plane;
};

// Value of lane - 1 (from_left) or lane + 1 (from_right) of the wave; 0 at
// the wave's ends, which hold the column's halo, outside every level's
// valid region.
__device__ __forceinline__ int dpp_left(int v) {
  return __builtin_amdgcn_update_dpp(0, v, 0x138, 0xF, 0xF, true);   // wave_shr:1
}
__device__ __forceinline__ int dpp_right(int v) {
  return __builtin_amdgcn_update_dpp(0, v, 0x130, 0xF, 0xF, true);   // wave_shl:1
}
__device__ __forceinline__ float from_left(float v) { return __int_as_float(dpp_left(__float_as_int(v))); }
__device__ __forceinline__ float from_right(float v) { return __int_as_float(dpp_right(__float_as_int(v))); }
__device__ __forceinline__ double from_left(double v) {
  return __hiloint2double(dpp_left(__double2hiint(v)), dpp_left(__double2loint(v)));
}
__device__ __forceinline__ double from_right(double v) {
  return __hiloint2double(dpp_right(__double2hiint(v)), dpp_right(__double2loint(v)));
}

template <typename T, int S, int RY>
__global__ void __launch_bounds__(kThreads)
k_explicit_tb(TbGeo g, Op<T> op, const T* __restrict__ x, T* __restrict__ y) {
  constexpr int TY = kWaves * RY;
  // input planes loaded ahead (measured: 2 is no faster, 3 slower)
  constexpr int PD = 1;
  constexpr int OW = kTX - 2 * S;
  constexpr int OH = TY - 2 * S;
  static_assert(OW > 0 && OH > 0, "tile too small for the number of fused steps");
  static_assert(RY >= 2, "a wave's first and last rows must differ");
  // [parity][level][wave][lane]: each wave's first (top) and last (bottom)
  // row of the middle plane of every level below S
  __shared__ T top[2][S][kWaves][kTX];
  __shared__ T bot[2][S][kWaves][kTX];

  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int tx = tile % g.tiles_x;
  const int rest = tile / g.tiles_x;
  const int ty = rest % g.tiles_y;
  const int tz = rest / g.tiles_y;
  const int i = tx * OW - S + lane;      // this lane's column
  const int j0 = ty * OH - S + wave * RY;  // the wave's first row (uniform)
  const int zs = tz * g.zc;
  const int ze = min(zs + g.zc, g.nz);
  const bool col_in = i >= 0 && i < g.nx;
  const bool col_out = lane >= S && lane < kTX - S && i < g.nx;
  const uint32_t ins_x = (i > 0 ? 1u : 0u) | (i < g.nx - 1 ? 2u : 0u);
  // the neighbouring waves' rows (the tile's outermost waves read a row of
  // their own instead: it lies in the halo, outside every valid region)
  const int wup = wave > 0 ? wave - 1 : wave;
  const int wdn = wave < kWaves - 1 ? wave + 1 : wave;

  // W[q][0..2]: level q on planes (newest - 2, newest - 1, newest)
  T W[S][3][RY];
#pragma unroll
  for (int q = 0; q < S; ++q)
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int r = 0; r < RY; ++r) W[q][a][r] = T(0);

  const int jb = zs - S > 0 ? zs - S : 0;
  // input planes jb .. jb + PD - 1 in flight before the first step; each
  // step consumes the oldest and issues the load of the plane PD ahead
  T pre[PD][RY];
#pragma unroll
  for (int d = 0; d < PD; ++d)
#pragma unroll
    for (int r = 0; r < RY; ++r) {
      const int j = j0 + r;
      const int kk = jb + d;
      const T* row = x + (size_t)kk * g.plane + (long long)j * g.nx;
      pre[d][r] = (col_in && j >= 0 && j < g.ny && kk < g.nz) ? row[i] : T(0);
    }

  const T kz[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};  // constant diffusivity
  const InteriorCoef<T> kin = interior_coef(op);
  int par = 0;
  for (int k = jb; k < ze + S; ++k, par ^= 1) {
    // opaque copies: the face masks below are recomputed every step instead
    // of being hoisted out of the loop as per-row coefficient registers
    int jr = j0;
    uint32_t ix = ins_x;
    asm volatile("" : "+s"(jr));
    asm volatile("" : "+v"(ix));
#pragma unroll
    for (int q = 0; q < S; ++q)
#pragma unroll
      for (int r = 0; r < RY; ++r) {
        W[q][0][r] = W[q][1][r];
        W[q][1][r] = W[q][2][r];
      }
#pragma unroll
    for (int r = 0; r < RY; ++r) W[0][2][r] = k < g.nz ? pre[0][r] : T(0);
#pragma unroll
    for (int d = 0; d + 1 < PD; ++d)
#pragma unroll
      for (int r = 0; r < RY; ++r) pre[d][r] = pre[d + 1][r];
    if (k + PD < g.nz) {
#pragma unroll
      for (int r = 0; r < RY; ++r) {
        const int j = j0 + r;
        const T* row = x + (size_t)(k + PD) * g.plane + (long long)j * g.nx;
        pre[PD - 1][r] = (col_in && j >= 0 && j < g.ny) ? row[i] : T(0);
      }
    }
    // every level's middle plane: the wave's boundary rows into LDS (the
    // buffer of this parity was last read two steps ago, before the
    // previous step's barrier)
#pragma unroll
    for (int q = 0; q < S; ++q) {
      top[par][q][wave][lane] = W[q][1][0];
      bot[par][q][wave][lane] = W[q][1][RY - 1];
    }
    __syncthreads();
#pragma unroll
    for (int s = 1; s <= S; ++s) {
      const int m = k - s;  // plane of level s computed in this step
      const bool plane_ok = m >= 0 && m < g.nz;
      const uint32_t ins_z = (m > 0 ? 16u : 0u) | (m < g.nz - 1 ? 32u : 0u);
      const T above = bot[par][s - 1][wup][lane];  // row j0 - 1
      const T below = top[par][s - 1][wdn][lane];  // row j0 + RY
#pragma unroll
      for (int r = 0; r < RY; ++r) {
        const int j = jr + r;
        const T c = W[s - 1][1][r];
        const T nb[6] = {from_left(c), from_right(c),
                         r > 0 ? W[s - 1][1][r - 1] : above,
                         r < RY - 1 ? W[s - 1][1][r + 1] : below,
                         W[s - 1][0][r], W[s - 1][2][r]};
        const uint32_t ins = ix | (j > 0 ? 4u : 0u) | (j < g.ny - 1 ? 8u : 0u) | ins_z;
        T v;
        if (__all(ins == 63u)) {  // the whole wave is interior: no face tests
          v = explicit_update(c, cell_apply_interior(kin, c, nb), T(0));
        } else {
          T dg;
          const T Au = cell_apply<T, false>(op, c, nb, T(0), kz, ins, dg);
          v = explicit_update(c, Au, cell_bterm<T, false>(op, T(0), ins));
        }
        if (s < S) {
          W[s][2][r] = plane_ok ? v : T(0);
        } else {
          const int lr = wave * RY + r;
          if (plane_ok && m >= zs && lr >= S && lr < TY - S && j < g.ny && col_out) {
            T* row = y + (size_t)m * g.plane + (long long)j * g.nx;
            __builtin_nontemporal_store(v, row + i);
          }
        }
      }
    }
  }
}

template <typename T, int S, int RY>
static void launch_tb(const Launch<T>& L, const T* x, T* y, int zc_override) {
  constexpr int TY = kWaves * RY;
  const Geo& G = L.tl.geo;
  TbGeo g{};
  g.nx = G.nx; g.ny = G.ny; g.nz = G.nz;
  g.plane = (long long)G.nx * G.ny;
  g.tiles_x = (G.nx + (kTX - 2 * S) - 1) / (kTX - 2 * S);
  g.tiles_y = (G.ny + (TY - 2 * S) - 1) / (TY - 2 * S);
  const long long txy = (long long)g.tiles_x * g.tiles_y;
  int zc = zc_override > 0 ? zc_override : 128;
  // >= 4096 workgroups (16 per CU: the register-heavy columns need many in
  // flight), without letting the 2S redundant z planes per tile exceed a
  // quarter of its planes; measured on 512x512x1024
  if (zc_override <= 0)
    while (zc > 8 * S && txy * ((G.nz + zc - 1) / zc) < 4096) zc /= 2;
  if (zc > G.nz) zc = G.nz;
  g.zc = zc;
  g.zchunks = (G.nz + zc - 1) / zc;
  g.ntiles = (int)(txy * g.zchunks);
  hipLaunchKernelGGL((k_explicit_tb<T, S, RY>), dim3(g.ntiles), dim3(kThreads), 0, L.stream, g,
                     L.op, x, y);
}

template <typename T>
void launch_explicit_fused(const Launch<T>& L, const T* x, T* y, int steps, int zc_override) {
  // FP32 columns of 32 rows, FP64 of 16 (registers hold 3 planes per level)
  constexpr int RY = sizeof(T) == 4 ? 8 : 4;
  switch (steps) {
    case 2: launch_tb<T, 2, RY>(L, x, y, zc_override); break;
    case 3: launch_tb<T, 3, RY>(L, x, y, zc_override); break;
    default: launch_tb<T, 4, RY>(L, x, y, zc_override); break;
  }
}

template void launch_explicit_fused<float>(const Launch<float>&, const float*, float*, int, int);
template void launch_explicit_fused<double>(const Launch<double>&, const double*, double*, int,
                                            int);

}  // namespace wfa
