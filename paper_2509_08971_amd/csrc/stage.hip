// Single-grid Heun-stage kernel: one workgroup per (x-y tile, z chunk), the
// tile body in stage_tile.hpp.  HBM traffic per stage is one read of the
// stencil source and one write of the result (plus one read of U^n in stage
// 2); halo re-reads hit the L2 of the XCD that owns the neighbouring tiles.
//
// Stage 2 optionally folds the CFL signal-speed max of the new state into
// the same pass (wave64 shuffle max -> LDS -> one slot per workgroup); a
// one-workgroup kernel after it turns the slots into dt.

#include "api_internal.hpp"
#include "hydro_device.hpp"
#include "launch.hpp"
#include "stage_tile.hpp"

namespace hard {

// Minimum waves per SIMD the register allocator must allow: 3 for the FP64
// 3D hydro kernels (their natural footprint sits just above the 168-VGPR
// limit of 3 waves), no constraint otherwise (the FP64 3D kernels carrying
// E_r hold 2 waves per SIMD by their LDS anyway).
#ifndef HARD_STAGE_WAVES
#define HARD_STAGE_WAVES(NDIM, R, RAD) ((NDIM) == 3 && sizeof(R) == 8 && !(RAD) ? 3 : 1)
#endif

template <int NDIM, typename R, int STAGE, int TX, int TY, int NTHR, bool RAD>
__global__ __launch_bounds__(NTHR) __attribute__((amdgpu_waves_per_eu(HARD_STAGE_WAVES(NDIM, R, RAD), 8)))
void stage_kernel(StageArgs a) {
  __shared__ R lds[TileShape<NDIM, R, TX, TY, RAD>::lds_elems];
  int L = xcd_tile(blockIdx.x, gridDim.x);
  const int tile_x = L % a.tiles_x;
  L /= a.tiles_x;
  const int tile_y = L % a.tiles_y;
  const int chunk = L / a.tiles_y;
  TileArgs t;
  t.src = a.src;
  t.un = a.un;
  t.dst = a.dst;
  for (int d = 0; d < 3; ++d) {
    t.n[d] = a.n[d];
    t.bc[d][0] = a.bc[d][0];
    t.bc[d][1] = a.bc[d][1];
    t.dx[d] = a.dx[d];
    t.inv_dx[d] = a.inv_dx[d];
  }
  t.dx_pow2 = a.dx_pow2;
  t.gamma = a.gamma;
  t.dt = *a.dt;
  t.x0 = tile_x * TX;
  t.y0 = tile_y * TY;
  constexpr bool WALK = TileShape<NDIM, R, TX, TY, RAD>::WALK;
  const int nwalk = NDIM == 3 ? a.n[2] : (NDIM == 2 ? a.n[1] : 1);
  t.w0 = WALK ? chunk * a.cz : 0;
  t.w1 = WALK ? min(t.w0 + a.cz, nwalk) : 1;
  t.fuse_cfl = STAGE == 2 && a.fuse_cfl;
  t.exchange = STAGE == 2 && RAD && a.exchange;
  t.kappa = a.kappa;
  t.mu = a.mu;
  unsigned flags = 0;
  double smax = 0.0;
  run_tile<NDIM, R, STAGE, TX, TY, NTHR, NDIM == 3, RAD>(t, lds, flags, smax);
  block_finish<NTHR>(flags, smax, STAGE == 2 && a.fuse_cfl, a.ctl, a.slots + blockIdx.x);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
// Launch shape of a stage: workgroups (tiles x walk chunks) and the chunk
// length.  TX x TY cells per tile (3D), or a row of TX cells (1D, 2D); cz_in
// walk positions per chunk (0 = cz_default).
template <int NDIM, int TX, int TY>
static long long stage_shape(const int* n, int cz_in, int cz_default, int& tiles_x, int& tiles_y,
                             int& cz) {
  constexpr bool walk = NDIM == 3 || (NDIM == 2 && TY == 1);
  tiles_x = (n[0] + TX - 1) / TX;
  tiles_y = (NDIM == 3 || TY > 1) ? (n[1] + TY - 1) / TY : 1;
  long long nchunk = 1;
  cz = 1;
  if (walk) {
    const int nwalk = NDIM == 3 ? n[2] : n[1];
    cz = cz_in > 0 ? cz_in : cz_default;
    nchunk = (nwalk + cz - 1) / cz;
  }
  return (long long)tiles_x * tiles_y * nchunk;
}

// NTHR threads per workgroup; stage 2 with a fused CFL step ends with the
// one-workgroup reduction of the slots.
template <int NDIM, typename R, int TX, int TY, int NTHR>
static hipError_t launch_stage_t(const StageArgs& a0, int stage, int cz_default, hipStream_t s) {
  StageArgs a = a0;
  const long long nb = stage_shape<NDIM, TX, TY>(a.n, a.cz, cz_default, a.tiles_x, a.tiles_y, a.cz);
  const bool fuse = stage == 2 && a.fuse_cfl;
  if (nb >= (1LL << 31) || (fuse && nb > a.nslots)) return hipErrorInvalidValue;
  dim3 grid((unsigned)nb), block(NTHR);
  if (a.rad) {
    if (stage == 1)
      hipLaunchKernelGGL((stage_kernel<NDIM, R, 1, TX, TY, NTHR, true>), grid, block, 0, s, a);
    else
      hipLaunchKernelGGL((stage_kernel<NDIM, R, 2, TX, TY, NTHR, true>), grid, block, 0, s, a);
  } else if (stage == 1) {
    hipLaunchKernelGGL((stage_kernel<NDIM, R, 1, TX, TY, NTHR, false>), grid, block, 0, s, a);
  } else {
    hipLaunchKernelGGL((stage_kernel<NDIM, R, 2, TX, TY, NTHR, false>), grid, block, 0, s, a);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !fuse) return e;
  return launch_cfl_final(a.slots, (int)nb, a.cfl, a.next_dt, s);
}

// tile shapes (x by y) of the 3D kernels.  32 x 8 also for FP64: its x halo
// (two cells at each end of a row, 16 bytes of a 128-byte line) spans 8 rows
// instead of 16, which the L1's data path, busy about 80% of stage 2, feels
#ifndef HARD_TILE64
#define HARD_TILE64 32, 8
#endif
#ifndef HARD_TILE32
#define HARD_TILE32 32, 8
#endif
// z planes per workgroup of the 3D kernels
#ifndef HARD_STAGE_CZ_3D
#define HARD_STAGE_CZ_3D 32
#endif
constexpr int STAGE_CZ_3D = HARD_STAGE_CZ_3D;

// z planes per workgroup of a 3D grid: STAGE_CZ_3D, halved while the launch
// would have fewer than about 1500 workgroups, down to 4 (each chunk loads
// four planes beyond its own).  Per step on periodic boxes (FP64, us), cz =
// 32 / 16 / 8 / 4: 64^3 198 / 107 / 62 / 39; 128^3 228 / 179 / 177 / 179;
// 192^3 563 / 508 / 521 / 539; 256^3 1045 / 1060 / 1078 / 1144.
template <int TX, int TY>
static int chunk_3d(const int* n) {
  const long long tiles = (long long)((n[0] + TX - 1) / TX) * ((n[1] + TY - 1) / TY);
  const long long want = tiles * n[2] / 1536;
  int cz = STAGE_CZ_3D;
  while (cz > 4 && cz > want) cz >>= 1;
  return cz;
}

// 2D grids: rows of 255, 127 or 63 cells (one face per thread per row) and
// enough walk chunks to give the machine a few thousand workgroups.
static int chunk_2d(int nx, int ny, int tx) {
  long long tiles = (nx + tx - 1) / tx;
  long long want = 4096;
  long long c = (tiles * ny + want - 1) / want;
  return (int)(c < 4 ? 4 : (c > 64 ? 64 : c));
}

// 2D grids of at most PLANE_2D_MAX cells: 32 x 8 tiles that do not walk
// (one workgroup per tile, four waves, every face of the tile from LDS).  The
// walk cuts such a grid into a few hundred workgroups of one or two waves,
// each stepping through a handful of rows.
#ifndef HARD_PLANE_2D_MAX
#define HARD_PLANE_2D_MAX (1 << 20)
#endif
constexpr long long PLANE_2D_MAX = HARD_PLANE_2D_MAX;

template <typename R>
static hipError_t launch_stage_2d(const StageArgs& a, int stage, hipStream_t s) {
  const int nx = a.n[0], ny = a.n[1];
  if ((long long)nx * ny <= PLANE_2D_MAX) return launch_stage_t<2, R, 32, 8, 256>(a, stage, 1, s);
  if (nx >= 1024) return launch_stage_t<2, R, 255, 1, 256>(a, stage, chunk_2d(nx, ny, 255), s);
  if (nx >= 256) return launch_stage_t<2, R, 127, 1, 128>(a, stage, chunk_2d(nx, ny, 127), s);
  return launch_stage_t<2, R, 63, 1, 64>(a, stage, chunk_2d(nx, ny, 63), s);
}

long long stage_launch_blocks(int ndim, int dtype, const int* n) {
  const int cz = stage_cz_override();
  int tx, ty, c;
  switch (ndim) {
    case 1: return stage_shape<1, 255, 1>(n, cz, 1, tx, ty, c);
    case 2:
      if ((long long)n[0] * n[1] <= PLANE_2D_MAX) return stage_shape<2, 32, 8>(n, cz, 1, tx, ty, c);
      if (n[0] >= 1024) return stage_shape<2, 255, 1>(n, cz, chunk_2d(n[0], n[1], 255), tx, ty, c);
      if (n[0] >= 256) return stage_shape<2, 127, 1>(n, cz, chunk_2d(n[0], n[1], 127), tx, ty, c);
      return stage_shape<2, 63, 1>(n, cz, chunk_2d(n[0], n[1], 63), tx, ty, c);
    default:
      return dtype == 0 ? stage_shape<3, HARD_TILE64>(n, cz, chunk_3d<HARD_TILE64>(n), tx, ty, c)
                        : stage_shape<3, HARD_TILE32>(n, cz, chunk_3d<HARD_TILE32>(n), tx, ty, c);
  }
}

hipError_t launch_stage(int ndim, int dtype, const StageArgs& a, int stage, hipStream_t s) {
  if (dtype == 0) {
    switch (ndim) {
      case 1: return launch_stage_t<1, double, 255, 1, 256>(a, stage, 1, s);
      case 2: return launch_stage_2d<double>(a, stage, s);
      case 3: return launch_stage_t<3, double, HARD_TILE64, 256>(a, stage, chunk_3d<HARD_TILE64>(a.n), s);
    }
  } else {
    switch (ndim) {
      case 1: return launch_stage_t<1, float, 255, 1, 256>(a, stage, 1, s);
      case 2: return launch_stage_2d<float>(a, stage, s);
      case 3: return launch_stage_t<3, float, HARD_TILE32, 256>(a, stage, chunk_3d<HARD_TILE32>(a.n), s);
    }
  }
  return hipErrorInvalidValue;
}

}  // namespace hard
