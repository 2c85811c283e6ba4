// Single-grid Heun-stage kernel: one workgroup per (x-y tile, z chunk), the
// tile body in stage_tile.hpp.  HBM traffic per stage is one read of the
// stencil source and one write of the result (plus one read of U^n in stage
// 2); halo re-reads hit the L2 of the XCD that owns the neighbouring tiles.
//
// Stage 2 optionally folds the CFL signal-speed max of the new state into
// the same pass (wave64 shuffle max -> LDS -> one atomicMax per workgroup;
// the last workgroup turns the max into dt and re-arms the slot).

#include "hydro_device.hpp"
#include "launch.hpp"
#include "stage_tile.hpp"

namespace hard {

// Minimum waves per SIMD the register allocator must allow: 3 for the FP64
// 3D kernels (their natural footprint sits just above the 168-VGPR limit of
// 3 waves), no constraint otherwise.
#ifndef HARD_STAGE_WAVES
#define HARD_STAGE_WAVES(NDIM, R) ((NDIM) == 3 && sizeof(R) == 8 ? 3 : 1)
#endif

template <int NDIM, typename R, int STAGE, int TX, int TY, int NTHR>
__global__ __launch_bounds__(NTHR) __attribute__((amdgpu_waves_per_eu(HARD_STAGE_WAVES(NDIM, R), 8)))
void stage_kernel(StageArgs a) {
  __shared__ R lds[TileShape<NDIM, R, TX, TY>::lds_elems];
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
  const int nwalk = NDIM == 3 ? a.n[2] : (NDIM == 2 ? a.n[1] : 1);
  t.w0 = NDIM >= 2 ? chunk * a.cz : 0;
  t.w1 = NDIM >= 2 ? min(t.w0 + a.cz, nwalk) : 1;
  t.fuse_cfl = STAGE == 2 && a.fuse_cfl;
  unsigned flags = 0;
  double smax = 0.0;
  run_tile<NDIM, R, STAGE, TX, TY, NTHR, NDIM == 3>(t, lds, flags, smax);
  block_finish<NTHR>(flags, smax, STAGE == 2 && a.fuse_cfl, a.ctl, a.cfl, a.next_dt);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
// TX x TY cells per tile (3D), or a row of TX cells (1D, 2D); NTHR threads;
// a.cz positions per walk chunk (0 = default).
template <int NDIM, typename R, int TX, int TY, int NTHR>
static hipError_t launch_stage_t(const StageArgs& a0, int stage, int cz_default, hipStream_t s) {
  StageArgs a = a0;
  a.tiles_x = (int)((a.n[0] + TX - 1) / TX);
  a.tiles_y = NDIM == 3 ? (int)((a.n[1] + TY - 1) / TY) : 1;
  int nchunk = 1;
  if (NDIM >= 2) {
    const int nwalk = NDIM == 3 ? a.n[2] : a.n[1];
    if (a.cz <= 0) a.cz = cz_default;
    nchunk = (nwalk + a.cz - 1) / a.cz;
  } else {
    a.cz = 1;
  }
  dim3 grid((unsigned)(a.tiles_x * a.tiles_y * nchunk)), block(NTHR);
  if (stage == 1)
    hipLaunchKernelGGL((stage_kernel<NDIM, R, 1, TX, TY, NTHR>), grid, block, 0, s, a);
  else
    hipLaunchKernelGGL((stage_kernel<NDIM, R, 2, TX, TY, NTHR>), grid, block, 0, s, a);
  return hipGetLastError();
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

// 2D grids: rows of 255, 127 or 63 cells (one face per thread per row) and
// enough walk chunks to give the machine a few thousand workgroups.
template <typename R>
static hipError_t launch_stage_2d(const StageArgs& a, int stage, hipStream_t s) {
  const int nx = a.n[0], ny = a.n[1];
  auto chunk_for = [&](int tx) {
    long long tiles = (nx + tx - 1) / tx;
    long long want = 4096;
    long long c = (tiles * ny + want - 1) / want;
    return (int)(c < 4 ? 4 : (c > 64 ? 64 : c));
  };
  if (nx >= 1024) return launch_stage_t<2, R, 255, 1, 256>(a, stage, chunk_for(255), s);
  if (nx >= 256) return launch_stage_t<2, R, 127, 1, 128>(a, stage, chunk_for(127), s);
  return launch_stage_t<2, R, 63, 1, 64>(a, stage, chunk_for(63), s);
}

hipError_t launch_stage(int ndim, int dtype, const StageArgs& a, int stage, hipStream_t s) {
  if (dtype == 0) {
    switch (ndim) {
      case 1: return launch_stage_t<1, double, 255, 1, 256>(a, stage, 1, s);
      case 2: return launch_stage_2d<double>(a, stage, s);
      case 3: return launch_stage_t<3, double, HARD_TILE64, 256>(a, stage, 32, s);
    }
  } else {
    switch (ndim) {
      case 1: return launch_stage_t<1, float, 255, 1, 256>(a, stage, 1, s);
      case 2: return launch_stage_2d<float>(a, stage, s);
      case 3: return launch_stage_t<3, float, HARD_TILE32, 256>(a, stage, 32, s);
    }
  }
  return hipErrorInvalidValue;
}

}  // namespace hard
