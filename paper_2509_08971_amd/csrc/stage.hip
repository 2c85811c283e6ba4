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
  t.gamma = a.gamma;
  t.dt = *a.dt;
  t.x0 = tile_x * TX;
  t.y0 = tile_y * TY;
  t.z0 = NDIM == 3 ? chunk * a.cz : 0;
  t.z1 = NDIM == 3 ? min(t.z0 + a.cz, a.n[2]) : 1;
  t.fuse_cfl = STAGE == 2 && a.fuse_cfl;
  unsigned flags = 0;
  double smax = 0.0;
  run_tile<NDIM, R, STAGE, TX, TY, NTHR>(t, lds, flags, smax);
  block_finish<NTHR>(flags, smax, STAGE == 2 && a.fuse_cfl, a.ctl, a.cfl, a.next_dt);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <int NDIM, typename R, int TX, int TY, int NTHR = TX * TY>
static hipError_t launch_stage_t(const StageArgs& a0, int stage, hipStream_t s) {
  StageArgs a = a0;
  a.tiles_x = (int)((a.n[0] + TX - 1) / TX);
  a.tiles_y = NDIM >= 2 ? (int)((a.n[1] + TY - 1) / TY) : 1;
  int nchunk = 1;
  if (NDIM == 3) {
    if (a.cz <= 0) a.cz = 32;
    nchunk = (int)((a.n[2] + a.cz - 1) / a.cz);
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

// tile shapes (x by y) of the 3D kernels
#ifndef HARD_TILE64
#define HARD_TILE64 16, 16
#endif
#ifndef HARD_TILE32
#define HARD_TILE32 32, 8
#endif

hipError_t launch_stage(int ndim, int dtype, const StageArgs& a, int stage, hipStream_t s) {
  if (dtype == 0) {
    switch (ndim) {
      case 1: return launch_stage_t<1, double, 255, 1, 256>(a, stage, s);
      case 2: return launch_stage_t<2, double, 16, 16>(a, stage, s);
      case 3: return launch_stage_t<3, double, HARD_TILE64>(a, stage, s);
    }
  } else {
    switch (ndim) {
      case 1: return launch_stage_t<1, float, 255, 1, 256>(a, stage, s);
      case 2: return launch_stage_t<2, float, 32, 8>(a, stage, s);
      case 3: return launch_stage_t<3, float, HARD_TILE32>(a, stage, s);
    }
  }
  return hipErrorInvalidValue;
}

}  // namespace hard
