// Host-side launch interface between the C ABI (api.hip) and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hard {

struct Control;

struct StageArgs {
  const void* src;       // stencil source: U^n (stage 1) or U^1 (stage 2)
  const void* un;        // U^n for the stage-2 combine
  void* dst;             // U^1 (stage 1) or U^{n+1} (stage 2; may alias un)
  const double* dt;      // device dt
  int n[3];              // cells per axis (1 for unused axes)
  int bc[3][2];          // boundary kinds
  double dx[3];          // cell widths (CFL)
  double inv_dx[3];      // 1/dx (flux difference)
  int dx_pow2;           // every dx is a power of two
  double gamma;
  double cfl;
  int fuse_cfl;          // stage 2: fold the CFL max of U^{n+1} into the pass
  int tiles_x, tiles_y;  // filled by the launcher
  int cz;                // walk positions per workgroup (z in 3D, y in 2D), 0 = default
  int rad;               // 1: field ndim + 2 is E_r, advected in the same pass
  int exchange;          // stage 2 with rad: the heating/cooling exchange of each
                         // new cell state before it is stored (and before its CFL)
  double kappa, mu;      // opacity and mean molecular weight (exchange)
  Control* ctl;          // workspace control block
  double* next_dt;       // fused CFL output (stage 2)
  double* slots;         // fused CFL: one signal-sum max per workgroup
  int nslots;            // room in slots (checked against the launch size)
};

hipError_t launch_stage(int ndim, int dtype, const StageArgs& a, int stage, hipStream_t s);

// Workgroups of the stage-2 launch of launch_stage for this grid (the CFL
// slots it needs).
long long stage_launch_blocks(int ndim, int dtype, const int* n);

// dt = cfl / max(slots[0 .. n)) by one workgroup (the second half of every
// fused or standalone CFL reduction).
hipError_t launch_cfl_final(const double* slots, int n, double cfl, double* dt, hipStream_t s);

// Upper bound on the workgroups of the grid-stride kernels that end in a
// CFL reduction (standalone CFL, WENO5-Z update, radiation exchange).
constexpr int GRID_STRIDE_MAX_BLOCKS = 4096;

// WENO5-Z + HLL stage (weno.hip): same stage semantics as StageArgs, with the
// workspace arrays of the pipeline.
struct WenoArgs {
  const void* src;
  const void* un;
  void* dst;
  const double* dt;
  int n[3];
  int bc[3][2];
  double dx[3];
  double inv_dx[3];
  int dx_pow2;
  double gamma;
  double cfl;
  int fuse_cfl;
  Control* ctl;
  double* next_dt;
  double* slots;
  int nslots;
  void* W;      // primitives of the stage source, [nvar][N]
  void* F[3];   // face fluxes per axis, [nvar][faces along that axis]
};

hipError_t launch_weno_stage(int ndim, int dtype, const WenoArgs& a, int stage, hipStream_t s);

// The time loop of hard_run for 1D grids of at most RUN1D_MAX cells in one
// workgroup (run1d.hip): up to `chunk` steps per launch; t, steps, the next
// dt, done and the status bits carried in the control block.
constexpr int RUN1D_THREADS = 1024;
constexpr int RUN1D_MAX = 2 * RUN1D_THREADS;
struct Run1dArgs {
  void* U;
  int n;
  int bc[2];
  double dx, inv_dx;
  int dx_pow2;
  double gamma, cfl, t_end;
  long long max_steps;
  int chunk;
  Control* ctl;
};
hipError_t launch_run1d(int dtype, const Run1dArgs& a, hipStream_t s);

// Standalone CFL dt (reads U once).
hipError_t launch_cfl(int ndim, int dtype, const int* n, const double* dx, const double* inv_dx,
                      int dx_pow2, double gamma, const void* U, double cfl, double* dt,
                      Control* ctl, double* slots, int nslots, hipStream_t s);

// hard_run time control (one thread).
hipError_t launch_time_control(Control* ctl, double t_end, long long max_steps, hipStream_t s);

// Zero the control block.
hipError_t launch_control_clear(Control* ctl, hipStream_t s);

// Compensated per-field sums: partials has room for nblocks_max * nvar * 2 doubles.
hipError_t launch_sums(int nvar, int dtype, const int* n, const void* U, double* partials,
                       int nblocks_max, double* out, hipStream_t s);
int sums_blocks(long long ncell);

}  // namespace hard
