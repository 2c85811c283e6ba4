// Host-side helpers shared by the C-ABI translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/hard.h"

namespace hard {

// Validated grid with derived quantities (unused axes: n = 1, dx = 1).
struct Grid {
  int ndim, dtype, nvar, wsize;
  long long ncell;
  int n[3];
  double dx[3], inv_dx[3];
  int bc[3][2];
  double gamma;
  int dx_pow2;  // every dx is a power of two (x/dx == x*(1/dx) exactly)
  int scheme;   // HARD_SCHEME_*
  int rad;      // 1: field ndim + 2 is the radiation energy density
  double kappa, mu;
};

// Byte offsets inside a single-grid workspace.
struct WorkLayout {
  size_t ctl;            // Control block (256 B)
  size_t stage;          // intermediate stage state U^1
  size_t stage_bytes;
  size_t partials;       // compensated-sum partials
  int partials_blocks;
  size_t slots;          // CFL reductions: one signal-sum max per workgroup
  int nslots;
  size_t weno_w;         // WENO5-Z pipeline: primitives (0 if unused)
  size_t weno_f[3];      // WENO5-Z pipeline: face fluxes per axis
  size_t total;
};

hard_status_t fail(hard_status_t code, const char* fmt, ...);
hard_status_t ok();
hard_status_t hip_fail(hipError_t e, const char* what);
hard_status_t check_grid(const hard_grid_t* g, Grid* out);
hard_status_t check_ptr(const void* p, size_t align, const char* name);
hard_status_t check_work(void* work, size_t have, size_t need);
hard_status_t check_cfl(double cfl);
WorkLayout layout_of(const Grid& g);
struct StageArgs;
hipError_t launch_scheme_stage(const Grid& G, const WorkLayout& L, char* wb, const StageArgs& a,
                               int stage, hipStream_t s);

// *to = *from on the stream (fld.hip).
hipError_t launch_fld_copy_dt(const double* from, double* to, hipStream_t s);

// z planes per workgroup for the 3D stage kernel: HARD_STAGE_CZ in the
// environment overrides the default (read once; 0 = default).
int stage_cz_override();

}  // namespace hard
