// C ABI of libhard (declared in include/hard.h): argument checks, workspace
// layout and kernel dispatch.  Nothing here computes the method; every step
// of it runs in the kernels of stage.hip, reduce.hip, batched.hip and
// adjoint.hip.

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>

#include "../../include/hard.h"
#include "api_internal.hpp"
#include "hydro_device.hpp"
#include "launch.hpp"

namespace hard {

static thread_local std::string g_last_error;

hard_status_t fail(hard_status_t code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

hard_status_t ok() {
  g_last_error.clear();
  return HARD_OK;
}

hard_status_t hip_fail(hipError_t e, const char* what) {
  return fail(HARD_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

hard_status_t check_grid(const hard_grid_t* g, Grid* out) {
  if (!g) return fail(HARD_ERR_INVALID_ARG, "grid is NULL");
  if (g->ndim < 1 || g->ndim > 3) return fail(HARD_ERR_INVALID_ARG, "ndim must be 1, 2 or 3 (got %d)", g->ndim);
  if (g->dtype != HARD_F64 && g->dtype != HARD_F32)
    return fail(HARD_ERR_INVALID_ARG, "dtype must be HARD_F64 or HARD_F32 (got %d)", g->dtype);
  long long ncell = 1;
  for (int d = 0; d < 3; ++d) {
    if (d < g->ndim) {
      if (g->n[d] < 2 || g->n[d] >= (1LL << 31))
        return fail(HARD_ERR_INVALID_ARG, "n[%d] = %lld must be in [2, 2^31)", d, (long long)g->n[d]);
      if (!(std::isfinite(g->dx[d]) && g->dx[d] > 0.0))
        return fail(HARD_ERR_INVALID_ARG, "dx[%d] must be finite and > 0", d);
      for (int s = 0; s < 2; ++s)
        if (g->bc[d][s] < HARD_BC_PERIODIC || g->bc[d][s] > HARD_BC_REFLECT)
          return fail(HARD_ERR_INVALID_ARG, "bc[%d][%d] = %d is not a boundary kind", d, s, g->bc[d][s]);
      if ((g->bc[d][0] == HARD_BC_PERIODIC) != (g->bc[d][1] == HARD_BC_PERIODIC))
        return fail(HARD_ERR_INVALID_ARG, "axis %d: periodic must be set on both sides", d);
    } else if (g->n[d] != 1) {
      return fail(HARD_ERR_INVALID_ARG, "n[%d] must be 1 for ndim = %d", d, g->ndim);
    }
    ncell *= g->n[d];
  }
  if (ncell >= (1LL << 31)) return fail(HARD_ERR_INVALID_ARG, "more than 2^31 - 1 cells");
  if (!(std::isfinite(g->gamma) && g->gamma > 1.0))
    return fail(HARD_ERR_INVALID_ARG, "gamma must be finite and > 1");
  if (g->scheme != HARD_SCHEME_MUSCL_HLLC && g->scheme != HARD_SCHEME_WENO5Z_HLL)
    return fail(HARD_ERR_INVALID_ARG, "scheme must be HARD_SCHEME_MUSCL_HLLC or HARD_SCHEME_WENO5Z_HLL");
  if (g->scheme == HARD_SCHEME_WENO5Z_HLL)
    for (int d = 0; d < g->ndim; ++d)
      if (g->n[d] < 3) return fail(HARD_ERR_INVALID_ARG, "WENO5-Z needs n[%d] >= 3", d);
  if (g->rad != 0 && g->rad != 1) return fail(HARD_ERR_INVALID_ARG, "rad must be 0 or 1");
  if (g->rad) {
    if (!(std::isfinite(g->kappa) && g->kappa >= 0.0))
      return fail(HARD_ERR_INVALID_ARG, "kappa must be finite and >= 0");
    if (!(std::isfinite(g->mu) && g->mu > 0.0))
      return fail(HARD_ERR_INVALID_ARG, "mu must be finite and > 0");
    if (g->scheme != HARD_SCHEME_MUSCL_HLLC)
      return fail(HARD_ERR_UNSUPPORTED, "radiation is built for HARD_SCHEME_MUSCL_HLLC");
  }
  if (out) {
    out->ndim = g->ndim;
    out->dtype = g->dtype;
    out->nvar = g->ndim + 2 + (g->rad ? 1 : 0);
    out->rad = g->rad;
    out->kappa = g->rad ? g->kappa : 0.0;
    out->mu = g->rad ? g->mu : 1.0;
    out->wsize = g->dtype == HARD_F64 ? 8 : 4;
    out->ncell = ncell;
    for (int d = 0; d < 3; ++d) {
      out->n[d] = (int)g->n[d];
      out->dx[d] = d < g->ndim ? g->dx[d] : 1.0;
      out->inv_dx[d] = 1.0 / out->dx[d];
      out->bc[d][0] = d < g->ndim ? g->bc[d][0] : HARD_BC_PERIODIC;
      out->bc[d][1] = d < g->ndim ? g->bc[d][1] : HARD_BC_PERIODIC;
    }
    out->gamma = g->gamma;
    out->scheme = g->scheme;
    out->dx_pow2 = 1;
    for (int d = 0; d < g->ndim; ++d) {
      int e;
      if (std::frexp(g->dx[d], &e) != 0.5) out->dx_pow2 = 0;
    }
  }
  return HARD_OK;
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

WorkLayout layout_of(const Grid& g) {
  WorkLayout w;
  w.ctl = 0;
  w.stage = 256;
  w.stage_bytes = align256((size_t)g.nvar * g.ncell * g.wsize);
  w.partials = w.stage + w.stage_bytes;
  w.partials_blocks = sums_blocks(g.ncell);
  w.slots = w.partials + align256((size_t)w.partials_blocks * g.nvar * 2 * sizeof(double));
  long long ns = stage_launch_blocks(g.ndim, g.dtype, g.n);
  if (ns < GRID_STRIDE_MAX_BLOCKS) ns = GRID_STRIDE_MAX_BLOCKS;
  w.nslots = (int)ns;
  w.total = w.slots + align256((size_t)ns * sizeof(double));
  w.weno_w = 0;
  w.weno_f[0] = w.weno_f[1] = w.weno_f[2] = 0;
  if (g.scheme == HARD_SCHEME_WENO5Z_HLL) {
    w.weno_w = w.total;
    w.total += align256((size_t)g.nvar * g.ncell * g.wsize);
    // face arrays of every axis but the last (x in 1D too); the faces of
    // the last axis of a 2D or 3D grid never leave registers
    for (int d = 0; d < (g.ndim == 1 ? 1 : g.ndim - 1); ++d) {
      w.weno_f[d] = w.total;
      w.total += align256((size_t)g.nvar * (g.ncell / g.n[d]) * (g.n[d] + 1) * g.wsize);
    }
  }
  return w;
}

hard_status_t check_ptr(const void* p, size_t align, const char* name) {
  if (!p) return fail(HARD_ERR_INVALID_ARG, "%s is NULL", name);
  if (((uintptr_t)p) % align) return fail(HARD_ERR_INVALID_ARG, "%s is not %zu-byte aligned", name, align);
  return HARD_OK;
}

hard_status_t check_work(void* work, size_t have, size_t need) {
  if (!work) return fail(HARD_ERR_INVALID_ARG, "work is NULL");
  if (((uintptr_t)work) % 256) return fail(HARD_ERR_INVALID_ARG, "work is not 256-byte aligned");
  if (have < need) return fail(HARD_ERR_WORKSPACE, "workspace has %zu bytes, needs %zu", have, need);
  return HARD_OK;
}

// One stage of the grid's scheme: the fused tile kernel (MUSCL-HLLC) or the
// WENO5-Z + HLL pipeline over the workspace arrays of layout L.
hipError_t launch_scheme_stage(const Grid& G, const WorkLayout& L, char* wb, const StageArgs& a,
                               int stage, hipStream_t s) {
  if (G.scheme == HARD_SCHEME_MUSCL_HLLC) return launch_stage(G.ndim, G.dtype, a, stage, s);
  WenoArgs w;
  std::memset(&w, 0, sizeof w);
  w.src = a.src;
  w.un = a.un;
  w.dst = a.dst;
  w.dt = a.dt;
  for (int d = 0; d < 3; ++d) {
    w.n[d] = a.n[d];
    w.bc[d][0] = a.bc[d][0];
    w.bc[d][1] = a.bc[d][1];
    w.dx[d] = a.dx[d];
    w.inv_dx[d] = a.inv_dx[d];
    w.F[d] = L.weno_f[d] ? wb + L.weno_f[d] : nullptr;
  }
  w.dx_pow2 = a.dx_pow2;
  w.gamma = a.gamma;
  w.cfl = a.cfl;
  w.fuse_cfl = a.fuse_cfl;
  w.ctl = a.ctl;
  w.next_dt = a.next_dt;
  w.slots = a.slots;
  w.nslots = a.nslots;
  w.W = wb + L.weno_w;
  return launch_weno_stage(G.ndim, G.dtype, w, stage, s);
}

int stage_cz_override() {
  static int v = [] {
    const char* e = std::getenv("HARD_STAGE_CZ");
    int x = e ? std::atoi(e) : 0;
    return x > 0 ? x : 0;
  }();
  return v;
}

hard_status_t check_cfl(double cfl) {
  if (!(std::isfinite(cfl) && cfl > 0.0 && cfl <= 1.0))
    return fail(HARD_ERR_INVALID_ARG, "cfl must be in (0, 1]");
  return HARD_OK;
}

}  // namespace hard

using namespace hard;

extern "C" {

const char* hard_last_error(void) { return g_last_error.c_str(); }

hard_status_t hard_workspace_bytes(const hard_grid_t* g, size_t* bytes) {
  Grid G;
  hard_status_t st = check_grid(g, &G);
  if (st) return st;
  if (!bytes) return fail(HARD_ERR_INVALID_ARG, "bytes is NULL");
  *bytes = layout_of(G).total;
  return ok();
}

hard_status_t hard_workspace_init(void* work, size_t work_bytes, void* stream) {
  hard_status_t st = check_work(work, work_bytes, sizeof(Control));
  if (st) return st;
  hipError_t e = launch_control_clear(static_cast<Control*>(work), (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "hard_workspace_init");
  return ok();
}

hard_status_t hard_cfl_dt(const hard_grid_t* g, const void* U, double cfl, double* dt_dev,
                          double* dt_host, void* work, size_t work_bytes, void* stream) {
  Grid G;
  hard_status_t st = check_grid(g, &G);
  if (st) return st;
  if ((st = check_ptr(U, G.wsize, "U"))) return st;
  if ((st = check_ptr(dt_dev, 8, "dt_dev"))) return st;
  if ((st = check_cfl(cfl))) return st;
  WorkLayout L = layout_of(G);
  if ((st = check_work(work, work_bytes, L.total))) return st;
  hipStream_t s = (hipStream_t)stream;
  Control* ctl = reinterpret_cast<Control*>(static_cast<char*>(work) + L.ctl);
  hipError_t e = launch_cfl(G.ndim, G.dtype, G.n, G.dx, G.inv_dx, G.dx_pow2, G.gamma, U, cfl, dt_dev,
                            ctl, reinterpret_cast<double*>(static_cast<char*>(work) + L.slots),
                            L.nslots, s);
  if (e != hipSuccess) return hip_fail(e, "hard_cfl_dt launch");
  if (dt_host) {
    unsigned flags = 0;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "hard_cfl_dt sync");
    if ((e = hipMemcpy(dt_host, dt_dev, sizeof(double), hipMemcpyDeviceToHost)) != hipSuccess)
      return hip_fail(e, "hard_cfl_dt copy");
    if ((e = hipMemcpy(&flags, &ctl->flags, sizeof flags, hipMemcpyDeviceToHost)) != hipSuccess)
      return hip_fail(e, "hard_cfl_dt flags");
    if (flags) return fail(HARD_ERR_NONPHYSICAL, "non-physical state (flags 0x%x)", flags);
  }
  return ok();
}

hard_status_t hard_hydro_step(const hard_grid_t* g, void* U, const double* dt_dev, double cfl,
                              double* next_dt_dev, void* work, size_t work_bytes, void* stream) {
  Grid G;
  hard_status_t st = check_grid(g, &G);
  if (st) return st;
  if ((st = check_ptr(U, G.wsize, "U"))) return st;
  if ((st = check_ptr(dt_dev, 8, "dt_dev"))) return st;
  if (next_dt_dev) {
    if ((st = check_ptr(next_dt_dev, 8, "next_dt_dev"))) return st;
    if ((st = check_cfl(cfl))) return st;
  }
  WorkLayout L = layout_of(G);
  if ((st = check_work(work, work_bytes, L.total))) return st;
  hipStream_t s = (hipStream_t)stream;
  char* wb = static_cast<char*>(work);
  StageArgs a;
  std::memset(&a, 0, sizeof a);
  for (int d = 0; d < 3; ++d) {
    a.n[d] = G.n[d];
    a.dx[d] = G.dx[d];
    a.inv_dx[d] = G.inv_dx[d];
    a.dx_pow2 = G.dx_pow2;
    a.bc[d][0] = G.bc[d][0];
    a.bc[d][1] = G.bc[d][1];
  }
  a.gamma = G.gamma;
  a.cfl = cfl;
  a.dt = dt_dev;
  a.ctl = reinterpret_cast<Control*>(wb + L.ctl);
  a.slots = reinterpret_cast<double*>(wb + L.slots);
  a.nslots = L.nslots;
  a.cz = stage_cz_override();
  a.rad = G.rad;  // E_r is advected by the same stage kernels
  a.kappa = G.kappa;
  a.mu = G.mu;
  void* U1 = wb + L.stage;
  // stage 1: U1 = U + dt L(U)
  a.src = U;
  a.un = U;
  a.dst = U1;
  a.fuse_cfl = 0;
  hipError_t e = launch_scheme_stage(G, L, wb, a, 1, s);
  if (e != hipSuccess) return hip_fail(e, "hard_hydro_step stage 1");
  // stage 2: U = (U + (U1 + dt L(U1))) / 2, with radiation followed cell by
  // cell by the heating/cooling exchange, optionally with the next dt (of
  // the state after the exchange)
  a.src = U1;
  a.un = U;
  a.dst = U;
  a.fuse_cfl = next_dt_dev != nullptr;
  a.exchange = G.rad;
  a.next_dt = next_dt_dev;
  e = launch_scheme_stage(G, L, wb, a, 2, s);
  if (e != hipSuccess) return hip_fail(e, "hard_hydro_step stage 2");
  return ok();
}

hard_status_t hard_hydro_stage(const hard_grid_t* g, int32_t stage, const void* src,
                               const void* un, void* dst, const double* dt_dev, double cfl,
                               double* next_dt_dev, void* work, size_t work_bytes, void* stream) {
  Grid G;
  hard_status_t st = check_grid(g, &G);
  if (st) return st;
  if (stage != 1 && stage != 2) return fail(HARD_ERR_INVALID_ARG, "stage must be 1 or 2");
  if (G.rad)
    return fail(HARD_ERR_UNSUPPORTED, "with radiation the step is not a pair of stages; use hard_hydro_step");
  if ((st = check_ptr(src, G.wsize, "src"))) return st;
  if ((st = check_ptr(dst, G.wsize, "dst"))) return st;
  if (stage == 2 && (st = check_ptr(un, G.wsize, "un"))) return st;
  if (src == dst) return fail(HARD_ERR_INVALID_ARG, "dst must not alias src");
  if ((st = check_ptr(dt_dev, 8, "dt_dev"))) return st;
  if (stage == 2 && next_dt_dev) {
    if ((st = check_ptr(next_dt_dev, 8, "next_dt_dev"))) return st;
    if ((st = check_cfl(cfl))) return st;
  }
  WorkLayout L = layout_of(G);
  const bool fused = stage == 2 && next_dt_dev;
  const size_t need = G.scheme == HARD_SCHEME_MUSCL_HLLC && !fused ? sizeof(Control) : L.total;
  if ((st = check_work(work, work_bytes, need))) return st;
  StageArgs a;
  std::memset(&a, 0, sizeof a);
  for (int d = 0; d < 3; ++d) {
    a.n[d] = G.n[d];
    a.dx[d] = G.dx[d];
    a.inv_dx[d] = G.inv_dx[d];
    a.dx_pow2 = G.dx_pow2;
    a.bc[d][0] = G.bc[d][0];
    a.bc[d][1] = G.bc[d][1];
  }
  a.gamma = G.gamma;
  a.cfl = cfl;
  a.dt = dt_dev;
  a.ctl = static_cast<Control*>(work);
  a.slots = fused ? reinterpret_cast<double*>(static_cast<char*>(work) + L.slots) : nullptr;
  a.nslots = fused ? L.nslots : 0;
  a.cz = stage_cz_override();
  a.src = src;
  a.un = stage == 2 ? un : src;
  a.dst = dst;
  a.fuse_cfl = stage == 2 && next_dt_dev != nullptr;
  a.next_dt = next_dt_dev;
  hipError_t e = launch_scheme_stage(G, L, static_cast<char*>(work), a, stage, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "hard_hydro_stage");
  return ok();
}

hard_status_t hard_run(const hard_grid_t* g, void* U, double cfl, double t_end,
                       int64_t max_steps, double* t_out, int64_t* steps_out, void* work,
                       size_t work_bytes, void* stream) {
  Grid G;
  hard_status_t st = check_grid(g, &G);
  if (st) return st;
  if ((st = check_ptr(U, G.wsize, "U"))) return st;
  if ((st = check_cfl(cfl))) return st;
  if (!(std::isfinite(t_end) && t_end > 0.0)) return fail(HARD_ERR_INVALID_ARG, "t_end must be finite and > 0");
  if (max_steps < 1) return fail(HARD_ERR_INVALID_ARG, "max_steps must be >= 1");
  if (!t_out || !steps_out) return fail(HARD_ERR_INVALID_ARG, "t_out and steps_out must not be NULL");
  WorkLayout L = layout_of(G);
  if ((st = check_work(work, work_bytes, L.total))) return st;
  hipStream_t s = (hipStream_t)stream;
  Control* ctl = reinterpret_cast<Control*>(static_cast<char*>(work) + L.ctl);
  hipError_t e = launch_control_clear(ctl, s);
  if (e != hipSuccess) return hip_fail(e, "hard_run clear");
  double* dt = &ctl->dt;
  if ((e = launch_cfl(G.ndim, G.dtype, G.n, G.dx, G.inv_dx, G.dx_pow2, G.gamma, U, cfl, dt,
                      ctl, reinterpret_cast<double*>(static_cast<char*>(work) + L.slots), L.nslots,
                      s)) != hipSuccess)
    return hip_fail(e, "hard_run cfl");
  int done = 0;
  if (G.ndim == 1 && G.n[0] <= RUN1D_MAX && G.scheme == HARD_SCHEME_MUSCL_HLLC && !G.rad) {
    // small 1D grids: the whole loop in one resident workgroup, 1024 steps
    // per launch
    Run1dArgs r;
    std::memset(&r, 0, sizeof r);
    r.U = U;
    r.n = G.n[0];
    r.bc[0] = G.bc[0][0];
    r.bc[1] = G.bc[0][1];
    r.dx = G.dx[0];
    r.inv_dx = G.inv_dx[0];
    r.dx_pow2 = G.dx_pow2;
    r.gamma = G.gamma;
    r.cfl = cfl;
    r.t_end = t_end;
    r.max_steps = max_steps;
    r.chunk = 1024;
    r.ctl = ctl;
    while (!done) {
      if ((e = launch_run1d(G.dtype, r, s)) != hipSuccess) return hip_fail(e, "hard_run 1D loop");
      if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "hard_run sync");
      if ((e = hipMemcpy(&done, &ctl->done, sizeof done, hipMemcpyDeviceToHost)) != hipSuccess)
        return hip_fail(e, "hard_run read");
    }
  }
  const int batch = 64;
  while (!done) {
    for (int i = 0; i < batch; ++i) {
      if ((e = launch_time_control(ctl, t_end, max_steps, s)) != hipSuccess)
        return hip_fail(e, "hard_run time control");
      if ((st = hard_hydro_step(g, U, dt, cfl, dt, work, work_bytes, stream))) return st;
    }
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "hard_run sync");
    if ((e = hipMemcpy(&done, &ctl->done, sizeof done, hipMemcpyDeviceToHost)) != hipSuccess)
      return hip_fail(e, "hard_run read");
  }
  long long steps = 0;
  unsigned flags = 0;
  if ((e = hipMemcpy(t_out, &ctl->t, sizeof(double), hipMemcpyDeviceToHost)) != hipSuccess ||
      (e = hipMemcpy(&steps, &ctl->steps, sizeof steps, hipMemcpyDeviceToHost)) != hipSuccess ||
      (e = hipMemcpy(&flags, &ctl->flags, sizeof flags, hipMemcpyDeviceToHost)) != hipSuccess)
    return hip_fail(e, "hard_run read");
  *steps_out = steps;
  if (flags) return fail(HARD_ERR_NONPHYSICAL, "non-physical state (flags 0x%x)", flags);
  return ok();
}

hard_status_t hard_run_rhd(const hard_grid_t* g, void* U, double cfl, double t_end,
                           int64_t max_steps, const hard_gmg_opts_t* opts, double* t_out,
                           int64_t* steps_out, void* work, size_t work_bytes, void* fld_work,
                           size_t fld_work_bytes, void* stream) {
  Grid G;
  hard_status_t st = check_grid(g, &G);
  if (st) return st;
  if (!G.rad) return fail(HARD_ERR_INVALID_ARG, "hard_run_rhd needs rad = 1");
  if ((st = check_ptr(U, G.wsize, "U"))) return st;
  if ((st = check_cfl(cfl))) return st;
  if (!(std::isfinite(t_end) && t_end > 0.0)) return fail(HARD_ERR_INVALID_ARG, "t_end must be finite and > 0");
  if (max_steps < 1) return fail(HARD_ERR_INVALID_ARG, "max_steps must be >= 1");
  if (!t_out || !steps_out) return fail(HARD_ERR_INVALID_ARG, "t_out and steps_out must not be NULL");
  WorkLayout L = layout_of(G);
  if ((st = check_work(work, work_bytes, L.total))) return st;
  size_t fld_need = 0;
  if ((st = hard_rad_diffuse_workspace_bytes(g, &fld_need))) return st;
  if ((st = check_work(fld_work, fld_work_bytes, fld_need))) return st;
  if (!opts) return fail(HARD_ERR_INVALID_ARG, "opts is NULL");
  hipStream_t s = (hipStream_t)stream;
  Control* ctl = reinterpret_cast<Control*>(static_cast<char*>(work) + L.ctl);
  // the diffusion reads the step size from its own control block's dt slot
  Control* fctl = static_cast<Control*>(fld_work);
  double* dt = &ctl->dt;
  double* dt_step = &fctl->dt;
  hipError_t e = launch_control_clear(ctl, s);
  if (e != hipSuccess) return hip_fail(e, "hard_run_rhd clear");
  if ((e = launch_cfl(G.ndim, G.dtype, G.n, G.dx, G.inv_dx, G.dx_pow2, G.gamma, U, cfl, dt,
                      ctl, reinterpret_cast<double*>(static_cast<char*>(work) + L.slots), L.nslots,
                      s)) != hipSuccess)
    return hip_fail(e, "hard_run_rhd cfl");
  const int batch = 64;
  int done = 0;
  while (!done) {
    for (int i = 0; i < batch; ++i) {
      if ((e = launch_time_control(ctl, t_end, max_steps, s)) != hipSuccess ||
          (e = launch_fld_copy_dt(dt, dt_step, s)) != hipSuccess)
        return hip_fail(e, "hard_run_rhd time control");
      if ((st = hard_hydro_step(g, U, dt, cfl, dt, work, work_bytes, stream))) return st;
      if ((st = hard_rad_diffuse(g, U, dt_step, opts, nullptr, fld_work, fld_work_bytes, stream)))
        return st;
    }
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "hard_run_rhd sync");
    if ((e = hipMemcpy(&done, &ctl->done, sizeof done, hipMemcpyDeviceToHost)) != hipSuccess)
      return hip_fail(e, "hard_run_rhd read");
  }
  long long steps = 0;
  unsigned flags = 0, fflags = 0;
  if ((e = hipMemcpy(t_out, &ctl->t, sizeof(double), hipMemcpyDeviceToHost)) != hipSuccess ||
      (e = hipMemcpy(&steps, &ctl->steps, sizeof steps, hipMemcpyDeviceToHost)) != hipSuccess ||
      (e = hipMemcpy(&flags, &ctl->flags, sizeof flags, hipMemcpyDeviceToHost)) != hipSuccess ||
      (e = hipMemcpy(&fflags, &fctl->flags, sizeof fflags, hipMemcpyDeviceToHost)) != hipSuccess)
    return hip_fail(e, "hard_run_rhd read");
  *steps_out = steps;
  if (flags | fflags)
    return fail(HARD_ERR_NONPHYSICAL, "non-physical state (flags 0x%x)", flags | fflags);
  return ok();
}

hard_status_t hard_status_read(void* work, size_t work_bytes, uint32_t* flags, void* stream) {
  hard_status_t st = check_work(work, work_bytes, sizeof(Control));
  if (st) return st;
  if (!flags) return fail(HARD_ERR_INVALID_ARG, "flags is NULL");
  hipStream_t s = (hipStream_t)stream;
  Control* ctl = static_cast<Control*>(work);
  hipError_t e;
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "hard_status_read sync");
  unsigned f = 0;
  if ((e = hipMemcpy(&f, &ctl->flags, sizeof f, hipMemcpyDeviceToHost)) != hipSuccess)
    return hip_fail(e, "hard_status_read copy");
  unsigned zero = 0;
  if ((e = hipMemcpy(&ctl->flags, &zero, sizeof zero, hipMemcpyHostToDevice)) != hipSuccess)
    return hip_fail(e, "hard_status_read clear");
  *flags = f;
  if (f) return fail(HARD_ERR_NONPHYSICAL, "non-physical state (flags 0x%x)", f);
  return ok();
}

hard_status_t hard_conservation_sums(const hard_grid_t* g, const void* U, double* sums_dev,
                                     void* work, size_t work_bytes, void* stream) {
  Grid G;
  hard_status_t st = check_grid(g, &G);
  if (st) return st;
  if ((st = check_ptr(U, G.wsize, "U"))) return st;
  if ((st = check_ptr(sums_dev, 8, "sums_dev"))) return st;
  WorkLayout L = layout_of(G);
  if ((st = check_work(work, work_bytes, L.total))) return st;
  double* partials = reinterpret_cast<double*>(static_cast<char*>(work) + L.partials);
  hipError_t e = launch_sums(G.nvar, G.dtype, G.n, U, partials, L.partials_blocks, sums_dev,
                             (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "hard_conservation_sums");
  return ok();
}

}  // extern "C"
