/*
 * libhard: explicit finite-volume hydro step on one AMD MI355X (gfx950).
 *
 * The operation (HARD paper, section 2.2.1 "Basic equations", section 2.2.2
 * "Numerical algorithms"): the hydro rows of the conservation law
 * d_t U + d_j F^j = 0 with U = (rho, rho v_d, e + rho v^2/2) and the fluxes of
 * the paper's equation "fluxes", closed by the ideal-gas law p = (gamma-1) e;
 * face fluxes F*_{i+-1/2} of the paper's finite-volume difference formula are
 * HLLC fluxes of MUSCL-minmod face states; time advance is Heun's method
 * (the paper's Butcher tableau) in Shu-Osher form; the time step comes from
 * the CFL condition (section 3.5).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - State arrays are device pointers (HIP global memory), contiguous,
 *    structure-of-arrays, field-major with x fastest:
 *        U[nvar][n2][n1][n0],  nvar = ndim + 2,
 *    fields (rho, m_x[, m_y[, m_z]], E) with E the total energy density.
 *    Element type is double (HARD_F64) or float (HARD_F32); the pointer must
 *    be aligned to the element size.
 *  - The domain is [0, n_d dx_d] per axis, cell-centred.  Each axis has two
 *    ghost layers per side generated inside the kernels from the boundary
 *    kind (periodic wrap, outflow copy of the edge cell, reflecting mirror
 *    with the normal momentum negated).
 *  - `stream` is a hipStream_t (NULL = the default stream).  All device work
 *    is enqueued on it; calls return once it is enqueued unless stated.
 *  - The caller owns every buffer.  The library keeps no pointer after a call
 *    returns, never allocates device memory on the step path, and does no
 *    host synchronisation except where stated.  Buffers must stay alive until
 *    the enqueued work has completed.
 *  - `work` is a caller-provided device workspace of at least the size the
 *    matching *_workspace_bytes query returns, 256-byte aligned.  It holds
 *    the intermediate stage state, reduction slots and the status word.  It
 *    must be cleared once with hard_workspace_init (or allocated zeroed)
 *    before first use; the kernels leave its control block ready for the
 *    next call.  Calls that share one workspace must be stream-ordered.
 *  - Argument errors are detected on the host before anything is enqueued
 *    and return HARD_ERR_INVALID_ARG / HARD_ERR_WORKSPACE /
 *    HARD_ERR_UNSUPPORTED; hard_last_error() then describes the problem.
 *    Non-physical states (rho <= 0, p <= 0, non-finite values) do not stop
 *    the kernels: they set bits in the workspace status word, reported as
 *    HARD_ERR_NONPHYSICAL by the calls that read it back.
 */
#ifndef HARD_H
#define HARD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t hard_status_t;

#define HARD_OK 0
#define HARD_ERR_INVALID_ARG 1
#define HARD_ERR_UNSUPPORTED 2
#define HARD_ERR_WORKSPACE 3
#define HARD_ERR_NONPHYSICAL 4
#define HARD_ERR_HIP 5

/* Boundary kinds. */
#define HARD_BC_PERIODIC 0
#define HARD_BC_OUTFLOW 1
#define HARD_BC_REFLECT 2

/* Element types.  HARD_F32 stores and computes reconstruction and fluxes in
 * float; the internal-energy recovery E - |m|^2/(2 rho), the time step and
 * the conservation sums are computed in double. */
#define HARD_F64 0
#define HARD_F32 1

/* Face schemes.  HARD_SCHEME_MUSCL_HLLC: MUSCL-minmod face states of the
 * primitive variables with the HLLC flux (two ghost layers), in the fused
 * tile kernels.  HARD_SCHEME_WENO5Z_HLL: the paper's own choice (section
 * 2.2.2), WENO5-Z face states of the primitive variables (Borges et al.
 * 2008) with the HLL flux (three ghost layers), as a pipeline of per-axis
 * face kernels; single-grid calls only (the batched and adjoint calls return
 * HARD_ERR_UNSUPPORTED for it). */
#define HARD_SCHEME_MUSCL_HLLC 0
#define HARD_SCHEME_WENO5Z_HLL 1

/* Radiation (rad = 1; section 2.2.1, the fourth row of the conservation law
 * and its heating source).  The state has nvar = ndim + 3 fields, E_r last.
 * Each Heun stage advects E_r with the fluid velocity through the local
 * Lax-Friedrichs (Rusanov) flux of its MUSCL-minmod face states (section
 * 2.2.2), with the signal speed max(|u_L| + c_L, |u_R| + c_R) of the hydro
 * face states; E_r does not act on the hydro fields.  Stage 2 then lets every
 * new cell state exchange energy between the fluid and the radiation by the heating
 * rate qdot = c kappa rho (E_r - a T^4) (equation "heating-cooling"), T =
 * (gamma - 1) e mu m_u / (rho k_B), integrated by backward Euler (Newton on
 * the new temperature; e + E_r is conserved); the fused next dt is that of
 * the state after the exchange.  CGS units for the constants (c, a, k_B,
 * m_u).  Single-grid calls with HARD_SCHEME_MUSCL_HLLC only:
 * hard_hydro_stage, the batched and the adjoint calls return
 * HARD_ERR_UNSUPPORTED for rad = 1. */

/* Status-word bits (hard_status_read). */
#define HARD_FLAG_DENSITY 1u   /* rho <= 0 or NaN in some cell */
#define HARD_FLAG_PRESSURE 2u  /* p <= 0 or NaN in some cell */
#define HARD_FLAG_NONFINITE 4u /* some conserved value is not finite */
#define HARD_FLAG_RADIATION 8u /* radiation diffusion: E_r <= 0 or NaN, or a
                                  diffusion coefficient that is not finite */

typedef struct hard_grid_t {
  int32_t ndim;     /* 1, 2 or 3 */
  int32_t dtype;    /* HARD_F64 or HARD_F32 */
  int64_t n[3];     /* cells per axis, 2 <= n < 2^31; axes >= ndim must be 1 */
  double dx[3];     /* cell width per axis, finite and > 0 */
  double gamma;     /* ratio of specific heats, > 1 */
  int32_t bc[3][2]; /* boundary kind per axis, [axis][0 = low, 1 = high];
                       periodic must be set on both sides of an axis */
  int32_t scheme;   /* face scheme: HARD_SCHEME_MUSCL_HLLC (0, the default of a
                       zero-initialised struct) or HARD_SCHEME_WENO5Z_HLL (1,
                       needs n >= 3 on every axis) */
  int32_t rad;      /* 1: the state carries the radiation energy density E_r
                       as field ndim + 2 (see "Radiation" below); 0: hydro only */
  double kappa;     /* rad = 1: mean opacity (cm^2/g), finite and >= 0 */
  double mu;        /* rad = 1: mean molecular weight, finite and > 0 */
} hard_grid_t;

/* Description of the last error on the calling thread ("" if none).  The
 * string is owned by the library and valid until the next call. */
const char* hard_last_error(void);

/* Bytes of workspace the single-grid calls (cfl_dt, hydro_step,
 * conservation_sums, status_read) need for grid g. */
hard_status_t hard_workspace_bytes(const hard_grid_t* g, size_t* bytes);

/* Clear the workspace control block (enqueued; no memset node is used, so
 * the call may be captured in a graph). */
hard_status_t hard_workspace_init(void* work, size_t work_bytes, void* stream);

/* CFL time step (section 3.5; the formula is this library's reading):
 *     dt = cfl / max_i sum_d (|u_{d,i}| + c_i) / dx_d
 * over the interior cells of U, c = sqrt(gamma p / rho), evaluated in double
 * with refined reciprocals of rho and of the square root (within a few ulp
 * of a plain IEEE evaluation).  Writes dt to the device double *dt_dev.  If dt_host is not NULL the call synchronises the
 * stream, copies dt to *dt_host and returns HARD_ERR_NONPHYSICAL if the
 * status word has any bit set.  0 < cfl <= 1. */
hard_status_t hard_cfl_dt(const hard_grid_t* g, const void* U, double cfl, double* dt_dev,
                          double* dt_host, void* work, size_t work_bytes, void* stream);

/* One Heun (SSP-RK2) step of size *dt_dev (section 2.2.2, Butcher tableau):
 *     U1 = U + dt L(U),   U_new = (U + (U1 + dt L(U1))) / 2,
 *     L(U)_i = - sum_d (F_{d,i+1/2} - F_{d,i-1/2}) / dx_d,
 * with the face states and fluxes of g->scheme.  U is overwritten
 * with U_new.  If next_dt_dev is not NULL the CFL step of U_new (same
 * formula as hard_cfl_dt, factor cfl) is written there in the same pass;
 * next_dt_dev may equal dt_dev.  Stream-ordered, no host synchronisation,
 * no allocation; graph-capturable. */
hard_status_t hard_hydro_step(const hard_grid_t* g, void* U, const double* dt_dev, double cfl,
                              double* next_dt_dev, void* work, size_t work_bytes, void* stream);

/* hard_hydro_step for callers that cannot allocate device memory (code
 * under graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same step through the same kernels, with the workspace
 * taken from a static device array of HARD_NOALLOC_SCRATCH_BYTES bytes that
 * the library holds on every GPU it runs on until the process ends.  The
 * call allocates nothing.  Grids whose hard_workspace_bytes exceeds that size
 * return HARD_ERR_WORKSPACE before anything is enqueued.  Each call first
 * clears the array's control block with a fill kernel; if flags_dev (device
 * uint32, may be NULL) is given it receives the status bits (HARD_FLAG_*)
 * of this call's step when the enqueued work completes.  All calls on one
 * GPU share that GPU's array: calls that may overlap in time (different
 * streams, threads or processes' own libraries aside) race and must be
 * stream-ordered by the caller.  The array's contents after a call are
 * those of its last step. */
#define HARD_NOALLOC_SCRATCH_BYTES (64u << 20)
hard_status_t hard_hydro_step_noalloc(const hard_grid_t* g, void* U, const double* dt_dev,
                                      double cfl, double* next_dt_dev, uint32_t* flags_dev,
                                      void* stream);

/* One stage of hard_hydro_step (stage = 1 or 2), for callers that schedule
 * the two stages themselves (hard_hydro_step is exactly stage 1 then 2):
 *   stage 1: dst = src + dt L(src)                      (src = U^n, dst = U^1)
 *   stage 2: dst = (un + (src + dt L(src))) / 2         (src = U^1, un = U^n)
 * dst may alias un in stage 2, never src.  next_dt_dev (stage 2 only, may be
 * NULL) receives the CFL step of dst.  Same layouts and rules as
 * hard_hydro_step; for HARD_SCHEME_MUSCL_HLLC without next_dt_dev the
 * workspace needs only the control block (256 bytes), otherwise the full
 * hard_workspace_bytes (which holds the per-workgroup slots of the CFL
 * reduction and, for HARD_SCHEME_WENO5Z_HLL, the pipeline arrays). */
hard_status_t hard_hydro_stage(const hard_grid_t* g, int32_t stage, const void* src,
                               const void* un, void* dst, const double* dt_dev, double cfl,
                               double* next_dt_dev, void* work, size_t work_bytes, void* stream);

/* Run to time t_end from U (in place), the time loop of the paper's control
 * model (section 2.1) with a CFL step each step: dt = min(CFL dt of U,
 * t_end - t); stops when t >= t_end (1 - 1e-14) or after max_steps steps.
 * The loop runs on the device in batches (t, dt and the stop flag live in
 * the workspace; steps after the end are exact no-ops with dt = 0); the host
 * synchronises once per batch.  A 1D MUSCL-HLLC grid of at most 2048 cells
 * without radiation runs the loop in one resident workgroup, up to 1024
 * steps per launch, with the same result bit for bit.  Writes the final t
 * and the number of steps taken; returns HARD_ERR_NONPHYSICAL if the status
 * word has bits set. */
hard_status_t hard_run(const hard_grid_t* g, void* U, double cfl, double t_end, int64_t max_steps,
                       double* t_out, int64_t* steps_out, void* work, size_t work_bytes,
                       void* stream);

/* Read the status word into *flags (HARD_FLAG_* bits), then clear it.
 * Synchronises the stream.  Returns HARD_ERR_NONPHYSICAL if any bit was set. */
hard_status_t hard_status_read(void* work, size_t work_bytes, uint32_t* flags, void* stream);

/* Per-field totals sum_i U[v][i] over the interior (v = 0..nvar-1) in
 * double, from compensated per-thread sums combined in a fixed order
 * (bitwise reproducible).  sums_dev: device array of nvar doubles. */
hard_status_t hard_conservation_sums(const hard_grid_t* g, const void* U, double* sums_dev,
                                     void* work, size_t work_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Batched: many independent problems, each with its own grid and its own
 * CFL time step, packed into one buffer and advanced by one launch per stage.
 * ------------------------------------------------------------------------ */
typedef struct hard_batch_plan hard_batch_plan_t;

/* Build a plan for nprob grids (host array, copied).  All grids must share
 * dtype and gamma.  Problem p's state occupies elements
 * [offset[p], offset[p+1]) of the packed buffer, laid out as a single grid.
 * tune_cache may name a text file of work-item shapes written by the
 * autotuner (NULL = built-in defaults).  *out is owned by the library until
 * hard_batch_plan_destroy.  Allocates device memory for the plan tables
 * (this is the only allocating call; it synchronises the device). */
hard_status_t hard_batch_plan_create(const hard_grid_t* grids, int32_t nprob,
                                     const char* tune_cache, hard_batch_plan_t** out);
hard_status_t hard_batch_plan_destroy(hard_batch_plan_t* plan);

/* Element offsets of each problem in the packed buffer (host array of
 * nprob + 1 int64; offsets[nprob] is the total element count). */
hard_status_t hard_batch_offsets(const hard_batch_plan_t* plan, int64_t* offsets);

hard_status_t hard_batch_workspace_bytes(const hard_batch_plan_t* plan, size_t* bytes);

/* Per-problem CFL steps dt_dev[p] (device array of nprob doubles). */
hard_status_t hard_cfl_dt_batched(const hard_batch_plan_t* plan, const void* U, double cfl,
                                  double* dt_dev, void* work, size_t work_bytes, void* stream);

/* One Heun step of every problem with its own dt_dev[p].  If update_dt is
 * non-zero, dt_dev[p] is replaced by the CFL step of the new state of
 * problem p (factor cfl).  Stream-ordered, graph-capturable. */
hard_status_t hard_hydro_step_batched(const hard_batch_plan_t* plan, void* U, double* dt_dev,
                                      double cfl, int32_t update_dt, void* work,
                                      size_t work_bytes, void* stream);

/* Run every problem of the batch to its own t = t_end with its own CFL step
 * (dt_p = min(CFL dt of problem p, t_end - t_p), the last step clipped; once
 * a problem reaches t_end its further steps are exact no-ops with dt = 0).
 * dt_dev is a device array of nprob doubles used as the step buffer.
 * t_host / steps_host (host arrays of nprob, may be NULL) receive each
 * problem's final time and step count.  Synchronises the stream once per 32
 * steps; returns HARD_ERR_NONPHYSICAL if the status word has bits set. */
hard_status_t hard_run_batched(const hard_batch_plan_t* plan, void* U, double cfl, double t_end,
                               int64_t max_steps, double* dt_dev, double* t_host,
                               int64_t* steps_host, void* work, size_t work_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Adjoint (vector-Jacobian product) of one step with dt held fixed.
 * ------------------------------------------------------------------------ */

/* Workspace bytes for hard_hydro_step_adjoint (HARD_F64 only). */
hard_status_t hard_adjoint_workspace_bytes(const hard_grid_t* g, size_t* bytes);

/* lam <- (d U_new / d U_n)^T lam for the step U_n -> U_new of
 * hard_hydro_step with the fixed step *dt_dev (the derivative of the branch
 * taken at U_n: minmod, min/max and HLLC region choices are held).  U_n is
 * not modified; the intermediate stage is recomputed internally.  lam is a
 * device array shaped like U. */
hard_status_t hard_hydro_step_adjoint(const hard_grid_t* g, const void* U_n, const double* dt_dev,
                                      void* lam, void* work, size_t work_bytes, void* stream);

/* hard_hydro_step_adjoint with the intermediate stage supplied: U_1 must be
 * the stage-1 state of U_n for the same dt, U_1 = U_n + dt L(U_n), as
 * hard_hydro_stage (stage 1) writes it (a checkpointed reverse pass has it
 * from recomputing the step forward).  The call then skips its own stage-1
 * recomputation; the result is the same.  U_1 is read only and must not
 * alias lam. */
hard_status_t hard_hydro_step_adjoint_given_u1(const hard_grid_t* g, const void* U_n,
                                               const void* U_1, const double* dt_dev, void* lam,
                                               void* work, size_t work_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Implicit radiation diffusion (rad = 1): one backward-Euler step of the
 * diffusion term of the radiation energy equation (section 2.2.1, equation
 * "radiation": d_t E_r = div(D grad E_r), D = c lambda / (kappa rho), lambda
 * from the flux limiter), solved by geometric multigrid V-cycles with regular
 * coarsening (section 2.2.2: the multigrid solver of A u = f, the residual
 * equation on every coarser grid, the V-cycle).
 *
 * The operator-split diffusion part of a step: call it after hard_hydro_step
 * with the same dt.  D is evaluated once from the state at the start of the
 * call (so the system is linear), and E_r (field ndim + 2 of U) is replaced by
 * the V-cycle iterate of
 *     A E_new = E_old,   (A x)_c = x_c + sum_faces a_f (x_c - x_nb),
 *     a_f = dt (D_c + D_nb)/2 / dx_d^2,
 * with grad E_r by central differences and zero-flux walls on non-periodic
 * sides.  The other fields are not modified.
 *
 * Solver: red-black Gauss-Seidel relaxation (cells with i + j + k even
 * first), residual restriction by the mean over the children, prolongation by
 * linear interpolation, coarse operators rediscretised from the mean of D
 * over the children.  Every axis whose size is even is halved (a periodic
 * axis only while the half is even or one); the coarsest level is relaxed
 * `ncoarse` sweeps from zero.  After pre-smoothing (nu1 > 0) the residuals
 * of the black cells, zero in exact arithmetic after a black half-sweep, are
 * taken as zero, so results agree with a plain evaluation to rounding only.
 * ------------------------------------------------------------------------ */
#define HARD_FLD_EDDINGTON 0 /* lambda = 1/3 (optically thick limit) */
#define HARD_FLD_LEVERMORE 1 /* lambda = (2 + R)/(6 + 3R + R^2),
                                R = |grad E_r| / (rho kappa E_r) */

typedef struct hard_gmg_opts_t {
  int32_t limiter; /* HARD_FLD_EDDINGTON or HARD_FLD_LEVERMORE */
  int32_t ncycles; /* V-cycles, 0..1000 (0: E_r unchanged) */
  int32_t nu1;     /* red-black sweeps before the coarse correction, 0..64 */
  int32_t nu2;     /* red-black sweeps after it, 0..64 */
  int32_t ncoarse; /* sweeps on the coarsest level, 1..1024 */
} hard_gmg_opts_t;

/* Sizes of the multigrid levels of grid g, finest first: levels_n[3 l + d]
 * for l < min(*nlevels, max_levels).  Host only.  The grid rules are those of
 * hard_rad_diffuse. */
hard_status_t hard_gmg_levels(const hard_grid_t* g, int32_t max_levels, int64_t* levels_n,
                              int32_t* nlevels);

/* Workspace bytes for hard_rad_diffuse (control block and the arrays of every
 * level: about 3.4 doubles per finest cell in 3D). */
hard_status_t hard_rad_diffuse_workspace_bytes(const hard_grid_t* g, size_t* bytes);

/* One implicit diffusion step of E_r in U (in place) with the step *dt_dev
 * (device double, dt >= 0), by opts->ncycles V(nu1, nu2) cycles starting from
 * E_old.  resid_dev (device array of ncycles + 1 doubles, or NULL) receives
 * the 2-norm of the finest-level residual E_old - A x before the first cycle
 * and after each one (per-tile sums added in a fixed order: bitwise
 * reproducible).
 * Requirements: g->rad = 1, g->kappa > 0, every periodic axis of even size
 * (odd: HARD_ERR_UNSUPPORTED).  HARD_F32 states are read into and solved in
 * double; E_r is rounded to float when it is stored back.
 * rho <= 0 sets HARD_FLAG_DENSITY, E_r <= 0 or a non-finite D sets
 * HARD_FLAG_RADIATION in the status word.  Stream-ordered, no host
 * synchronisation, no allocation; graph-capturable. */
hard_status_t hard_rad_diffuse(const hard_grid_t* g, void* U, const double* dt_dev,
                               const hard_gmg_opts_t* opts, double* resid_dev, void* work,
                               size_t work_bytes, void* stream);

/* hard_run for a state with the radiation field, with the implicit
 * diffusion in every step: the operator split of section 2.2.2 under the
 * control model of section 2.1.  Each step takes dt = min(CFL dt, t_end - t)
 * as hard_run does, then hard_hydro_step (hydro fields and E_r advected,
 * heating/cooling exchange) and hard_rad_diffuse with the same dt and
 * `opts`.  work: a hard_workspace_bytes workspace; fld_work: a
 * hard_rad_diffuse_workspace_bytes workspace (its control block's dt slot
 * holds the step size).  Both must be cleared before first use.  The host
 * synchronises once per 64 steps; steps after the end are exact no-ops.
 * Writes the final t and the number of steps; returns HARD_ERR_NONPHYSICAL
 * if either status word has bits set.  Requires g->rad = 1, g->kappa > 0. */
hard_status_t hard_run_rhd(const hard_grid_t* g, void* U, double cfl, double t_end,
                           int64_t max_steps, const hard_gmg_opts_t* opts, double* t_out,
                           int64_t* steps_out, void* work, size_t work_bytes, void* fld_work,
                           size_t fld_work_bytes, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* HARD_H */
