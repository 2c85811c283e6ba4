// The time loop of hard_run for small 1D grids in one resident workgroup.
//
// A 1D grid of up to RUN1D_MAX cells fits one workgroup: each thread keeps
// its cells' conserved states in registers, the row of primitives (with the
// two ghost cells at each end) and the face fluxes live in LDS, and the
// workgroup runs up to `chunk` steps of the loop -- time control, both Heun
// stages, the CFL step of the new state -- per launch, with barriers between
// the phases instead of kernel boundaries.  The general loop pays four
// launches per step (time control, two stages, the dt reduction), which on a
// grid of a thousand cells are almost all of its time.
//
// The arithmetic is that of the tiled path, expression for expression: the
// same face states (muscl_pair), flux (hllc_ordered), update and stage
// combine, CFL signal (cfl_signal), dt = cfl / max and time control, so a run
// gives the same bits as the step-by-step loop (tested).

#include "hydro_device.hpp"
#include "launch.hpp"

namespace hard {

// K cells per thread: cell c is owned by thread c % RUN1D_THREADS.
template <typename R, int K>
__global__ __launch_bounds__(RUN1D_THREADS) void run1d_kernel(Run1dArgs a) {
  constexpr int NV = 3, NT = RUN1D_THREADS, MAXN = NT * K;
  __shared__ R W[NV][MAXN + 4];  // primitives of cells -2 .. n+1 at index q + 2
  __shared__ R F[NV][MAXN + 1];  // flux through face f (between cells f-1 and f)
  __shared__ double red[NT / 64];
  const int tid = threadIdx.x, n = a.n;
  R* Ug = static_cast<R*>(a.U);
  const double gm1 = a.gamma - 1.0;
  const R gam = R(a.gamma);
  const R inv_gm1 = R(1.0 / gm1);
  const R idx0 = R(a.inv_dx);
  const double idxa[3] = {a.inv_dx, 1.0, 1.0};

  R Un[K][NV], U1[K][NV];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int c = tid + k * NT;
#pragma unroll
    for (int v = 0; v < NV; ++v) Un[k][v] = c < n ? Ug[v * n + c] : R(0);
  }
  Control* ctl = a.ctl;
  double t = ctl->t, dtn = ctl->dt;
  long long steps = ctl->steps;
  int done = ctl->done;
  unsigned flags = 0;

  // one Heun stage: primitives of Src into W, faces into F, then for every
  // own cell Out = Src + dt L (stage 1) or 1/2 (Un + (Src + dt L)) (stage 2)
  auto stage = [&](R (&Src)[K][NV], R (&Out)[K][NV], R dt, bool second) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int c = tid + k * NT;
      if (c < n) {
        R P[NV];
        to_primitive<R, 1>(Src[k], P, gm1);
        flags |= cell_flags<R, NV>(Src[k], P[NV - 1]);
#pragma unroll
        for (int v = 0; v < NV; ++v) W[v][c + 2] = P[v];
        if (c < 2 || c >= n - 2) {
          // the ghost cells -2, -1, n, n+1 whose source this cell is
          for (int gi = 0; gi < 4; ++gi) {
            const int q = gi < 2 ? gi - 2 : n + gi - 2;
            bool flip;
            if (remap(q, n, a.bc[0], a.bc[1], flip) != c) continue;
#pragma unroll
            for (int v = 0; v < NV; ++v) W[v][q + 2] = (v == 1 && flip) ? -P[v] : P[v];
          }
        }
      }
    }
    __syncthreads();
    for (int f = tid; f <= n; f += NT) {
      R WL[NV], WR[NV], Fn[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) muscl_pair(W[v][f], W[v][f + 1], W[v][f + 2], W[v][f + 3], WL[v], WR[v]);
      hllc_ordered<R, NV>(WL, WR, gam, inv_gm1, Fn);
#pragma unroll
      for (int v = 0; v < NV; ++v) F[v][f] = Fn[v];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int c = tid + k * NT;
      if (c < n) {
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          R l = R(0) - (F[v][c + 1] - F[v][c]) * idx0;
          if (!second) {
            Out[k][v] = Src[k][v] + dt * l;
          } else {
            Out[k][v] = R(0.5) * (Out[k][v] + (Src[k][v] + dt * l));
          }
        }
      }
    }
    // no barrier here: the next stage writes W, whose last reads came before
    // the barrier above, and F only after its own first barrier, which every
    // thread passes after this update
  };

  for (int it = 0; it < a.chunk; ++it) {
    {
      // time control: clamp dt so the run lands on t_end, advance t
#pragma clang fp contract(off)
      if (done || !(t < a.t_end * (1.0 - 1e-14)) || steps >= a.max_steps) {
        done = 1;
        break;
      }
      double d = dtn;
      if (d > a.t_end - t) d = a.t_end - t;
      dtn = d;
      t = t + d;
      steps = steps + 1;
    }
    const R dt = R(dtn);
    stage(Un, U1, dt, false);
    stage(U1, Un, dt, true);
    // CFL step of the new state: dt = cfl / max over the cells
    double smax = 0.0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int c = tid + k * NT;
      if (c < n) {
        double Ud[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) Ud[v] = (double)Un[k][v];
        smax = fmax(smax, cfl_signal<R, 1>(Ud, idxa, a.gamma));
      }
    }
    smax = wave_max(smax);
    if ((tid & 63) == 0) red[tid >> 6] = smax;
    __syncthreads();
    double m = 0.0;
#pragma unroll
    for (int i = 0; i < NT / 64; ++i) m = fmax(m, red[i]);
    dtn = a.cfl / m;
    // red is written again only after the next step's four barriers
  }

#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int c = tid + k * NT;
    if (c < n) {
      // the step-by-step loop checks the final state once more, as the
      // source of the exact no-op step (dt = 0) that follows the end
      if (done) {
        R P[NV];
        to_primitive<R, 1>(Un[k], P, gm1);
        flags |= cell_flags<R, NV>(Un[k], P[NV - 1]);
      }
#pragma unroll
      for (int v = 0; v < NV; ++v) Ug[v * n + c] = Un[k][v];
    }
  }
  flags = wave_or(flags);
  if ((tid & 63) == 0 && flags) atomicOr(&ctl->flags, flags);
  if (tid == 0) {
    ctl->t = t;
    ctl->steps = steps;
    ctl->dt = done ? 0.0 : dtn;
    ctl->done = done;
  }
}

hipError_t launch_run1d(int dtype, const Run1dArgs& a, hipStream_t s) {
  if (a.n < 2 || a.n > RUN1D_MAX || a.chunk < 1) return hipErrorInvalidValue;
  const bool one = a.n <= RUN1D_THREADS;
  if (dtype == 0) {
    if (one) hipLaunchKernelGGL((run1d_kernel<double, 1>), dim3(1), dim3(RUN1D_THREADS), 0, s, a);
    else hipLaunchKernelGGL((run1d_kernel<double, 2>), dim3(1), dim3(RUN1D_THREADS), 0, s, a);
  } else {
    if (one) hipLaunchKernelGGL((run1d_kernel<float, 1>), dim3(1), dim3(RUN1D_THREADS), 0, s, a);
    else hipLaunchKernelGGL((run1d_kernel<float, 2>), dim3(1), dim3(RUN1D_THREADS), 0, s, a);
  }
  return hipGetLastError();
}

}  // namespace hard
