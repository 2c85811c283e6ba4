// Reductions over a whole grid: the standalone CFL time step, the
// compensated conservation sums, and the control-block clear.

#include "hydro_device.hpp"
#include "launch.hpp"

namespace hard {

constexpr int RED_THREADS = 256;

// dt = cfl / max_i sum_d (|u_d| + c)/dx_d over the interior (the paper's
// section 3.5 says only that dt follows the CFL condition; this is the
// library's reading).  Grid-stride over cells; also ORs the status bits.
struct CflGeo {
  int n[3];
  double dx[3], inv_dx[3];
  int dx_pow2;
};

template <int NDIM, typename R>
__global__ __launch_bounds__(RED_THREADS) void cfl_kernel(const R* __restrict__ U, CflGeo g,
                                                          double gamma, Control* ctl,
                                                          double* slots) {
  constexpr int NV = NDIM + 2;
  const long long N = (long long)g.n[0] * g.n[1] * g.n[2];
  double smax = 0.0;
  unsigned flags = 0;
  for (long long c = (long long)blockIdx.x * RED_THREADS + threadIdx.x; c < N;
       c += (long long)gridDim.x * RED_THREADS) {
    double Ud[NV];
    R Ur[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      Ur[v] = U[v * N + c];
      Ud[v] = (double)Ur[v];
    }
    R W[NV];
    to_primitive<R, NDIM>(Ur, W, gamma - 1.0);
    flags |= cell_flags<R, NV>(Ur, W[NV - 1]);
    smax = fmax(smax, cfl_signal<R, NDIM>(Ud, g.inv_dx, gamma));
  }
  block_finish<RED_THREADS>(flags, smax, true, ctl, slots + blockIdx.x);
}

// dt = cfl / (max of the per-workgroup signal-sum maxima), one workgroup.
constexpr int FINAL_THREADS = 1024;
__global__ __launch_bounds__(FINAL_THREADS) void cfl_final_kernel(const double* __restrict__ slots,
                                                                  int n, double cfl, double* dt) {
  __shared__ double red[FINAL_THREADS / 64];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += FINAL_THREADS) s = fmax(s, slots[i]);
  s = wave_max(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = 0.0;
    for (int i = 0; i < FINAL_THREADS / 64; ++i) m = fmax(m, red[i]);
    *dt = cfl / m;
  }
}

hipError_t launch_cfl_final(const double* slots, int n, double cfl, double* dt, hipStream_t s) {
  hipLaunchKernelGGL(cfl_final_kernel, dim3(1), dim3(FINAL_THREADS), 0, s, slots, n, cfl, dt);
  return hipGetLastError();
}

static int cfl_blocks(long long N) {
  long long b = (N + RED_THREADS * 4 - 1) / (RED_THREADS * 4);
  if (b > GRID_STRIDE_MAX_BLOCKS) b = GRID_STRIDE_MAX_BLOCKS;
  if (b < 1) b = 1;
  return (int)b;
}

hipError_t launch_cfl(int ndim, int dtype, const int* n, const double* dx, const double* inv_dx,
                      int dx_pow2, double gamma, const void* U, double cfl, double* dt,
                      Control* ctl, double* slots, int nslots, hipStream_t s) {
  long long N = (long long)n[0] * n[1] * n[2];
  const int nb = cfl_blocks(N);
  if (nb > nslots) return hipErrorInvalidValue;
  dim3 grid(nb), block(RED_THREADS);
  CflGeo g;
  for (int d = 0; d < 3; ++d) {
    g.n[d] = n[d];
    g.dx[d] = dx[d];
    g.inv_dx[d] = inv_dx[d];
  }
  g.dx_pow2 = dx_pow2;
#define HARD_CFL(D, T)                                                                      \
  hipLaunchKernelGGL((cfl_kernel<D, T>), grid, block, 0, s, static_cast<const T*>(U), g, gamma, \
                     ctl, slots)
  if (dtype == 0) {
    if (ndim == 1) HARD_CFL(1, double);
    else if (ndim == 2) HARD_CFL(2, double);
    else HARD_CFL(3, double);
  } else {
    if (ndim == 1) HARD_CFL(1, float);
    else if (ndim == 2) HARD_CFL(2, float);
    else HARD_CFL(3, float);
  }
#undef HARD_CFL
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_cfl_final(slots, nb, cfl, dt, s);
}

__global__ void control_clear_kernel(Control* ctl) {
  unsigned long long* w = reinterpret_cast<unsigned long long*>(ctl);
  if (threadIdx.x < sizeof(Control) / 8) w[threadIdx.x] = 0ull;
}

// Time control of hard_run: clamp dt so the run lands on t_end, advance t,
// and turn every step after the end into dt = 0 (an exact no-op step).
__global__ void time_control_kernel(Control* ctl, double t_end, long long max_steps) {
#pragma clang fp contract(off)
  if (threadIdx.x != 0) return;
  double t = ctl->t;
  long long s = ctl->steps;
  if (ctl->done || !(t < t_end * (1.0 - 1e-14)) || s >= max_steps) {
    ctl->done = 1;
    ctl->dt = 0.0;
    return;
  }
  double d = ctl->dt;
  if (d > t_end - t) d = t_end - t;
  ctl->dt = d;
  ctl->t = t + d;
  ctl->steps = s + 1;
}

hipError_t launch_time_control(Control* ctl, double t_end, long long max_steps, hipStream_t s) {
  hipLaunchKernelGGL(time_control_kernel, dim3(1), dim3(64), 0, s, ctl, t_end, max_steps);
  return hipGetLastError();
}

hipError_t launch_control_clear(Control* ctl, hipStream_t s) {
  hipLaunchKernelGGL(control_clear_kernel, dim3(1), dim3(64), 0, s, ctl);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Compensated sums.  Each thread keeps (hi, lo) with an error-free TwoSum per
// added value; pairs are then combined in a fixed tree inside the block and
// in fixed block order by a second kernel, so the result does not depend on
// scheduling.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void two_sum(double a, double b, double& s, double& e) {
  s = a + b;
  double bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

__device__ __forceinline__ void pair_add(double& hi, double& lo, double h2, double l2) {
  double s, e;
  two_sum(hi, h2, s, e);
  hi = s;
  lo = lo + l2 + e;
}

template <typename R>
__global__ __launch_bounds__(RED_THREADS) void sums_kernel(const R* __restrict__ U, long long N,
                                                           int nvar, double* partials) {
  __shared__ double sh[RED_THREADS], sl[RED_THREADS];
  for (int v = 0; v < nvar; ++v) {
    double hi = 0.0, lo = 0.0;
    for (long long c = (long long)blockIdx.x * RED_THREADS + threadIdx.x; c < N;
         c += (long long)gridDim.x * RED_THREADS) {
      double s, e;
      two_sum(hi, (double)U[v * N + c], s, e);
      hi = s;
      lo += e;
    }
    sh[threadIdx.x] = hi;
    sl[threadIdx.x] = lo;
    __syncthreads();
    for (int w = RED_THREADS / 2; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) {
        double h = sh[threadIdx.x], l = sl[threadIdx.x];
        pair_add(h, l, sh[threadIdx.x + w], sl[threadIdx.x + w]);
        sh[threadIdx.x] = h;
        sl[threadIdx.x] = l;
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      partials[((long long)blockIdx.x * nvar + v) * 2] = sh[0];
      partials[((long long)blockIdx.x * nvar + v) * 2 + 1] = sl[0];
    }
    __syncthreads();
  }
}

__global__ void sums_final_kernel(const double* partials, int nblocks, int nvar, double* out) {
  int v = threadIdx.x;
  if (v >= nvar) return;
  double hi = 0.0, lo = 0.0;
  for (int b = 0; b < nblocks; ++b)
    pair_add(hi, lo, partials[((long long)b * nvar + v) * 2], partials[((long long)b * nvar + v) * 2 + 1]);
  out[v] = hi + lo;
}

int sums_blocks(long long N) {
  long long b = (N + RED_THREADS * 16 - 1) / (RED_THREADS * 16);
  if (b > 1024) b = 1024;
  if (b < 1) b = 1;
  return (int)b;
}

hipError_t launch_sums(int nvar, int dtype, const int* n, const void* U, double* partials,
                       int nblocks_max, double* out, hipStream_t s) {
  long long N = (long long)n[0] * n[1] * n[2];
  int nb = sums_blocks(N);
  if (nb > nblocks_max) return hipErrorInvalidValue;
  if (dtype == 0)
    hipLaunchKernelGGL(sums_kernel<double>, dim3(nb), dim3(RED_THREADS), 0, s,
                       static_cast<const double*>(U), N, nvar, partials);
  else
    hipLaunchKernelGGL(sums_kernel<float>, dim3(nb), dim3(RED_THREADS), 0, s,
                       static_cast<const float*>(U), N, nvar, partials);
  hipLaunchKernelGGL(sums_final_kernel, dim3(1), dim3(64), 0, s, partials, nb, nvar, out);
  return hipGetLastError();
}

}  // namespace hard
