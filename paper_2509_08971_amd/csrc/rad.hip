// Radiation energy density E_r as one more conserved field (section 2.2.1:
// the fourth row of the conservation law and its heating source).
//
// The advection of E_r in each Heun stage runs inside the stage kernels
// (the tile carries E_r as one more field; its face flux is rusanov_er in
// hydro_device.hpp).  This file holds the exchange after stage 2:
//   rad_source  grid-stride over the cells: the exchange between fluid
//               internal energy and radiation by the heating rate
//               qdot = c kappa rho (E_r - a T^4) (equation "heating-cooling"),
//               backward Euler solved for the new temperature by Newton
//               iterations from an upper bound; then the CFL step of the
//               state after the exchange, folded into the same pass.
//
// Plain arithmetic (IEEE division and square root, no contraction): the
// Newton iteration stops on a rounding-level test.

#include "hydro_device.hpp"
#include "launch.hpp"

namespace hard {

// CGS constants (CODATA 2018): speed of light, radiation constant a = 4 sigma/c,
// Boltzmann constant, atomic mass unit.
constexpr double RC_LIGHT = 2.99792458e10;
constexpr double RA_RAD = 4.0 * 5.670374419e-5 / 2.99792458e10;
constexpr double RK_B = 1.380649e-16;
constexpr double RM_U = 1.66053906660e-24;

// Backward-Euler exchange of one cell (see the file comment); returns the
// new (E_fluid, E_r).  e + E_r is conserved; the kinetic energy is untouched.
__device__ __forceinline__ void exchange(double rho, double ke, double& Ef, double& Er, double dt,
                                         double gamma, double kappa, double mu) {
#pragma clang fp contract(off)
  const double q = RC_LIGHT * kappa * rho;
  const double dq = dt * q;
  if (!(dq > 0.0)) return;
  const double e = Ef - ke;
  const double Cv = rho * RK_B / (mu * RM_U * (gamma - 1.0));
  const double W = e + Er;
  const double t1 = W / Cv;
  const double t2 = sqrt(sqrt((W * (1.0 + dq) - Er) / (dq * RA_RAD)));
  double T = t1 < t2 ? t1 : t2;
  for (int it = 0; it < 200; ++it) {
    const double T3 = T * T * T;
    const double f = Cv * T + (Er + dq * RA_RAD * (T3 * T)) / (1.0 + dq) - W;
    const double fp = Cv + 4.0 * dq * RA_RAD * T3 / (1.0 + dq);
    const double Tn = T - f / fp;
    if (!(Tn < T)) break;
    T = Tn;
  }
  const double e_new = Cv * T;
  Ef = Ef + (e_new - e);
  Er = W - e_new;
}

// Grid-stride over the cells with a bounded grid (a few thousand workgroups,
// one CFL slot each).
constexpr unsigned RAD_SOURCE_BLOCKS = 2048;

template <typename R, int NDIM>
__global__ __launch_bounds__(256) void rad_source(RadArgs a) {
#pragma clang fp contract(off)
  constexpr int NH = NDIM + 2;
  const long long N = (long long)a.n[0] * a.n[1] * a.n[2];
  double smax = 0.0;
  unsigned flags = 0;
  R* U = static_cast<R*>(a.dst);
  for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < N;
       c += (long long)gridDim.x * blockDim.x) {
    double Ud[NH];  // the cell's hydro state after the exchange, as stored
    const double rho = (double)U[c];
    Ud[0] = rho;
    double m2 = 0.0;
#pragma unroll
    for (int k = 0; k < NDIM; ++k) {
      const double m = (double)U[(1 + k) * N + c];
      Ud[1 + k] = m;
      m2 = k == 0 ? m * m : m2 + m * m;
    }
    const double ke = 0.5 * m2 / rho;
    double Ef = (double)U[(NDIM + 1) * N + c], Er = (double)U[NH * N + c];
    const double Ef0 = Ef, Er0 = Er;
    exchange(rho, ke, Ef, Er, *a.dt, a.gamma, a.kappa, a.mu);
    if (Ef != Ef0) U[(NDIM + 1) * N + c] = R(Ef);
    if (Er != Er0) U[NH * N + c] = R(Er);
    if (!isfinite(Er) || !isfinite(Ef)) flags |= FLAG_NONFINITE;
    if (a.fuse_cfl) {
      // an unchanged value came from R, so R(value) is the stored word either
      // way; E_r is not part of the signal sum
      Ud[NDIM + 1] = (double)R(Ef);
      smax = fmax(smax, cfl_signal<R, NDIM>(Ud, a.dx, a.inv_dx, a.dx_pow2, a.gamma));
    }
  }
  block_finish<256>(flags, smax, a.fuse_cfl != 0, a.ctl, a.slots + blockIdx.x);
}

hipError_t launch_rad_source(int ndim, int dtype, const RadArgs& a, hipStream_t s) {
  const long long N = (long long)a.n[0] * a.n[1] * a.n[2];
  const long long nb = (N + 255) / 256;
  const unsigned nbs = (unsigned)(nb < RAD_SOURCE_BLOCKS ? nb : RAD_SOURCE_BLOCKS);
  if (a.fuse_cfl && (int)nbs > a.nslots) return hipErrorInvalidValue;
  const dim3 grid(nbs), block(256);
  if (dtype == 0) {
    if (ndim == 1) hipLaunchKernelGGL((rad_source<double, 1>), grid, block, 0, s, a);
    else if (ndim == 2) hipLaunchKernelGGL((rad_source<double, 2>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((rad_source<double, 3>), grid, block, 0, s, a);
  } else {
    if (ndim == 1) hipLaunchKernelGGL((rad_source<float, 1>), grid, block, 0, s, a);
    else if (ndim == 2) hipLaunchKernelGGL((rad_source<float, 2>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((rad_source<float, 3>), grid, block, 0, s, a);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !a.fuse_cfl) return e;
  return launch_cfl_final(a.slots, (int)nbs, a.cfl, a.next_dt, s);
}

}  // namespace hard
