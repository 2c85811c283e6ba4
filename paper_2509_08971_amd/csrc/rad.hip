// Radiation energy density E_r as one more conserved field (section 2.2.1:
// the fourth row of the conservation law and its heating source).
//
//   rad_advect  per Heun stage, one thread per cell: the E_r update of that
//               stage, L(E_r) = -sum_d (F+ - F-)/dx_d with the local
//               Lax-Friedrichs (Rusanov) flux of MUSCL-minmod face states
//               (section 2.2.2), the signal speed max(|u_L| + c_L, |u_R| +
//               c_R) taken from the hydro face states.  The hydro fields of
//               the same stage are updated by the fused stage kernel; E_r
//               does not act on them, so the two kernels are independent.
//   rad_source  after stage 2, one thread per cell: the exchange between
//               fluid internal energy and radiation by the heating rate
//               qdot = c kappa rho (E_r - a T^4) (equation "heating-cooling"),
//               backward Euler solved for the new temperature by Newton
//               iterations from an upper bound; then the CFL step of the
//               state after the exchange, folded into the same pass.
//
// Plain arithmetic throughout (IEEE division and square root, no
// contraction): the face states of E_r react to the last bits of the
// primitives, and the Newton iteration stops on a rounding-level test.

#include "hydro_device.hpp"
#include "launch.hpp"

namespace hard {

// CGS constants (CODATA 2018): speed of light, radiation constant a = 4 sigma/c,
// Boltzmann constant, atomic mass unit.
constexpr double RC_LIGHT = 2.99792458e10;
constexpr double RA_RAD = 4.0 * 5.670374419e-5 / 2.99792458e10;
constexpr double RK_B = 1.380649e-16;
constexpr double RM_U = 1.66053906660e-24;

// minmod with the zero and tie rules of the method: 0 if a b <= 0, else the
// argument of smaller magnitude, a on a tie.
__device__ __forceinline__ double minmod_rule(double a, double b) {
  if (a * b <= 0.0) return 0.0;
  return fabs(a) <= fabs(b) ? a : b;
}

template <typename R, int NDIM, int STAGE>
__global__ __launch_bounds__(256) void rad_advect(RadArgs a) {
#pragma clang fp contract(off)
  constexpr int NH = NDIM + 2;  // hydro fields; E_r is field NH
  const int nx = a.n[0], ny = a.n[1], nz = a.n[2];
  const long long N = (long long)nx * ny * nz;
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  unsigned flags = 0;
  if (c < N) {
    const R* src = static_cast<const R*>(a.src);
    const int ci[3] = {(int)(c % nx), (int)((c / nx) % ny), (int)(c / ((long long)nx * ny))};
    double l = 0.0;
#pragma unroll
    for (int d = 0; d < NDIM; ++d) {
      // five cells c-2 .. c+2 along d: rho, u_d, p, E_r (wall flip of m_d)
      double rho[5], un[5], p[5], er[5];
#pragma unroll
      for (int s = 0; s < 5; ++s) {
        bool flip;
        int cc[3] = {ci[0], ci[1], ci[2]};
        cc[d] = remap(ci[d] - 2 + s, a.n[d], a.bc[d][0], a.bc[d][1], flip);
        const long long q = ((long long)cc[2] * ny + cc[1]) * nx + cc[0];
        const double r = (double)src[q];
        double m2 = 0.0, md = 0.0;
#pragma unroll
        for (int k = 0; k < NDIM; ++k) {
          const double m = (double)src[(1 + k) * N + q];
          m2 = k == 0 ? m * m : m2 + m * m;
          if (k == d) md = m;
        }
        if (flip) md = -md;
        const double ke = 0.5 * m2 / r;
        rho[s] = r;
        un[s] = md / r;
        p[s] = (a.gamma - 1.0) * ((double)src[(NDIM + 1) * N + q] - ke);
        er[s] = (double)src[NH * N + q];
      }
      // faces c-1/2 (cells 0..3 of the five) and c+1/2 (cells 1..4)
      double F[2];
#pragma unroll
      for (int f = 0; f < 2; ++f) {
        const double* R_ = rho + f;
        const double* U_ = un + f;
        const double* P_ = p + f;
        const double* E_ = er + f;
        auto face = [](const double* w, double& wl, double& wr) {
          const double sl = minmod_rule(w[1] - w[0], w[2] - w[1]);
          const double sr = minmod_rule(w[2] - w[1], w[3] - w[2]);
          wl = w[1] + 0.5 * sl;
          wr = w[2] - 0.5 * sr;
        };
        double rL, rR, uL, uR, pL, pR, eL, eR;
        face(R_, rL, rR);
        face(U_, uL, uR);
        face(P_, pL, pR);
        face(E_, eL, eR);
        const double cL = sqrt(a.gamma * pL / rL), cR = sqrt(a.gamma * pR / rR);
        const double sL = fabs(uL) + cL, sR = fabs(uR) + cR;
        const double sm = sL >= sR ? sL : sR;
        F[f] = 0.5 * (eL * uL + eR * uR) - 0.5 * sm * (eR - eL);
      }
      const double df = F[1] - F[0];
      l = l - (a.dx_pow2 ? df * a.inv_dx[d] : df / a.dx[d]);
    }
    R* dst = static_cast<R*>(a.dst);
    const R* un_ = static_cast<const R*>(a.un);
    const R ec = src[NH * N + c];
    const R dt = R(*a.dt);
    R out;
    if (STAGE == 1)
      out = ec + dt * R(l);
    else
      out = R(0.5) * (un_[NH * N + c] + (ec + dt * R(l)));
    dst[NH * N + c] = out;
    if (!isfinite(out)) flags = FLAG_NONFINITE;
  }
  flags = wave_or(flags);
  if ((threadIdx.x & 63) == 0 && flags) atomicOr(&a.ctl->flags, flags);
}

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

template <typename R, int NDIM>
__global__ __launch_bounds__(256) void rad_source(RadArgs a) {
#pragma clang fp contract(off)
  constexpr int NH = NDIM + 2;
  const long long N = (long long)a.n[0] * a.n[1] * a.n[2];
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  double smax = 0.0;
  unsigned flags = 0;
  if (c < N) {
    R* U = static_cast<R*>(a.dst);
    const double rho = (double)U[c];
    double m2 = 0.0;
#pragma unroll
    for (int k = 0; k < NDIM; ++k) {
      const double m = (double)U[(1 + k) * N + c];
      m2 = k == 0 ? m * m : m2 + m * m;
    }
    const double ke = 0.5 * m2 / rho;
    double Ef = (double)U[(NDIM + 1) * N + c], Er = (double)U[NH * N + c];
    const double Ef0 = Ef, Er0 = Er;
    exchange(rho, ke, Ef, Er, *a.dt, a.gamma, a.kappa, a.mu);
    if (Ef != Ef0) U[(NDIM + 1) * N + c] = R(Ef);
    if (Er != Er0) U[NH * N + c] = R(Er);
    if (!isfinite(Er) || !isfinite(Ef)) flags = FLAG_NONFINITE;
    if (a.fuse_cfl) {
      double Ud[NH];
#pragma unroll
      for (int v = 0; v < NH; ++v) Ud[v] = (double)U[v * N + c];
      smax = signal_sum<NDIM>(Ud, a.dx, a.inv_dx, a.dx_pow2, a.gamma);
    }
  }
  block_finish<256>(flags, smax, a.fuse_cfl != 0, a.ctl, a.cfl, a.next_dt);
}

template <typename R, int NDIM>
static void rad_advect_t(const RadArgs& a, int stage, dim3 grid, hipStream_t s) {
  if (stage == 1)
    hipLaunchKernelGGL((rad_advect<R, NDIM, 1>), grid, dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL((rad_advect<R, NDIM, 2>), grid, dim3(256), 0, s, a);
}

hipError_t launch_rad_advect(int ndim, int dtype, const RadArgs& a, int stage, hipStream_t s) {
  const long long N = (long long)a.n[0] * a.n[1] * a.n[2];
  const dim3 grid((unsigned)((N + 255) / 256));
  if (dtype == 0) {
    if (ndim == 1) rad_advect_t<double, 1>(a, stage, grid, s);
    else if (ndim == 2) rad_advect_t<double, 2>(a, stage, grid, s);
    else rad_advect_t<double, 3>(a, stage, grid, s);
  } else {
    if (ndim == 1) rad_advect_t<float, 1>(a, stage, grid, s);
    else if (ndim == 2) rad_advect_t<float, 2>(a, stage, grid, s);
    else rad_advect_t<float, 3>(a, stage, grid, s);
  }
  return hipGetLastError();
}

hipError_t launch_rad_source(int ndim, int dtype, const RadArgs& a, hipStream_t s) {
  const long long N = (long long)a.n[0] * a.n[1] * a.n[2];
  const dim3 grid((unsigned)((N + 255) / 256)), block(256);
  if (dtype == 0) {
    if (ndim == 1) hipLaunchKernelGGL((rad_source<double, 1>), grid, block, 0, s, a);
    else if (ndim == 2) hipLaunchKernelGGL((rad_source<double, 2>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((rad_source<double, 3>), grid, block, 0, s, a);
  } else {
    if (ndim == 1) hipLaunchKernelGGL((rad_source<float, 1>), grid, block, 0, s, a);
    else if (ndim == 2) hipLaunchKernelGGL((rad_source<float, 2>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((rad_source<float, 3>), grid, block, 0, s, a);
  }
  return hipGetLastError();
}

}  // namespace hard
