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
//   rad_source  after stage 2, grid-stride over the cells: the exchange between
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

// The E_r part of a Heun stage on a 3D grid, as a walk: a workgroup takes a
// 32 x 8 tile of cells in x-y and walks it along z over a chunk of planes.
// For each plane the primitives (rho, u_x, u_y, p, E_r) of the tile and its
// two-cell halo in x and y (ghosts by index remap, the normal velocity
// negated beyond a reflecting wall) go to LDS once, every x and y face of the
// plane is computed once into LDS, and the z faces come from a window of five
// planes of (rho, u_z, p, E_r) that each thread keeps for its own column (the
// face above a cell is the face below it on the next plane).  The window is
// fed from the LDS plane, so each cell of a plane is read and its primitives
// recovered once (its halo copies aside): a thread finishes plane q-2 when
// plane q arrives, carrying the x and y part of L of the planes in between.
// Face states, fluxes and the stage combine are those of rad_advect, term for
// term and in the same order.
constexpr int RW_TX = 32, RW_TY = 8, RW_CZ = 32;
constexpr int RW_LX = RW_TX + 4, RW_LY = RW_TY + 4;

// Primitives of cell q of src: rho, u_x, u_y, u_z, p, E_r; the momentum of
// axis `flip_axis` (or none, -1) negated first.
template <typename R>
__device__ __forceinline__ void rad_prims(const R* src, long long N, long long q, double gamma,
                                          int flip_axis, double* w) {
#pragma clang fp contract(off)
  const double r = (double)src[q];
  double m[3];
  double m2 = 0.0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    m[k] = (double)src[(1 + k) * N + q];
    m2 = k == 0 ? m[k] * m[k] : m2 + m[k] * m[k];
  }
  const double ke = 0.5 * m2 / r;
#pragma unroll
  for (int k = 0; k < 3; ++k) w[1 + k] = (k == flip_axis ? -m[k] : m[k]) / r;
  w[0] = r;
  w[4] = (gamma - 1.0) * ((double)src[4 * N + q] - ke);
  w[5] = (double)src[5 * N + q];
}

// Rusanov flux of E_r at the face between cells 1 and 2 of four cells
// (rho, u_n, p, E_r per cell), from MUSCL-minmod face states.
__device__ __forceinline__ double rad_face(const double* rho, const double* un, const double* p,
                                           const double* er, double gamma) {
#pragma clang fp contract(off)
  auto face = [](const double* w, double& wl, double& wr) {
    const double sl = minmod_rule(w[1] - w[0], w[2] - w[1]);
    const double sr = minmod_rule(w[2] - w[1], w[3] - w[2]);
    wl = w[1] + 0.5 * sl;
    wr = w[2] - 0.5 * sr;
  };
  double rL, rR, uL, uR, pL, pR, eL, eR;
  face(rho, rL, rR);
  face(un, uL, uR);
  face(p, pL, pR);
  face(er, eL, eR);
  const double cL = sqrt(gamma * pL / rL), cR = sqrt(gamma * pR / rR);
  const double sL = fabs(uL) + cL, sR = fabs(uR) + cR;
  const double sm = sL >= sR ? sL : sR;
  return 0.5 * (eL * uL + eR * uR) - 0.5 * sm * (eR - eL);
}

template <typename R, int STAGE>
__global__ __launch_bounds__(256) void rad_advect_walk(RadArgs a) {
#pragma clang fp contract(off)
  __shared__ double P[5][RW_LY][RW_LX];        // rho, u_x, u_y, p, E_r of one plane
  __shared__ double UZ[RW_TY][RW_TX];          // u_z of the plane's tile cells
  __shared__ double FX[RW_TY][RW_TX + 1];      // x faces of the plane's rows
  __shared__ double FY[RW_TY + 1][RW_TX];      // y faces of the plane's columns
  const int nx = a.n[0], ny = a.n[1], nz = a.n[2];
  const long long N = (long long)nx * ny * nz;
  const R* src = static_cast<const R*>(a.src);
  const unsigned tx = (nx + RW_TX - 1) / RW_TX, ty = (ny + RW_TY - 1) / RW_TY;
  const unsigned b = (unsigned)xcd_tile(blockIdx.x, gridDim.x);
  const unsigned bx = b % tx, rest = b / tx;
  const unsigned by = rest % ty, bz = rest / ty;
  const int x0 = (int)bx * RW_TX, y0 = (int)by * RW_TY;
  const int lx = threadIdx.x % RW_TX, ly = threadIdx.x / RW_TX;
  const int i = x0 + lx, j = y0 + ly;
  const bool own = i < nx && j < ny;
  const int z0 = (int)bz * RW_CZ, z1 = min(nz, z0 + RW_CZ);
  // z window of the own column: planes q-4 .. q when plane q has been loaded
  double wr_[5], wu[5], wp[5], we[5];
  // x and y part of L for the own cell of planes q-2, q-1, q
  double lxy[3] = {0.0, 0.0, 0.0};
  auto load_z = [&](int s, int kk) {
    if (!own) return;
    bool flip;
    const int kq = remap(kk, nz, a.bc[2][0], a.bc[2][1], flip);
    double w[6];
    rad_prims<R>(src, N, ((long long)kq * ny + j) * nx + i, a.gamma, flip ? 2 : -1, w);
    wr_[s] = w[0];
    wu[s] = w[3];
    wp[s] = w[4];
    we[s] = w[5];
  };
  // planes z0-4 .. z0-1 of the window (slots 0..3; z0-4 and z0-3 are never
  // read by a face of this chunk, but keep the slot arithmetic uniform)
#pragma unroll
  for (int s = 2; s < 4; ++s) load_z(s, z0 - 4 + s);
  unsigned flags = 0;
  double fz_lo = 0.0;  // z face below plane q-2, carried from the plane before
  for (int q = z0; q < z1 + 2; ++q) {
    if (q < z1) {
      // plane q: the tile and its halo (corners are not needed) into LDS, the
      // own column's (rho, u_z, p, E_r) into the window from there
      for (int t = threadIdx.x; t < RW_LX * RW_LY; t += 256) {
        const int px = t % RW_LX, py = t / RW_LX;
        const int gi = x0 - 2 + px, gj = y0 - 2 + py;
        const bool xin = gi >= 0 && gi < nx, yin = gj >= 0 && gj < ny;
        if (!xin && !yin) continue;
        bool fx = false, fy = false;
        const int qi = xin ? gi : remap(gi, nx, a.bc[0][0], a.bc[0][1], fx);
        const int qj = yin ? gj : remap(gj, ny, a.bc[1][0], a.bc[1][1], fy);
        double w[6];
        rad_prims<R>(src, N, ((long long)q * ny + qj) * nx + qi, a.gamma, fx ? 0 : (fy ? 1 : -1), w);
        P[0][py][px] = w[0];
        P[1][py][px] = w[1];
        P[2][py][px] = w[2];
        P[3][py][px] = w[4];
        P[4][py][px] = w[5];
        const int cx = px - 2, cy = py - 2;
        if (cx >= 0 && cx < RW_TX && cy >= 0 && cy < RW_TY) UZ[cy][cx] = w[3];
      }
      __syncthreads();
      if (own) {
        wr_[4] = P[0][ly + 2][lx + 2];
        wu[4] = UZ[ly][lx];
        wp[4] = P[3][ly + 2][lx + 2];
        we[4] = P[4][ly + 2][lx + 2];
      }
      // every x and y face of the plane once: x face f of row r lies between
      // tile cells f-1 and f (LDS cells f .. f+3), y face f of column c likewise
      for (int t = threadIdx.x; t < RW_TY * (RW_TX + 1) + (RW_TY + 1) * RW_TX; t += 256) {
        double rho[4], un[4], p[4], er[4];
        if (t < RW_TY * (RW_TX + 1)) {
          const int r = t / (RW_TX + 1), f = t % (RW_TX + 1);
#pragma unroll
          for (int s = 0; s < 4; ++s) {
            rho[s] = P[0][r + 2][f + s];
            un[s] = P[1][r + 2][f + s];
            p[s] = P[3][r + 2][f + s];
            er[s] = P[4][r + 2][f + s];
          }
          FX[r][f] = rad_face(rho, un, p, er, a.gamma);
        } else {
          const int u = t - RW_TY * (RW_TX + 1);
          const int f = u / RW_TX, cc = u % RW_TX;
#pragma unroll
          for (int s = 0; s < 4; ++s) {
            rho[s] = P[0][f + s][cc + 2];
            un[s] = P[2][f + s][cc + 2];
            p[s] = P[3][f + s][cc + 2];
            er[s] = P[4][f + s][cc + 2];
          }
          FY[f][cc] = rad_face(rho, un, p, er, a.gamma);
        }
      }
      __syncthreads();
      if (own) {
        double l = 0.0;
        {
          const double df = FX[ly][lx + 1] - FX[ly][lx];
          l = l - (a.dx_pow2 ? df * a.inv_dx[0] : df / a.dx[0]);
        }
        {
          const double df = FY[ly + 1][lx] - FY[ly][lx];
          l = l - (a.dx_pow2 ? df * a.inv_dx[1] : df / a.dx[1]);
        }
        lxy[2] = l;
      }
      // no barrier here: the next plane's loader writes only P and UZ, whose
      // last reads came before the barrier above, and FX and FY are written
      // again only after the loader's barrier, which every reader reaches
      // after its reads
    } else {
      // planes z1 and z1+1 close the window (the next chunk's, or ghosts)
      load_z(4, q);
    }
    // plane k = q-2 is complete: its z faces from planes k-2 .. k+2
    const int k = q - 2;
    if (own && k >= z0) {
      if (k == z0) fz_lo = rad_face(wr_, wu, wp, we, a.gamma);
      const double fz_hi = rad_face(wr_ + 1, wu + 1, wp + 1, we + 1, a.gamma);
      double l = lxy[0];
      {
        const double df = fz_hi - fz_lo;
        l = l - (a.dx_pow2 ? df * a.inv_dx[2] : df / a.dx[2]);
      }
      fz_lo = fz_hi;
      const long long c = ((long long)k * ny + j) * nx + i;
      R* dst = static_cast<R*>(a.dst);
      const R* un_ = static_cast<const R*>(a.un);
      const R ec = src[5 * N + c];
      const R dt = R(*a.dt);
      R out;
      if (STAGE == 1)
        out = ec + dt * R(l);
      else
        out = R(0.5) * (un_[5 * N + c] + (ec + dt * R(l)));
      dst[5 * N + c] = out;
      if (!isfinite(out)) flags = FLAG_NONFINITE;
    }
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      wr_[s] = wr_[s + 1];
      wu[s] = wu[s + 1];
      wp[s] = wp[s + 1];
      we[s] = we[s + 1];
    }
    lxy[0] = lxy[1];
    lxy[1] = lxy[2];
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

// Grid-stride over the cells with a bounded grid: the fused CFL step ends
// with one pair of atomics per workgroup, and a few thousand workgroups keep
// those from queueing on the control block.
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

template <typename R, int NDIM>
static void rad_advect_t(const RadArgs& a, int stage, dim3 grid, hipStream_t s) {
  if (stage == 1)
    hipLaunchKernelGGL((rad_advect<R, NDIM, 1>), grid, dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL((rad_advect<R, NDIM, 2>), grid, dim3(256), 0, s, a);
}

template <typename R>
static void rad_advect_walk_t(const RadArgs& a, int stage, hipStream_t s) {
  const unsigned tiles = (unsigned)(((a.n[0] + RW_TX - 1) / RW_TX) * ((a.n[1] + RW_TY - 1) / RW_TY) *
                                    ((a.n[2] + RW_CZ - 1) / RW_CZ));
  if (stage == 1)
    hipLaunchKernelGGL((rad_advect_walk<R, 1>), dim3(tiles), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL((rad_advect_walk<R, 2>), dim3(tiles), dim3(256), 0, s, a);
}

hipError_t launch_rad_advect(int ndim, int dtype, const RadArgs& a, int stage, hipStream_t s) {
  if (ndim == 3) {
    if (dtype == 0) rad_advect_walk_t<double>(a, stage, s);
    else rad_advect_walk_t<float>(a, stage, s);
    return hipGetLastError();
  }
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
