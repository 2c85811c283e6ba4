// Device-side building blocks of the hydro step for gfx950.
//
// Primitive recovery with the ideal-gas closure, the minmod-limited MUSCL
// face states and the HLLC flux (HARD paper section 2.2.1 for the equations,
// section 2.2.2 for the finite-volume face difference; HLLC after Toro,
// "Riemann Solvers and Numerical Methods for Fluid Dynamics", section 10.4,
// with Davis wave-speed estimates).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hard {

enum { BC_PERIODIC = 0, BC_OUTFLOW = 1, BC_REFLECT = 2 };
enum : unsigned { FLAG_DENSITY = 1u, FLAG_PRESSURE = 2u, FLAG_NONFINITE = 4u, FLAG_RADIATION = 8u };

// Workspace control block (first 256 bytes of every workspace).
struct Control {
  unsigned long long reserved0;
  unsigned int reserved1;
  unsigned int flags;            // status bits (FLAG_*)
  double t;                      // simulated time (hard_run)
  long long steps;               // steps taken (hard_run)
  int done;                      // hard_run reached t_end or max_steps
  int pad;
  double dt;                     // step size slot (hard_run)
  unsigned long long aux[26];
};
static_assert(sizeof(Control) == 256, "control block is 256 bytes");

// Index along one axis of n cells for a (possibly ghost) position q.
// Periodic wraps, outflow copies the edge cell, reflecting mirrors and sets
// `flip` (normal momentum changes sign).  Positions further out than the two
// ghost layers occur only in the overhang of ragged tiles; they are clamped
// into range and their values never reach an interior result.
__device__ __forceinline__ int remap(int q, int n, int bclo, int bchi, bool& flip) {
  flip = false;
  if (q < 0) {
    if (bclo == BC_PERIODIC) return q + n >= 0 ? q + n : 0;
    if (bclo == BC_OUTFLOW) return 0;
    flip = true;
    int s = -q - 1;
    return s < n ? s : n - 1;
  }
  if (q >= n) {
    if (bchi == BC_PERIODIC) return q - n < n ? q - n : n - 1;
    if (bchi == BC_OUTFLOW) return n - 1;
    flip = true;
    int s = 2 * n - 1 - q;
    return s >= 0 ? s : 0;
  }
  return q;
}

// minmod(a, b): 0 if a and b differ in sign (or one is 0), else the argument
// of smaller magnitude -- which is the median of a, b and 0 (up to the sign
// of a zero result): max(min(a, b), min(max(a, b), 0)), no compares or
// selects; one v_med3 in float.
template <typename R>
__device__ __forceinline__ R minmod(R a, R b) {
  return fmax(fmin(a, b), fmin(fmax(a, b), R(0)));
}
template <>
__device__ __forceinline__ float minmod<float>(float a, float b) {
  return __builtin_amdgcn_fmed3f(a, b, 0.0f);
}

// Reciprocal and square root.  FP64: the hardware v_rcp_f64 / v_rsq_f64
// seeds (relative error about 5e-8 on gfx950) refined by Newton steps; each
// step squares the error.  FP32: the hardware instructions (about 1 ulp).
// The CFL sum keeps IEEE division and square root.
//   fast_rcp   two steps, within about 1 ulp: primitive recovery (1/rho).
//   flux_rcp   one step, within about 1e-14: the two quotients of the HLLC
//              flux (S* and the star factor q).
//   sound_speed  one step, within about 1e-14.
// The flux tolerances are far below the 1e-12 parity bar and cost a third
// of the instructions of the IEEE sequences.
__device__ __forceinline__ double fast_rcp(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}
__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }

__device__ __forceinline__ double flux_rcp(double x) {
  double r = __builtin_amdgcn_rcp(x);
  return fma(r, fma(-x, r, 1.0), r);
}
__device__ __forceinline__ float flux_rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// c = sqrt(gp / rho) = gp * rsq(gp * rho): one reciprocal square root
// instead of a reciprocal and a square root.
__device__ __forceinline__ double sound_speed(double gp, double rho) {
  double x = gp * rho;
  double y = __builtin_amdgcn_rsq(x);
  // one Newton step for 1/sqrt(x): y <- y (3 - x y^2) / 2
  double h = 0.5 * x;
  y = y * fma(-h * y, y, 1.5);
  return gp * y;
}
__device__ __forceinline__ float sound_speed(float gp, float rho) {
  return gp * __builtin_amdgcn_rsqf(gp * rho);
}

// Pressure from conserved values.  The internal energy E - |m|^2/(2 rho) is
// a difference of nearly equal numbers near vacuum and in fast flow, so for
// float storage it is recovered in double.
template <int NDIM>
__device__ __forceinline__ double pressure_f64(const double* U, double inv_rho, double gm1) {
  double q = U[1] * U[1];
#pragma unroll
  for (int d = 1; d < NDIM; ++d) q = q + U[1 + d] * U[1 + d];
  return gm1 * (U[NDIM + 1] - 0.5 * q * inv_rho);
}
// float storage: E - |m|^2/(2 rho) in double (the float inputs are exact in double)
template <int NDIM>
__device__ __forceinline__ float pressure_f32(const float* U, double inv_rho, double gm1) {
  double q = (double)U[1] * (double)U[1];
#pragma unroll
  for (int d = 1; d < NDIM; ++d) q = q + (double)U[1 + d] * (double)U[1 + d];
  double e = (double)U[NDIM + 1] - 0.5 * q * inv_rho;
  return (float)(gm1 * e);
}

// Conserved (rho, m_d, E) -> primitive (rho, u_d, p), in place in W.
template <typename R, int NDIM>
__device__ __forceinline__ void to_primitive(const R* U, R* W, double gm1);

template <int NDIM>
__device__ __forceinline__ void to_primitive_f64(const double* U, double* W, double gm1) {
  double inv = fast_rcp(U[0]);
  W[0] = U[0];
#pragma unroll
  for (int d = 0; d < NDIM; ++d) W[1 + d] = U[1 + d] * inv;
  W[NDIM + 1] = pressure_f64<NDIM>(U, inv, gm1);
}
template <int NDIM>
__device__ __forceinline__ void to_primitive_f32(const float* U, float* W, double gm1) {
  double inv = fast_rcp((double)U[0]);
  float invf = (float)inv;
  W[0] = U[0];
#pragma unroll
  for (int d = 0; d < NDIM; ++d) W[1 + d] = U[1 + d] * invf;
  W[NDIM + 1] = pressure_f32<NDIM>(U, inv, gm1);
}
template <>
__device__ __forceinline__ void to_primitive<double, 1>(const double* U, double* W, double g) { to_primitive_f64<1>(U, W, g); }
template <>
__device__ __forceinline__ void to_primitive<double, 2>(const double* U, double* W, double g) { to_primitive_f64<2>(U, W, g); }
template <>
__device__ __forceinline__ void to_primitive<double, 3>(const double* U, double* W, double g) { to_primitive_f64<3>(U, W, g); }
template <>
__device__ __forceinline__ void to_primitive<float, 1>(const float* U, float* W, double g) { to_primitive_f32<1>(U, W, g); }
template <>
__device__ __forceinline__ void to_primitive<float, 2>(const float* U, float* W, double g) { to_primitive_f32<2>(U, W, g); }
template <>
__device__ __forceinline__ void to_primitive<float, 3>(const float* U, float* W, double g) { to_primitive_f32<3>(U, W, g); }

// Status bits of one interior cell from its conserved values and pressure.
template <typename R, int NV>
__device__ __forceinline__ unsigned cell_flags(const R* U, R p) {
  unsigned f = 0;
  if (!(U[0] > R(0))) f |= FLAG_DENSITY;
  if (!(p > R(0))) f |= FLAG_PRESSURE;
  bool fin = true;
#pragma unroll
  for (int v = 0; v < NV; ++v) fin = fin && isfinite(U[v]);
  if (!fin) f |= FLAG_NONFINITE;
  return f;
}

// HLLC flux across a face whose normal velocity is un; NT transverse
// velocities ut.  Output: mass, normal momentum, NT transverse momenta, energy.
// Only the side selected by the wave pattern is evaluated:
//   S_L >= 0         -> F_L
//   S_L < 0 <= S*    -> F_L + S_L (U*_L - U_L)
//   S* < 0 < S_R     -> F_R + S_R (U*_R - U_R)
//   S_R <= 0         -> F_R
// With q = (S* - u_K)/(S_K - S*) (so that (S_K - u_K)/(S_K - S*) = 1 + q), the
// jumps U*_K - U_K of the star state are formed directly:
//   mass              rho q
//   normal momentum   rho (S* - u_K + q S*)
//   transverse        rho q ut
//   energy            q (E + p + rho (S_K - u_K) S*)
// which is Toro's star state rearranged: one reciprocal per face for q (plus
// one for S*), and q = 0 exactly at a stationary contact (S* = u_K), where
// the flux reduces to the physical flux.
template <typename R, int NT>
__device__ __forceinline__ void hllc(R rL, R unL, const R* utL, R pL, R rR, R unR, const R* utR,
                                     R pR, R gam, R inv_gm1, R* F) {
  R cL = sound_speed(gam * pL, rL);
  R cR = sound_speed(gam * pR, rR);
  R aL = unL - cL, bL = unR - cR;
  R SL = (aL <= bL) ? aL : bL;
  R aR = unL + cL, bR = unR + cR;
  R SR = (aR >= bR) ? aR : bR;
  R dL = SL - unL, dR = SR - unR;
  R mL = rL * dL, mR = rR * dR;  // rho_K (S_K - u_K)
  R Ss = (pR - pL + mL * unL - mR * unR) * flux_rcp(mL - mR);

  // pick the side
  bool left = (SL >= R(0)) || (Ss >= R(0));
  bool star = left ? !(SL >= R(0)) : (SR > R(0));
  R r = left ? rL : rR;
  R un = left ? unL : unR;
  R p = left ? pL : pR;
  R S = left ? SL : SR;
  R d = left ? dL : dR;
  R ut[NT > 0 ? NT : 1];
  R k2 = un * un;
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    ut[t] = left ? utL[t] : utR[t];
    k2 = k2 + ut[t] * ut[t];
  }
  R Ep = p * inv_gm1 + R(0.5) * r * k2 + p;  // E + p

  // star jump factors; outside the star regions they are 0, which leaves
  // the physical flux (S_K - S* may vanish there, so q is masked, not used)
  R g = Ss - un;
  R q = g * flux_rcp(S - Ss);
  g = star ? g : R(0);
  q = star ? q : R(0);
  R mn = r * un;
  R Sr = S * r;
  R F0 = mn + Sr * q;
  F[0] = F0;
  F[1] = (mn * un + p) + Sr * (g + q * Ss);
#pragma unroll
  for (int t = 0; t < NT; ++t) F[2 + t] = ut[t] * F0;
  F[NT + 2] = Ep * un + (S * q) * (Ep + r * d * Ss);
}

// Rusanov (local Lax-Friedrichs) flux of the radiation energy density E_r at
// a face, from the face states in face order (rho, u_n, u_t..., p, E_r):
// the mean of E_r u_n on the two sides minus half the larger signal speed
// |u_n| + c of the two hydro face states times the jump of E_r.
template <typename R, int NH>
__device__ __forceinline__ R rusanov_er(const R* A, const R* B, R gam) {
  const R cL = sound_speed(gam * A[NH - 1], A[0]);
  const R cR = sound_speed(gam * B[NH - 1], B[0]);
  const R sL = fabs(A[1]) + cL, sR = fabs(B[1]) + cR;
  const R sm = sL >= sR ? sL : sR;
  return R(0.5) * (A[NH] * A[1] + B[NH] * B[1]) - R(0.5) * sm * (B[NH] - A[NH]);
}

// MUSCL-minmod face states from four cell states along the face normal
// (cells i-1, i | i+1, i+2 around face i+1/2 are w0, w1 | w2, w3).
template <typename R>
__device__ __forceinline__ void muscl_pair(R w0, R w1, R w2, R w3, R& wl, R& wr) {
  R d01 = w1 - w0, d12 = w2 - w1, d23 = w3 - w2;
  R sl = minmod(d01, d12);
  R sr = minmod(d12, d23);
  wl = w1 + R(0.5) * sl;
  wr = w2 - R(0.5) * sr;
}

// HLLC flux from primitive face states already ordered (rho, u_n, u_t..., p);
// output (mass, normal momentum, transverse momenta, energy).
template <typename R, int NV>
__device__ __forceinline__ void hllc_ordered(const R* WL, const R* WR, R gam, R inv_gm1, R* F) {
  constexpr int NT = NV - 3;
  R utL[NT > 0 ? NT : 1], utR[NT > 0 ? NT : 1];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    utL[t] = WL[2 + t];
    utR[t] = WR[2 + t];
  }
  hllc<R, NT>(WL[0], WL[1], utL, WL[NV - 1], WR[0], WR[1], utR, WR[NV - 1], gam, inv_gm1, F);
}

// Heating and cooling of the radiation field (section 2.2.1, the heating
// rate qdot = c kappa rho (E_r - a T^4)) over one step: backward Euler for the
// fluid temperature, solved by Newton iterations from an upper bound; plain
// IEEE arithmetic, so the iteration count and result are those of a plain
// evaluation.  CGS constants (CODATA 2018): speed of light, radiation
// constant a = 4 sigma/c, Boltzmann constant, atomic mass unit.
constexpr double RC_LIGHT = 2.99792458e10;
constexpr double RA_RAD = 4.0 * 5.670374419e-5 / 2.99792458e10;
constexpr double RK_B = 1.380649e-16;
constexpr double RM_U = 1.66053906660e-24;

// Backward-Euler exchange of one cell; returns the new (E_fluid, E_r).
// e + E_r is conserved; the kinetic energy is untouched.
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

// The exchange applied to one new cell state U (conserved, as stored,
// E_r in field NDIM + 2): in double on the stored values, the kinetic energy
// from the momenta; changed energies are rounded back to R.  Returns the
// status bits (non-finite energies).
template <typename R, int NDIM>
__device__ __forceinline__ unsigned exchange_cell(R* U, double dt, double gamma, double kappa,
                                                  double mu) {
#pragma clang fp contract(off)
  constexpr int NH = NDIM + 2;
  const double rho = (double)U[0];
  double m2 = 0.0;
#pragma unroll
  for (int k = 0; k < NDIM; ++k) {
    const double m = (double)U[1 + k];
    m2 = k == 0 ? m * m : m2 + m * m;
  }
  const double ke = 0.5 * m2 / rho;
  double Ef = (double)U[NH - 1], Er = (double)U[NH];
  const double Ef0 = Ef, Er0 = Er;
  exchange(rho, ke, Ef, Er, dt, gamma, kappa, mu);
  if (Ef != Ef0) U[NH - 1] = R(Ef);
  if (Er != Er0) U[NH] = R(Er);
  return (!isfinite(Er) || !isfinite(Ef)) ? FLAG_NONFINITE : 0u;
}

// Wave64 reductions
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ unsigned wave_or(unsigned v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v |= __shfl_xor(v, o, 64);
  return v;
}

// Map hardware block id to a logical tile id so that the blocks one XCD
// receives (the dispatcher deals blocks round-robin over the 8 XCDs) form one
// contiguous run of logical tiles, which share halos through that XCD's L2.
__device__ __forceinline__ int xcd_tile(int b, int nb) {
  const int nx = 8;
  int xcd = b % nx, slot = b / nx;
  int per = nb / nx, rem = nb % nx;
  return xcd * per + (xcd < rem ? xcd : rem) + slot;
}

// The CFL signal sum sum_d (|u_d| + c)/dx_d of one conserved state stored as
// R (FP64 or FP32 storage, the sum in double), with the refined reciprocal
// of rho and the refined reciprocal square root: within a few ulp of the
// plain IEEE evaluation for a third of its FP64 instructions.
template <typename R, int NDIM>
__device__ __forceinline__ double cfl_signal(const double* U, const double* inv_dx, double gamma) {
  const double inv = fast_rcp(U[0]);
  double q = U[1] * U[1];
#pragma unroll
  for (int d = 1; d < NDIM; ++d) q = q + U[1 + d] * U[1 + d];
  const double gp = gamma * ((gamma - 1.0) * (U[NDIM + 1] - 0.5 * q * inv));
  const double cs = sound_speed(gp, U[0]);
  double s = 0.0;
#pragma unroll
  for (int d = 0; d < NDIM; ++d) s = s + (fabs(U[1 + d]) * inv + cs) * inv_dx[d];
  return s;
}

// Block-wide: OR of status flags (one atomic per block, only when a bit is
// set) and the max of the CFL signal sums of the block, stored to the
// block's own slot (a plain store: same-address device-scope atomics from
// thousands of workgroups serialise, about 55 ns each on gfx950).  The dt
// itself comes from cfl_final_kernel over all slots, launched after the
// kernel.  Must be called by every thread.
template <int NTHREADS>
__device__ __forceinline__ void block_finish(unsigned flags, double smax, bool do_cfl,
                                             Control* ctl, double* slot) {
  constexpr int NW = NTHREADS / 64;
  __shared__ double red_s[NW];
  __shared__ unsigned red_f[NW];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  flags = wave_or(flags);
  if (do_cfl) smax = wave_max(smax);
  if (lane == 0) {
    red_f[w] = flags;
    red_s[w] = smax;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned f = 0;
    double s = 0.0;
    for (int i = 0; i < NW; ++i) {
      f |= red_f[i];
      s = fmax(s, red_s[i]);
    }
    if (f) atomicOr(&ctl->flags, f);
    if (do_cfl) *slot = s;
  }
}

}  // namespace hard
