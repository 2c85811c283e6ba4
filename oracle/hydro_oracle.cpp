// Plain CPU oracle for the explicit finite-volume hydro step.
//
// TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
// benchmark's CPU-baseline leg may load this code.  It shares nothing with
// the HIP path: no headers, no helpers, no tables.
//
// What it computes (HARD paper, section 2.2.1 "Basic equations" and
// section 2.2.2 "Numerical algorithms"):
//   * conserved state U = (rho, rho*v_d, e + rho v^2/2) of the conservation law
//     d_t U + d_j F^j = 0 (paper equations "conservative form" and "fluxes",
//     hydro rows, radiation row and sources dropped);
//   * ideal-gas closure p = (gamma-1) e (the paper's "ideal EoS" of the
//     temperature-induced shock example, section 3.3);
//   * finite-volume flux difference on a uniform cell-centred Cartesian mesh
//     (section 2.2.2, the face-difference formula), summed over axes;
//   * face states by MUSCL with the minmod limiter on primitive variables,
//     face fluxes by the HLLC approximate Riemann solver (Toro, "Riemann
//     Solvers and Numerical Methods for Fluid Dynamics", 3rd ed., section 10.4,
//     Davis wave-speed estimates);
//   * optionally the radiation energy density E as one more conserved field
//     (section 2.2.1: the fourth row of the conservation law and its source):
//     advected with the fluid velocity through the local Lax-Friedrichs
//     (Rusanov) flux (section 2.2.2), and exchanged with the fluid internal
//     energy by the heating rate qdot = c kappa rho (E - a T^4) (equation
//     "heating-cooling"), integrated implicitly after each step; the
//     diffusion flux and the radiation pressure work are not part of it;
//   * or, as a second scheme, the paper's own choice (section 2.2.2): WENO5-Z
//     face states (Borges, Carmona, Costa and Don 2008) on primitive
//     variables with the HLL flux (Harten, Lax and van Leer 1983; Davis
//     speeds), which needs three ghost layers instead of two;
//   * Heun's two-stage Runge-Kutta step (paper table "Butcher tableau for
//     Heun's method") written in Shu-Osher form, which is the same method;
//   * the CFL time step dt = C / max_i sum_d (|u_d| + c)/dx_d (section 3.5
//     says only that dt comes from the CFL condition; this is the reading).
//
// Everything is a plain loop over cells in FP64.  OpenMP splits the cell
// loops; every cell is computed by one thread in a fixed order, so the result
// does not depend on the thread count.
//
// The scalar type is a template parameter: `double` gives the values, the
// forward-mode dual number `Dual` gives the exact directional derivative of
// the same discrete map (it follows the branch taken at the base point; at a
// tie min/max/minmod pass the derivative to their first argument and
// |x| uses sign(0) = +1).

#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <type_traits>
#include <vector>

namespace hard_oracle {

// ----------------------------------------------------------------------------
// Forward-mode dual number
// ----------------------------------------------------------------------------
struct Dual {
  double v, d;
  Dual() : v(0.0), d(0.0) {}
  Dual(double a) : v(a), d(0.0) {}  // NOLINT: constants promote implicitly
  Dual(double a, double b) : v(a), d(b) {}
};
inline Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
inline Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
inline Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
inline Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
inline Dual operator/(Dual a, Dual b) {
  double q = a.v / b.v;
  return Dual(q, (a.d - q * b.d) / b.v);
}
inline Dual sqrt(Dual a) {
  double s = std::sqrt(a.v);
  return Dual(s, a.d / (2.0 * s));
}
inline Dual fabs(Dual a) { return a.v >= 0.0 ? a : -a; }
inline bool operator<(Dual a, Dual b) { return a.v < b.v; }
inline bool operator<=(Dual a, Dual b) { return a.v <= b.v; }
inline bool operator>(Dual a, Dual b) { return a.v > b.v; }
inline bool operator>=(Dual a, Dual b) { return a.v >= b.v; }
inline double value(double a) { return a; }
inline double value(Dual a) { return a.v; }

// K directional derivatives carried at once: the rules of Dual applied to
// each derivative component (one evaluation of the values for K directions).
template <int K>
struct DualN {
  double v;
  double d[K];
  DualN() : v(0.0) {
    for (int k = 0; k < K; ++k) d[k] = 0.0;
  }
  DualN(double a) : v(a) {  // NOLINT: constants promote implicitly
    for (int k = 0; k < K; ++k) d[k] = 0.0;
  }
};
template <int K>
inline DualN<K> operator+(const DualN<K>& a, const DualN<K>& b) {
  DualN<K> r(a.v + b.v);
  for (int k = 0; k < K; ++k) r.d[k] = a.d[k] + b.d[k];
  return r;
}
template <int K>
inline DualN<K> operator-(const DualN<K>& a, const DualN<K>& b) {
  DualN<K> r(a.v - b.v);
  for (int k = 0; k < K; ++k) r.d[k] = a.d[k] - b.d[k];
  return r;
}
template <int K>
inline DualN<K> operator-(const DualN<K>& a) {
  DualN<K> r(-a.v);
  for (int k = 0; k < K; ++k) r.d[k] = -a.d[k];
  return r;
}
template <int K>
inline DualN<K> operator*(const DualN<K>& a, const DualN<K>& b) {
  DualN<K> r(a.v * b.v);
  for (int k = 0; k < K; ++k) r.d[k] = a.d[k] * b.v + a.v * b.d[k];
  return r;
}
template <int K>
inline DualN<K> operator/(const DualN<K>& a, const DualN<K>& b) {
  const double q = a.v / b.v;
  DualN<K> r(q);
  for (int k = 0; k < K; ++k) r.d[k] = (a.d[k] - q * b.d[k]) / b.v;
  return r;
}
template <int K>
inline DualN<K> sqrt(const DualN<K>& a) {
  const double s = std::sqrt(a.v);
  DualN<K> r(s);
  for (int k = 0; k < K; ++k) r.d[k] = a.d[k] / (2.0 * s);
  return r;
}
template <int K>
inline DualN<K> fabs(const DualN<K>& a) { return a.v >= 0.0 ? a : -a; }
template <int K>
inline bool operator<(const DualN<K>& a, const DualN<K>& b) { return a.v < b.v; }
template <int K>
inline bool operator<=(const DualN<K>& a, const DualN<K>& b) { return a.v <= b.v; }
template <int K>
inline bool operator>(const DualN<K>& a, const DualN<K>& b) { return a.v > b.v; }
template <int K>
inline bool operator>=(const DualN<K>& a, const DualN<K>& b) { return a.v >= b.v; }
template <int K>
inline double value(const DualN<K>& a) { return a.v; }

using std::fabs;
using std::sqrt;

// ----------------------------------------------------------------------------
// Branch-recording scalar: a double whose comparisons (every branch of the
// method: minmod picks, wave-speed min/max, the HLLC region, |x|) fold their
// outcomes into a running hash, so two inputs that take the same branches
// everywhere give the same signature.  The hash is a plain global, so
// recording runs use one thread.
// ----------------------------------------------------------------------------
static uint64_t g_sig;
inline bool sig_note(bool b) {
  g_sig = (g_sig ^ (b ? 0x9e3779b97f4a7c15ull : 0x7f4a7c159e3779b9ull)) * 0x100000001b3ull;
  return b;
}
struct Sig {
  double v;
  Sig() : v(0.0) {}
  Sig(double a) : v(a) {}  // NOLINT: constants promote implicitly
};
inline Sig operator+(Sig a, Sig b) { return Sig(a.v + b.v); }
inline Sig operator-(Sig a, Sig b) { return Sig(a.v - b.v); }
inline Sig operator-(Sig a) { return Sig(-a.v); }
inline Sig operator*(Sig a, Sig b) { return Sig(a.v * b.v); }
inline Sig operator/(Sig a, Sig b) { return Sig(a.v / b.v); }
inline Sig sqrt(Sig a) { return Sig(std::sqrt(a.v)); }
inline Sig fabs(Sig a) { return sig_note(a.v >= 0.0) ? a : -a; }
inline bool operator<(Sig a, Sig b) { return sig_note(a.v < b.v); }
inline bool operator<=(Sig a, Sig b) { return sig_note(a.v <= b.v); }
inline bool operator>(Sig a, Sig b) { return sig_note(a.v > b.v); }
inline bool operator>=(Sig a, Sig b) { return sig_note(a.v >= b.v); }
inline double value(Sig a) { return a.v; }

// ----------------------------------------------------------------------------
// Operation-counting scalar: a double that tallies the floating-point
// operations applied to it (for the algorithmic operation count per
// zone-update).  The tallies are plain globals, so counting runs use one
// thread.
// ----------------------------------------------------------------------------
struct OpTally {
  long long add, mul, div, sqrt, cmp, abs;
};
static OpTally g_ops;

struct Cnt {
  double v;
  Cnt() : v(0.0) {}
  Cnt(double a) : v(a) {}  // NOLINT: constants promote implicitly
};
inline Cnt operator+(Cnt a, Cnt b) { ++g_ops.add; return Cnt(a.v + b.v); }
inline Cnt operator-(Cnt a, Cnt b) { ++g_ops.add; return Cnt(a.v - b.v); }
inline Cnt operator-(Cnt a) { return Cnt(-a.v); }
inline Cnt operator*(Cnt a, Cnt b) { ++g_ops.mul; return Cnt(a.v * b.v); }
inline Cnt operator/(Cnt a, Cnt b) { ++g_ops.div; return Cnt(a.v / b.v); }
inline Cnt sqrt(Cnt a) { ++g_ops.sqrt; return Cnt(std::sqrt(a.v)); }
inline Cnt fabs(Cnt a) { ++g_ops.abs; return Cnt(std::fabs(a.v)); }
inline bool operator<(Cnt a, Cnt b) { ++g_ops.cmp; return a.v < b.v; }
inline bool operator<=(Cnt a, Cnt b) { ++g_ops.cmp; return a.v <= b.v; }
inline bool operator>(Cnt a, Cnt b) { ++g_ops.cmp; return a.v > b.v; }
inline bool operator>=(Cnt a, Cnt b) { ++g_ops.cmp; return a.v >= b.v; }
inline double value(Cnt a) { return a.v; }

// Status bits reported for a non-physical state.
enum : int { ST_RHO = 1, ST_PRES = 2, ST_NONFINITE = 4 };

enum : int { BC_PERIODIC = 0, BC_OUTFLOW = 1, BC_REFLECT = 2 };

enum : int { SCHEME_MUSCL_HLLC = 0, SCHEME_WENO5Z_HLL = 1 };

struct Grid {
  int ndim;       // 1, 2 or 3
  int nvar;       // ndim + 2 (+1 with radiation)
  int nh;         // hydro fields: ndim + 2
  int rad;        // 1: field nh is the radiation energy density E
  double kappa;   // opacity (cm^2/g), radiation only
  double mu;      // mean molecular weight, radiation only
  int64_t n[3];   // cells per axis; unused axes have n = 1
  double dx[3];   // cell width per axis
  double gamma;   // ratio of specific heats
  int bc[3][2];   // boundary kind per axis and side (0 = low, 1 = high)
  int64_t ncell;  // n[0]*n[1]*n[2]
  int scheme;     // SCHEME_MUSCL_HLLC or SCHEME_WENO5Z_HLL
  int ng;         // ghost layers per side: 2 (MUSCL) or 3 (WENO5-Z)

  // padded shape: axes below ndim get ng ghosts on each side
  int64_t pn[3];
  int64_t pcell;
};

static Grid make_grid(int ndim, const int64_t* n, const double* dx, double gamma,
                      const int* bc, int scheme, const double* radp) {
  Grid g;
  g.scheme = scheme;
  g.ng = scheme == SCHEME_WENO5Z_HLL ? 3 : 2;
  g.ndim = ndim;
  g.nh = ndim + 2;
  g.rad = radp != nullptr;
  g.kappa = radp ? radp[0] : 0.0;
  g.mu = radp ? radp[1] : 1.0;
  g.nvar = g.nh + g.rad;
  g.gamma = gamma;
  for (int d = 0; d < 3; ++d) {
    g.n[d] = d < ndim ? n[d] : 1;
    g.dx[d] = d < ndim ? dx[d] : 1.0;
    g.bc[d][0] = d < ndim ? bc[2 * d] : BC_PERIODIC;
    g.bc[d][1] = d < ndim ? bc[2 * d + 1] : BC_PERIODIC;
    g.pn[d] = d < ndim ? g.n[d] + 2 * g.ng : 1;
  }
  g.ncell = g.n[0] * g.n[1] * g.n[2];
  g.pcell = g.pn[0] * g.pn[1] * g.pn[2];
  return g;
}

// index of interior cell (i, j, k) in the unpadded array
static inline int64_t cidx(const Grid& g, int64_t i, int64_t j, int64_t k) {
  return (k * g.n[1] + j) * g.n[0] + i;
}
// index of cell (i, j, k), counted from the first interior cell, in the padded
// array (negative or >= n indices address ghosts)
static inline int64_t pidx(const Grid& g, int64_t i, int64_t j, int64_t k) {
  int64_t oi = i + (g.ndim > 0 ? g.ng : 0);
  int64_t oj = j + (g.ndim > 1 ? g.ng : 0);
  int64_t ok = k + (g.ndim > 2 ? g.ng : 0);
  return (ok * g.pn[1] + oj) * g.pn[0] + oi;
}

// Source interior index along one axis for ghost position q (q < 0 or q >= n,
// at most ng <= n cells out), and whether the normal momentum changes sign
// (reflecting wall).
static inline int64_t ghost_source(int64_t q, int64_t n, int bc_lo, int bc_hi, bool* flip) {
  *flip = false;
  if (q < 0) {
    int64_t k = -q;  // 1 .. ng
    if (bc_lo == BC_PERIODIC) return n - k;
    if (bc_lo == BC_OUTFLOW) return 0;
    *flip = true;
    return k - 1;
  }
  int64_t k = q - (n - 1);  // 1 .. ng
  if (bc_hi == BC_PERIODIC) return k - 1;
  if (bc_hi == BC_OUTFLOW) return n - 1;
  *flip = true;
  return n - k;
}

// ----------------------------------------------------------------------------
// Pieces of the method
// ----------------------------------------------------------------------------

// minmod(a, b): zero when the one-sided differences disagree in sign (or one
// is zero), otherwise the one of smaller magnitude; ties pick a.
template <class T>
static inline T minmod(T a, T b) {
  if (a * b <= T(0.0)) return T(0.0);
  if (fabs(a) <= fabs(b)) return a;
  return b;
}

// Primitive state seen by a face along the normal axis:
// rho, normal velocity un, transverse velocities ut[0..nt-1], pressure p.
template <class T>
struct Prim {
  T rho, un, ut[2], p;
};

// Physical flux F_K and conserved state U_K of one face state (normal axis
// first): F = (rho u, rho u^2 + p, rho u u_t, (E + p) u), U = (rho, rho u,
// rho u_t, E), with E the total energy density.
template <class T>
static void physical_flux(const Prim<T>& W, T E, int nt, T* FK, T* UK) {
  const int nv = nt + 3;
  T mn = W.rho * W.un;
  UK[0] = W.rho;
  UK[1] = mn;
  FK[0] = mn;
  FK[1] = mn * W.un + W.p;
  for (int t = 0; t < nt; ++t) {
    UK[2 + t] = W.rho * W.ut[t];
    FK[2 + t] = mn * W.ut[t];
  }
  UK[nv - 1] = E;
  FK[nv - 1] = (E + W.p) * W.un;
}

// HLLC flux for the normal direction (Toro section 10.4, Davis speeds).
// Output order: mass, normal momentum, transverse momenta, energy.
template <class T>
static void hllc_flux(const Prim<T>& L, const Prim<T>& R, int nt, double gamma, T* F) {
  const T g(gamma);
  const T gm1(gamma - 1.0);
  T cL = sqrt(g * L.p / L.rho);
  T cR = sqrt(g * R.p / R.rho);
  T qL = L.un * L.un;
  T qR = R.un * R.un;
  for (int t = 0; t < nt; ++t) {
    qL = qL + L.ut[t] * L.ut[t];
    qR = qR + R.ut[t] * R.ut[t];
  }
  T EL = L.p / gm1 + T(0.5) * L.rho * qL;
  T ER = R.p / gm1 + T(0.5) * R.rho * qR;

  // Davis estimates; min/max pass ties to their first argument
  T aL = L.un - cL, bL = R.un - cR;
  T SL = aL <= bL ? aL : bL;
  T aR = L.un + cL, bR = R.un + cR;
  T SR = aR >= bR ? aR : bR;

  // contact speed
  T num = R.p - L.p + L.rho * L.un * (SL - L.un) - R.rho * R.un * (SR - R.un);
  T den = L.rho * (SL - L.un) - R.rho * (SR - R.un);
  T Ss = num / den;

  const int nv = nt + 3;
  auto side = [&](const Prim<T>& W, T E, T* FK, T* UK) { physical_flux(W, E, nt, FK, UK); };
  // HLLC star state of one side:
  //   rho_K r [1, S*, v_K, w_K, E_K/rho_K + (S*-u_K)(S* + p_K/(rho_K (S_K-u_K)))]
  // with r = (S_K - u_K)/(S_K - S*); the energy entry is expanded as
  //   r E_K + r (S*-u_K) (rho_K S* + p_K/(S_K-u_K))
  // so that a stationary contact (u = 0, equal p) maps U_K to itself exactly.
  auto star = [&](const Prim<T>& W, T E, T S, T* Us) {
    T r = (S - W.un) / (S - Ss);
    T fac = W.rho * r;
    Us[0] = fac;
    Us[1] = fac * Ss;
    for (int t = 0; t < nt; ++t) Us[2 + t] = fac * W.ut[t];
    Us[nv - 1] = r * E + r * (Ss - W.un) * (W.rho * Ss + W.p / (S - W.un));
  };

  T FK[5], UK[5], Us[5];
  if (SL >= T(0.0)) {
    side(L, EL, FK, UK);
    for (int v = 0; v < nv; ++v) F[v] = FK[v];
  } else if (Ss >= T(0.0)) {
    side(L, EL, FK, UK);
    star(L, EL, SL, Us);
    for (int v = 0; v < nv; ++v) F[v] = FK[v] + SL * (Us[v] - UK[v]);
  } else if (SR > T(0.0)) {
    side(R, ER, FK, UK);
    star(R, ER, SR, Us);
    for (int v = 0; v < nv; ++v) F[v] = FK[v] + SR * (Us[v] - UK[v]);
  } else {
    side(R, ER, FK, UK);
    for (int v = 0; v < nv; ++v) F[v] = FK[v];
  }
}

// HLL flux (Harten, Lax and van Leer 1983) with the Davis wave speeds:
//   F_L if S_L >= 0;  F_R if S_R <= 0;  otherwise
//   (S_R F_L - S_L F_R + S_L S_R (U_R - U_L)) / (S_R - S_L).
template <class T>
static void hll_flux(const Prim<T>& L, const Prim<T>& R, int nt, double gamma, T* F) {
  const T g(gamma);
  const T gm1(gamma - 1.0);
  T cL = sqrt(g * L.p / L.rho);
  T cR = sqrt(g * R.p / R.rho);
  T qL = L.un * L.un;
  T qR = R.un * R.un;
  for (int t = 0; t < nt; ++t) {
    qL = qL + L.ut[t] * L.ut[t];
    qR = qR + R.ut[t] * R.ut[t];
  }
  T EL = L.p / gm1 + T(0.5) * L.rho * qL;
  T ER = R.p / gm1 + T(0.5) * R.rho * qR;
  T aL = L.un - cL, bL = R.un - cR;
  T SL = aL <= bL ? aL : bL;
  T aR = L.un + cL, bR = R.un + cR;
  T SR = aR >= bR ? aR : bR;
  const int nv = nt + 3;
  T FL[5], UL[5], FR[5], UR[5];
  physical_flux(L, EL, nt, FL, UL);
  physical_flux(R, ER, nt, FR, UR);
  if (SL >= T(0.0)) {
    for (int v = 0; v < nv; ++v) F[v] = FL[v];
  } else if (SR <= T(0.0)) {
    for (int v = 0; v < nv; ++v) F[v] = FR[v];
  } else {
    for (int v = 0; v < nv; ++v)
      F[v] = (SR * FL[v] - SL * FR[v] + SL * SR * (UR[v] - UL[v])) / (SR - SL);
  }
}

// Jiang-Shu smoothness indicators of the three candidate stencils of
// v[0..4]: beta_k = sum over l = 1, 2 of the integral over the middle cell of
// dx^(2l-1) (d^l p_k/dx^l)^2, p_k the quadratic with the stencil's three cell
// averages; in closed form 13/12 (second difference)^2 + 1/4 (first-order
// combination)^2.
template <class T>
static void weno5z_indicators(const T* v, T* beta) {
  T s0 = v[0] - T(2.0) * v[1] + v[2];
  T t0 = v[0] - T(4.0) * v[1] + T(3.0) * v[2];
  T s1 = v[1] - T(2.0) * v[2] + v[3];
  T t1 = v[1] - v[3];
  T s2 = v[2] - T(2.0) * v[3] + v[4];
  T t2 = T(3.0) * v[2] - T(4.0) * v[3] + v[4];
  const T c1(13.0 / 12.0), c2(0.25);
  beta[0] = c1 * s0 * s0 + c2 * t0 * t0;
  beta[1] = c1 * s1 * s1 + c2 * t1 * t1;
  beta[2] = c1 * s2 * s2 + c2 * t2 * t2;
}

// WENO5-Z value at the right face of the middle cell of v[0..4] (cells
// i-2 .. i+2), Borges et al. 2008: the three third-order candidate values on
// the stencils {i-2,i-1,i}, {i-1,i,i+1}, {i,i+1,i+2}; the Jiang-Shu
// smoothness indicators beta_k; tau5 = |beta_0 - beta_2|; the weights
// alpha_k = d_k (1 + tau5 / (beta_k + eps)) with the optimal weights
// d = (1/10, 6/10, 3/10) and eps = 1e-40; the value sum alpha_k q_k / sum alpha_k.
// The left face of cell i is the same function of the mirrored cells
// (i+2, i+1, i, i-1, i-2).
template <class T>
static T weno5z(const T* v) {
  // the three third-order candidate values
  T q0 = (T(2.0) * v[0] - T(7.0) * v[1] + T(11.0) * v[2]) / T(6.0);
  T q1 = (-v[1] + T(5.0) * v[2] + T(2.0) * v[3]) / T(6.0);
  T q2 = (T(2.0) * v[2] + T(5.0) * v[3] - v[4]) / T(6.0);
  T beta[3];
  weno5z_indicators(v, beta);
  T b0 = beta[0], b1 = beta[1], b2 = beta[2];
  const T eps(1e-40);
  // global smoothness measure and the unnormalised Z weights
  T tau = fabs(b0 - b2);
  T a0 = T(0.1) * (T(1.0) + tau / (b0 + eps));
  T a1 = T(0.6) * (T(1.0) + tau / (b1 + eps));
  T a2 = T(0.3) * (T(1.0) + tau / (b2 + eps));
  return (a0 * q0 + a1 * q1 + a2 * q2) / (a0 + a1 + a2);
}

// Primitive variables of one conserved state: rho, u_0..u_{ndim-1}, p.
// Returns status bits.
template <class T>
static int primitives(const T* u, int ndim, double gamma, T* w, int nextra = 0) {
  for (int x = 0; x < nextra; ++x) w[ndim + 2 + x] = u[ndim + 2 + x];
  T rho = u[0];
  T q = u[1] * u[1];
  for (int d = 1; d < ndim; ++d) q = q + u[1 + d] * u[1 + d];
  T ke = T(0.5) * q / rho;
  T e = u[ndim + 1] - ke;
  T p = T(gamma - 1.0) * e;
  w[0] = rho;
  for (int d = 0; d < ndim; ++d) w[1 + d] = u[1 + d] / rho;
  w[ndim + 1] = p;
  int st = 0;
  if (!(value(rho) > 0.0)) st |= ST_RHO;
  if (!(value(p) > 0.0)) st |= ST_PRES;
  for (int v = 0; v < ndim + 2 + nextra; ++v)
    if (!std::isfinite(value(u[v]))) st |= ST_NONFINITE;
  return st;
}

// Local Lax-Friedrichs (Rusanov) flux of the radiation energy density E
// advected with the normal fluid velocity: (E_L u_L + E_R u_R)/2 -
// s (E_R - E_L)/2, s = max(|u_L| + c_L, |u_R| + c_R), from the same face
// states as the hydro flux.
template <class T>
static T rusanov_E(const Prim<T>& L, const Prim<T>& R, T EL, T ER, double gamma) {
  const T g(gamma);
  T cL = sqrt(g * L.p / L.rho);
  T cR = sqrt(g * R.p / R.rho);
  T sL = fabs(L.un) + cL, sR = fabs(R.un) + cR;
  T s = sL >= sR ? sL : sR;
  return T(0.5) * (EL * L.un + ER * R.un) - T(0.5) * s * (ER - EL);
}

// Physical constants (CGS; CODATA 2018): speed of light, radiation constant
// a = 4 sigma / c, Boltzmann constant, atomic mass unit.
constexpr double C_LIGHT = 2.99792458e10;
constexpr double A_RAD = 4.0 * 5.670374419e-5 / 2.99792458e10;
constexpr double K_BOLTZ = 1.380649e-16;
constexpr double M_U = 1.66053906660e-24;

// Radiation-matter exchange of one cell over dt, backward Euler on
//   de/dt = qdot,  dE/dt = -qdot,  qdot = c kappa rho (E - a T^4),
// with T = e / C_v, C_v = rho k_B / (mu m_u (gamma - 1)) the ideal-gas heat
// capacity per volume.  e + E = W is conserved; with E' = (E + dt q a T'^4) /
// (1 + dt q), q = c kappa rho, the new temperature is the root of the
// increasing convex f(T) = C_v T + E'(T) - W, found by Newton iterations from
// an upper bound (so they decrease monotonically onto the root).  The
// kinetic energy is untouched: the total fluid energy changes by e' - e.
static void exchange(double rho, double ke, double& Ef, double& Er, double dt,
                     const Grid& g) {
  const double q = C_LIGHT * g.kappa * rho;
  const double dq = dt * q;
  if (!(dq > 0.0)) return;
  const double e = Ef - ke;
  const double Cv = rho * K_BOLTZ / (g.mu * M_U * (g.gamma - 1.0));
  const double W = e + Er;
  // upper bounds: all energy in the fluid; or none of it (C_v T dropped)
  const double t1 = W / Cv;
  const double t2 = std::sqrt(std::sqrt((W * (1.0 + dq) - Er) / (dq * A_RAD)));
  double T = t1 < t2 ? t1 : t2;
  for (int it = 0; it < 200; ++it) {
    const double T3 = T * T * T;
    const double f = Cv * T + (Er + dq * A_RAD * (T3 * T)) / (1.0 + dq) - W;
    const double fp = Cv + 4.0 * dq * A_RAD * T3 / (1.0 + dq);
    const double Tn = T - f / fp;
    if (!(Tn < T)) break;  // monotone from above: stop when it no longer decreases
    T = Tn;
  }
  const double e_new = Cv * T;
  Ef = Ef + (e_new - e);
  Er = W - e_new;
}

// ----------------------------------------------------------------------------
// L(U) = - sum_d (F_{d,i+1/2} - F_{d,i-1/2}) / dx_d
// ----------------------------------------------------------------------------
template <class T>
static int rhs(const Grid& g, const T* U, T* Lout) {
  const int nv = g.nvar;
  const int nd = g.ndim;
  const int64_t N = g.ncell, PN = g.pcell;

  // 1. ghost-padded conserved copy; corner ghosts stay NaN (never read by the
  //    star-shaped stencil, so a wrong read shows up as NaN)
  std::vector<T> G((size_t)nv * PN, T(std::numeric_limits<double>::quiet_NaN()));
#pragma omp parallel for schedule(static)
  for (int64_t c = 0; c < N; ++c) {
    int64_t i = c % g.n[0], j = (c / g.n[0]) % g.n[1], k = c / (g.n[0] * g.n[1]);
    for (int v = 0; v < nv; ++v) G[(size_t)v * PN + pidx(g, i, j, k)] = U[(size_t)v * N + c];
  }
  for (int d = 0; d < nd; ++d) {
    int64_t nd_ = g.n[d];
    // all cells interior in the other axes, ghost position along d
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < N / nd_; ++c) {
      int64_t o[3];
      int64_t rem = c;
      for (int a = 0; a < 3; ++a) {
        if (a == d) { o[a] = 0; continue; }
        o[a] = rem % g.n[a];
        rem /= g.n[a];
      }
      for (int side = 0; side < 2; ++side)
        for (int kk = 1; kk <= g.ng; ++kk) {
          int64_t q = side == 0 ? -kk : nd_ - 1 + kk;
          bool flip;
          int64_t s = ghost_source(q, nd_, g.bc[d][0], g.bc[d][1], &flip);
          int64_t dst[3] = {o[0], o[1], o[2]}, src[3] = {o[0], o[1], o[2]};
          dst[d] = q;
          src[d] = s;
          for (int v = 0; v < nv; ++v) {
            T val = U[(size_t)v * N + cidx(g, src[0], src[1], src[2])];
            if (flip && v == 1 + d) val = -val;
            G[(size_t)v * PN + pidx(g, dst[0], dst[1], dst[2])] = val;
          }
        }
    }
  }

  // 2. primitives over every padded cell (corners give NaN, unused)
  std::vector<T> W((size_t)nv * PN);
  int status = 0;
#pragma omp parallel for schedule(static) reduction(| : status)
  for (int64_t c = 0; c < PN; ++c) {
    T u[6], w[6];
    for (int v = 0; v < nv; ++v) u[v] = G[(size_t)v * PN + c];
    int st = primitives(u, nd, g.gamma, w, g.rad);
    for (int v = 0; v < nv; ++v) W[(size_t)v * PN + c] = w[v];
    // validity is judged on interior cells only (ghosts are copies of them)
    int64_t i = c % g.pn[0], j = (c / g.pn[0]) % g.pn[1], k = c / (g.pn[0] * g.pn[1]);
    bool interior = true;
    int64_t ii[3] = {i, j, k};
    for (int a = 0; a < nd; ++a)
      if (ii[a] < g.ng || ii[a] >= g.ng + g.n[a]) interior = false;
    if (interior) status |= st;
  }

  for (int64_t x = 0; x < (int64_t)nv * N; ++x) Lout[x] = T(0.0);

  // 3. faces along each axis in the order x, y, z
  for (int d = 0; d < nd; ++d) {
    int64_t nf = g.n[d] + 1;  // faces i-1/2 for i = 0..n
    int64_t nother = N / g.n[d];
    std::vector<T> F((size_t)nv * nf * nother);
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < nother; ++c) {
      int64_t o[3];
      int64_t rem = c;
      for (int a = 0; a < 3; ++a) {
        if (a == d) { o[a] = 0; continue; }
        o[a] = rem % g.n[a];
        rem /= g.n[a];
      }
      const int ns = 2 * g.ng;  // stencil cells f-ng .. f+ng-1
      for (int64_t f = 0; f < nf; ++f) {
        // face between cells f-1 and f along d
        T Wst[6][6];
        for (int s = 0; s < ns; ++s) {
          int64_t p[3] = {o[0], o[1], o[2]};
          p[d] = f - g.ng + s;
          int64_t pi = pidx(g, p[0], p[1], p[2]);
          for (int v = 0; v < nv; ++v) Wst[s][v] = W[(size_t)v * PN + pi];
        }
        T WL[6], WR[6];
        if (g.scheme == SCHEME_MUSCL_HLLC) {
          // Wc[0..3] = cells f-2 .. f+1
          T (*Wc)[6] = Wst;
          for (int v = 0; v < nv; ++v) {
            T sl = minmod(Wc[1][v] - Wc[0][v], Wc[2][v] - Wc[1][v]);  // slope of cell f-1
            T sr = minmod(Wc[2][v] - Wc[1][v], Wc[3][v] - Wc[2][v]);  // slope of cell f
            WL[v] = Wc[1][v] + T(0.5) * sl;
            WR[v] = Wc[2][v] - T(0.5) * sr;
          }
        } else {
          // Wst[0..5] = cells f-3 .. f+2: the right face of cell f-1 from
          // cells f-3..f+1, the left face of cell f from f+2..f-2 (mirrored)
          for (int v = 0; v < nv; ++v) {
            T a[5] = {Wst[0][v], Wst[1][v], Wst[2][v], Wst[3][v], Wst[4][v]};
            T b[5] = {Wst[5][v], Wst[4][v], Wst[3][v], Wst[2][v], Wst[1][v]};
            WL[v] = weno5z(a);
            WR[v] = weno5z(b);
          }
        }
        // rotate: normal velocity is axis d, transverse are the others in order
        Prim<T> PL, PR;
        PL.rho = WL[0];
        PR.rho = WR[0];
        PL.un = WL[1 + d];
        PR.un = WR[1 + d];
        int t = 0;
        for (int a = 0; a < nd; ++a) {
          if (a == d) continue;
          PL.ut[t] = WL[1 + a];
          PR.ut[t] = WR[1 + a];
          ++t;
        }
        PL.p = WL[nd + 1];
        PR.p = WR[nd + 1];
        T Fn[6];
        if (g.scheme == SCHEME_MUSCL_HLLC)
          hllc_flux(PL, PR, nd - 1, g.gamma, Fn);
        else
          hll_flux(PL, PR, nd - 1, g.gamma, Fn);
        // rotate back to (mass, m_0.., energy)
        T Fo[6];
        Fo[0] = Fn[0];
        Fo[1 + d] = Fn[1];
        t = 0;
        for (int a = 0; a < nd; ++a) {
          if (a == d) continue;
          Fo[1 + a] = Fn[2 + t];
          ++t;
        }
        Fo[nd + 1] = Fn[nd + 1];
        if (g.rad) Fo[g.nh] = rusanov_E(PL, PR, WL[g.nh], WR[g.nh], g.gamma);
        for (int v = 0; v < nv; ++v) F[((size_t)v * nother + c) * nf + f] = Fo[v];
      }
    }
    // divergence contribution of axis d
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < N; ++c) {
      int64_t ii[3] = {c % g.n[0], (c / g.n[0]) % g.n[1], c / (g.n[0] * g.n[1])};
      // index of this cell's row among the "other" cells
      int64_t oc = 0, mul = 1;
      for (int a = 0; a < 3; ++a) {
        if (a == d) continue;
        oc += ii[a] * mul;
        mul *= g.n[a];
      }
      int64_t f = ii[d];
      for (int v = 0; v < nv; ++v) {
        T Fm = F[((size_t)v * nother + oc) * nf + f];
        T Fp = F[((size_t)v * nother + oc) * nf + f + 1];
        Lout[(size_t)v * N + c] = Lout[(size_t)v * N + c] - (Fp - Fm) / T(g.dx[d]);
      }
    }
  }
  return status;
}

// One SSP-RK2 (Heun) step, same dt in both stages:
//   U1 = U + dt L(U);   U_new = 0.5 (U + (U1 + dt L(U1)))
template <class T>
static int step(const Grid& g, T* U, T dt) {
  const int64_t M = (int64_t)g.nvar * g.ncell;
  std::vector<T> L(M), U1(M);
  int st = rhs(g, U, L.data());
#pragma omp parallel for schedule(static)
  for (int64_t x = 0; x < M; ++x) U1[x] = U[x] + dt * L[x];
  st |= rhs(g, U1.data(), L.data());
#pragma omp parallel for schedule(static)
  for (int64_t x = 0; x < M; ++x) U[x] = T(0.5) * (U[x] + (U1[x] + dt * L[x]));
  if constexpr (std::is_same<T, double>::value) {
    if (g.rad) {
      const int nd = g.ndim;
      const int64_t N = g.ncell;
#pragma omp parallel for schedule(static)
      for (int64_t c = 0; c < N; ++c) {
        const double rho = U[c];
        double q = U[N + c] * U[N + c];
        for (int d = 1; d < nd; ++d)
          q = q + U[(size_t)(1 + d) * N + c] * U[(size_t)(1 + d) * N + c];
        const double ke = 0.5 * q / rho;
        exchange(rho, ke, U[(size_t)(nd + 1) * N + c], U[(size_t)(nd + 2) * N + c], value(dt), g);
      }
    }
  }
  return st;
}

// Largest signal speed sum over the interior: max_i sum_d (|u_d| + c)/dx_d
template <class T>
static double max_signal(const Grid& g, const T* U, int* status) {
  const int nv = g.nvar, nd = g.ndim;
  const int64_t N = g.ncell;
  double smax = 0.0;
  int st = 0;
#pragma omp parallel for schedule(static) reduction(max : smax) reduction(| : st)
  for (int64_t c = 0; c < N; ++c) {
    T u[6], w[6];
    for (int v = 0; v < nv; ++v) u[v] = U[(size_t)v * N + c];
    st |= primitives(u, nd, g.gamma, w, g.rad);
    T cs = sqrt(T(g.gamma) * w[nd + 1] / w[0]);
    T s(0.0);
    for (int d = 0; d < nd; ++d) s = s + (fabs(w[1 + d]) + cs) / T(g.dx[d]);
    if (value(s) > smax) smax = value(s);
  }
  *status = st;
  return smax;
}

}  // namespace hard_oracle

// ----------------------------------------------------------------------------
// C entry points (called from Python through ctypes)
// ----------------------------------------------------------------------------
using namespace hard_oracle;

// The K-direction tangent of nsteps steps (oracle_steps_tangent_multi).
template <int K>
static int steps_tangent_multi(const Grid& g, int64_t nsteps, const double* dts, double* U,
                               double* dU) {
  const int64_t M = (int64_t)g.nvar * g.ncell;
  std::vector<DualN<K>> X(M);
  for (int64_t x = 0; x < M; ++x) {
    X[x].v = U[x];
    for (int k = 0; k < K; ++k) X[x].d[k] = dU[k * M + x];
  }
  int st = 0;
  for (int64_t s = 0; s < nsteps; ++s) st |= step<DualN<K>>(g, X.data(), DualN<K>(dts[s]));
  for (int64_t x = 0; x < M; ++x) {
    U[x] = X[x].v;
    for (int k = 0; k < K; ++k) dU[k * M + x] = X[x].d[k];
  }
  return st;
}

extern "C" {

// L(U) for one state; returns status bits.
int oracle_rhs(int ndim, const int64_t* n, const double* dx, double gamma, const int* bc,
               int scheme, const double* radp,
               const double* U, double* L) {
  Grid g = make_grid(ndim, n, dx, gamma, bc, scheme, radp);
  return rhs<double>(g, U, L);
}

// One SSP-RK2 step in place; returns status bits.
int oracle_step(int ndim, const int64_t* n, const double* dx, double gamma, const int* bc,
                int scheme, const double* radp,
                double dt, double* U) {
  Grid g = make_grid(ndim, n, dx, gamma, bc, scheme, radp);
  return step<double>(g, U, dt);
}

// nsteps SSP-RK2 steps in place with the given dt list; returns OR of status.
int oracle_steps_fixed(int ndim, const int64_t* n, const double* dx, double gamma, const int* bc,
                       int scheme, const double* radp,
                       int64_t nsteps, const double* dts, double* U) {
  Grid g = make_grid(ndim, n, dx, gamma, bc, scheme, radp);
  int st = 0;
  for (int64_t s = 0; s < nsteps; ++s) st |= step<double>(g, U, dts[s]);
  return st;
}

// dt = cfl / max signal sum; writes the status bits of the state.
double oracle_cfl_dt(int ndim, const int64_t* n, const double* dx, double gamma, const int* bc,
                     int scheme, const double* radp,
                     double cfl, const double* U, int* status) {
  Grid g = make_grid(ndim, n, dx, gamma, bc, scheme, radp);
  double smax = max_signal(g, U, status);
  return cfl / smax;
}

// CFL-driven run to t_end: dt <- min(cfl dt, t_end - t); stops when
// t >= t_end (1 - 1e-14) or after max_steps.  Records each dt used if
// dts_out is not null (capacity max_steps).  Returns OR of status bits.
int oracle_run(int ndim, const int64_t* n, const double* dx, double gamma, const int* bc,
               int scheme, const double* radp,
               double cfl, double t_end, int64_t max_steps, double* U, double* t_out,
               int64_t* nsteps_out, double* dts_out) {
  Grid g = make_grid(ndim, n, dx, gamma, bc, scheme, radp);
  double t = 0.0;
  int64_t s = 0;
  int st = 0;
  while (t < t_end * (1.0 - 1e-14) && s < max_steps) {
    int st_dt = 0;
    double dt = cfl / max_signal(g, U, &st_dt);
    st |= st_dt;
    if (dt > t_end - t) dt = t_end - t;
    st |= step<double>(g, U, dt);
    if (dts_out) dts_out[s] = dt;
    t = t + dt;
    ++s;
  }
  *t_out = t;
  *nsteps_out = s;
  return st;
}

// Forward-mode derivative of nsteps steps with a frozen dt list:
// (U, dU) -> (U_n, dU_n) in place.  Returns OR of status bits.
int oracle_steps_tangent(int ndim, const int64_t* n, const double* dx, double gamma,
                         const int* bc, int scheme, const double* radp, int64_t nsteps,
                         const double* dts, double* U, double* dU) {
  Grid g = make_grid(ndim, n, dx, gamma, bc, scheme, radp);
  const int64_t M = (int64_t)g.nvar * g.ncell;
  std::vector<Dual> X(M);
  for (int64_t x = 0; x < M; ++x) X[x] = Dual(U[x], dU[x]);
  int st = 0;
  for (int64_t s = 0; s < nsteps; ++s) st |= step<Dual>(g, X.data(), Dual(dts[s]));
  for (int64_t x = 0; x < M; ++x) {
    U[x] = X[x].v;
    dU[x] = X[x].d;
  }
  return st;
}

// K directional derivatives of nsteps steps at once (K = 1, 2, 4 or 8): dU
// holds K state-shaped directions one after another and receives the
// derivatives.
int oracle_steps_tangent_multi(int ndim, const int64_t* n, const double* dx, double gamma,
                               const int* bc, int scheme, const double* radp, int64_t nsteps,
                               const double* dts, int ndir, double* U, double* dU) {
  Grid g = make_grid(ndim, n, dx, gamma, bc, scheme, radp);
  switch (ndir) {
    case 1: return steps_tangent_multi<1>(g, nsteps, dts, U, dU);
    case 2: return steps_tangent_multi<2>(g, nsteps, dts, U, dU);
    case 4: return steps_tangent_multi<4>(g, nsteps, dts, U, dU);
    case 8: return steps_tangent_multi<8>(g, nsteps, dts, U, dU);
    default: return -1;
  }
}

// HLLC flux for one face: WL, WR = (rho, un, ut[0..nt-1], p); F gets
// (mass, normal momentum, transverse momenta, energy).
void oracle_hllc(int nt, double gamma, const double* WL, const double* WR, double* F) {
  Prim<double> L, R;
  L.rho = WL[0];
  L.un = WL[1];
  R.rho = WR[0];
  R.un = WR[1];
  for (int t = 0; t < nt; ++t) {
    L.ut[t] = WL[2 + t];
    R.ut[t] = WR[2 + t];
  }
  L.p = WL[2 + nt];
  R.p = WR[2 + nt];
  hllc_flux(L, R, nt, gamma, F);
}

double oracle_minmod(double a, double b) { return minmod<double>(a, b); }

// HLL flux for one face (same layout as oracle_hllc).
void oracle_hll(int nt, double gamma, const double* WL, const double* WR, double* F) {
  Prim<double> L, R;
  L.rho = WL[0];
  L.un = WL[1];
  R.rho = WR[0];
  R.un = WR[1];
  for (int t = 0; t < nt; ++t) {
    L.ut[t] = WL[2 + t];
    R.ut[t] = WR[2 + t];
  }
  L.p = WL[2 + nt];
  R.p = WR[2 + nt];
  hll_flux(L, R, nt, gamma, F);
}

// WENO5-Z value at the right face of the middle cell of v[0..4].
double oracle_weno5z(const double* v) { return weno5z<double>(v); }

// The three smoothness indicators beta_k of v[0..4].
void oracle_weno5z_indicators(const double* v, double* beta) { weno5z_indicators<double>(v, beta); }

// Floating-point operations of one CFL dt plus one SSP-RK2 step of U (left
// unchanged), tallied by kind: out[0..5] = add/sub, mul, div, sqrt, compare,
// abs.  Runs on one thread.
void oracle_count_ops(int ndim, const int64_t* n, const double* dx, double gamma, const int* bc,
                      int scheme, const double* radp,
                      double dt, const double* U, int64_t* out);

#ifdef _OPENMP
#include <omp.h>
int oracle_threads(void) { return omp_get_max_threads(); }
#else
int oracle_threads(void) { return 1; }
static void omp_set_num_threads(int) {}
static int omp_get_max_threads(void) { return 1; }
#endif
// Threads of the OpenMP loops from now on (results do not depend on it).
void oracle_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }

// Branch signature of nsteps steps from U with the step sizes dts: a hash of
// the outcome of every comparison the method makes, in evaluation order (one
// thread).  U is left unchanged.
uint64_t oracle_branch_signature(int ndim, const int64_t* n, const double* dx, double gamma,
                                 const int* bc, int scheme, const double* radp, int64_t nsteps,
                                 const double* dts, const double* U) {
  Grid g = make_grid(ndim, n, dx, gamma, bc, scheme, radp);
  const int64_t M = (int64_t)g.nvar * g.ncell;
  std::vector<Sig> X(M);
  for (int64_t x = 0; x < M; ++x) X[x] = Sig(U[x]);
  const int threads = omp_get_max_threads();
  omp_set_num_threads(1);
  g_sig = 0xcbf29ce484222325ull;
  for (int64_t s = 0; s < nsteps; ++s) (void)step<Sig>(g, X.data(), Sig(dts[s]));
  omp_set_num_threads(threads);
  return g_sig;
}

void oracle_count_ops(int ndim, const int64_t* n, const double* dx, double gamma, const int* bc,
                      int scheme, const double* radp,
                      double dt, const double* U, int64_t* out) {
  Grid g = make_grid(ndim, n, dx, gamma, bc, scheme, radp);
  const int64_t M = (int64_t)g.nvar * g.ncell;
  std::vector<Cnt> X(M);
  for (int64_t x = 0; x < M; ++x) X[x] = Cnt(U[x]);
  const int threads = omp_get_max_threads();
  omp_set_num_threads(1);
  g_ops = OpTally{0, 0, 0, 0, 0, 0};
  int st = 0;
  (void)max_signal(g, X.data(), &st);
  (void)step<Cnt>(g, X.data(), Cnt(dt));
  omp_set_num_threads(threads);
  out[0] = g_ops.add;
  out[1] = g_ops.mul;
  out[2] = g_ops.div;
  out[3] = g_ops.sqrt;
  out[4] = g_ops.cmp;
  out[5] = g_ops.abs;
}

}  // extern "C"
