// Adjoint (vector-Jacobian product) of one Heun step with dt held fixed.
//
// Forward map (HARD paper section 2.2.2: face-difference formula, Heun's
// Butcher tableau in Shu-Osher form):
//     U1 = U + dt L(U),   U' = (U + (U1 + dt L(U1))) / 2.
// Given lam = dJ/dU', the chain rule gives
//     lam1 = lam/2 + (dL/dU1)^T (dt lam/2)          (= dJ/dU1)
//     lam0 = lam/2 + lam1 + (dL/dU)^T (dt lam1)      (= dJ/dU).
// (dL/dX)^T mu is evaluated face by face: each face flux F_f enters
// L_{f-1} with -1/dx and L_f with +1/dx, so its adjoint is
// Fbar_f = (mu_f - mu_{f-1})/dx; Fbar_f is pulled back through HLLC and the
// MUSCL-minmod face states to the primitive states of the four stencil cells
// (kernel adj_face), the contributions are summed per cell in a fixed order,
// ghost contributions folded into their source cells (adj_gather), and the
// primitive adjoint is mapped to conserved variables (adj_final).
//
// Branches: the derivative is that of the branch taken at X (minmod picks,
// min/max of the wave speeds with ties to the first argument, the HLLC
// region).  To take the same branches as a plain evaluation of the formulas
// when values sit on a tie (for instance the pressure slopes of an exactly
// uniform pressure field, whose recovered values differ only by rounding),
// this recomputation evaluates primitives, face states and wave speeds with
// IEEE division and square root, no contraction, in the order of the
// formulas.  The value kernels use faster equivalent arithmetic.

#include <cmath>
#include <cstring>

#include "../../include/hard.h"
#include "api_internal.hpp"
#include "hydro_device.hpp"
#include "launch.hpp"

namespace hard {

struct AdjGeo {
  int n[3];
  int bc[3][2];
  double inv_dx[3];
  double gamma;
};

// Plain-formula primitive state of a conserved state (rho, u_d, p).
template <int NDIM>
__device__ __forceinline__ void prim_plain(const double* u, double gamma, double* w) {
#pragma clang fp contract(off)
  double rho = u[0];
  double q = u[1] * u[1];
#pragma unroll
  for (int d = 1; d < NDIM; ++d) q = q + u[1 + d] * u[1 + d];
  double ke = 0.5 * q / rho;
  double e = u[NDIM + 1] - ke;
  double p = (gamma - 1.0) * e;
  w[0] = rho;
#pragma unroll
  for (int d = 0; d < NDIM; ++d) w[1 + d] = u[1 + d] / rho;
  w[NDIM + 1] = p;
}

__device__ __forceinline__ double minmod_plain(double a, double b, int& pick) {
  // pick: 0 = zero, 1 = a, 2 = b
  if (a * b <= 0.0) {
    pick = 0;
    return 0.0;
  }
  if (fabs(a) <= fabs(b)) {
    pick = 1;
    return a;
  }
  pick = 2;
  return b;
}

// HLLC value and its vector-Jacobian product for one face (normal order:
// rho, u_n, u_t..., p in; mass, normal momentum, transverse momenta, energy
// out).  Given Fb (adjoint of the flux), returns WLb, WRb.
template <int NT>
__device__ __forceinline__ void hllc_vjp(const double* WL, const double* WR, double gamma,
                                         const double* Fb, double* WLb, double* WRb) {
#pragma clang fp contract(off)
  constexpr int NV = NT + 3;
  const double g = gamma, gm1 = gamma - 1.0;
  const double rL = WL[0], uL = WL[1], pL = WL[NV - 1];
  const double rR = WR[0], uR = WR[1], pR = WR[NV - 1];
  const double cL = sqrt(g * pL / rL);
  const double cR = sqrt(g * pR / rR);
  const double aL = uL - cL, bL = uR - cR;
  const bool pickL = aL <= bL;
  const double SL = pickL ? aL : bL;
  const double aR = uL + cL, bR = uR + cR;
  const bool pickR = aR >= bR;
  const double SR = pickR ? aR : bR;
  const double dLp = SL - uL, dRp = SR - uR;
  const double num = pR - pL + rL * uL * dLp - rR * uR * dRp;
  const double den = rL * dLp - rR * dRp;
  const double Ss = num / den;

  int region;
  if (SL >= 0.0) region = 0;
  else if (Ss >= 0.0) region = 1;
  else if (SR > 0.0) region = 2;
  else region = 3;
  const bool left = region <= 1;
  const bool star = region == 1 || region == 2;
  const double* W = left ? WL : WR;
  const double r = W[0], u = W[1], p = W[NV - 1];
  double v[NT > 0 ? NT : 1];
  double q = u * u;
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    v[t] = W[2 + t];
    q = q + v[t] * v[t];
  }
  const double igm1 = 1.0 / gm1;
  const double E = p * igm1 + 0.5 * r * q;
  const double S = left ? SL : SR;
  const double mn = r * u;

  // accumulators of the selected side and of the shared quantities
  double rb = 0, ub = 0, pb = 0, Eb = 0, Sb = 0, Ssb = 0, db = 0;
  double vb[NT > 0 ? NT : 1];
#pragma unroll
  for (int t = 0; t < NT; ++t) vb[t] = 0;

  // F = FK (+ S (U* - UK) in the star regions)
  double mnb = Fb[0];
  mnb += Fb[1] * u;
  ub += Fb[1] * mn;
  pb += Fb[1];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    mnb += Fb[2 + t] * v[t];
    vb[t] += Fb[2 + t] * mn;
  }
  Eb += Fb[NV - 1] * u;
  pb += Fb[NV - 1] * u;
  ub += Fb[NV - 1] * (E + p);
  rb += mnb * u;
  ub += mnb * r;

  if (star) {
    // the reverse sweep makes no branch decision: it uses reciprocals formed
    // once (within an ulp of the divisions they replace)
    const double d = S - u;
    const double id = 1.0 / d, iS = 1.0 / (S - Ss);
    const double rr = d * iS;
    const double fac = r * rr;
    const double X = r * Ss + p * id;
    double US[NV], UK[NV];
    US[0] = fac;
    US[1] = fac * Ss;
    UK[0] = r;
    UK[1] = r * u;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      US[2 + t] = fac * v[t];
      UK[2 + t] = r * v[t];
    }
    US[NV - 1] = rr * E + rr * (Ss - u) * X;
    UK[NV - 1] = E;
#pragma unroll
    for (int k = 0; k < NV; ++k) Sb += Fb[k] * (US[k] - UK[k]);
    // U*: adjoint S Fb
    const double USb0 = S * Fb[0], USb1 = S * Fb[1], USbE = S * Fb[NV - 1];
    double facb = USb0 + USb1 * Ss;
    Ssb += USb1 * fac;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const double USbt = S * Fb[2 + t];
      facb += USbt * v[t];
      vb[t] += USbt * fac;
    }
    double rrb = USbE * (E + (Ss - u) * X);
    Eb += USbE * rr;
    const double Xb = USbE * rr * (Ss - u);
    Ssb += USbE * rr * X;
    ub -= USbE * rr * X;
    rb += Xb * Ss;
    Ssb += Xb * r;
    pb += Xb * id;
    db -= Xb * p * id * id;
    rb += facb * rr;
    rrb += facb * r;
    db += rrb * iS;
    const double tS = -rrb * d * iS * iS;
    Sb += tS;
    Ssb -= tS;
    // UK: adjoint -S Fb
    rb -= S * Fb[0];
    rb -= S * Fb[1] * u;
    ub -= S * Fb[1] * r;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      rb -= S * Fb[2 + t] * v[t];
      vb[t] -= S * Fb[2 + t] * r;
    }
    Eb -= S * Fb[NV - 1];
    // d = S - u
    Sb += db;
    ub -= db;
  }
  // E = p/(gamma-1) + r q / 2
  pb += Eb * igm1;
  rb += Eb * 0.5 * q;
  const double qb = Eb * 0.5 * r;
  ub += 2.0 * u * qb;
#pragma unroll
  for (int t = 0; t < NT; ++t) vb[t] += 2.0 * v[t] * qb;

  // side-K adjoints into L or R
  double rLb = 0, uLb = 0, pLb = 0, rRb = 0, uRb = 0, pRb = 0, SLb = 0, SRb = 0;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    WLb[k] = 0;
    WRb[k] = 0;
  }
  if (left) {
    rLb += rb; uLb += ub; pLb += pb; SLb += Sb;
#pragma unroll
    for (int t = 0; t < NT; ++t) WLb[2 + t] += vb[t];
  } else {
    rRb += rb; uRb += ub; pRb += pb; SRb += Sb;
#pragma unroll
    for (int t = 0; t < NT; ++t) WRb[2 + t] += vb[t];
  }
  // S* = num / den
  const double iden = 1.0 / den;
  const double numb = Ssb * iden;
  const double denb = -Ssb * Ss * iden;
  pRb += numb;
  pLb -= numb;
  rLb += numb * uL * dLp;
  uLb += numb * rL * dLp;
  double dLpb = numb * rL * uL;
  rRb -= numb * uR * dRp;
  uRb -= numb * rR * dRp;
  double dRpb = -numb * rR * uR;
  rLb += denb * dLp;
  dLpb += denb * rL;
  rRb -= denb * dRp;
  dRpb -= denb * rR;
  SLb += dLpb;
  uLb -= dLpb;
  SRb += dRpb;
  uRb -= dRpb;
  // S_L = min(uL - cL, uR - cR), S_R = max(uL + cL, uR + cR)
  double cLb = 0, cRb = 0;
  if (pickL) { uLb += SLb; cLb -= SLb; } else { uRb += SLb; cRb -= SLb; }
  if (pickR) { uLb += SRb; cLb += SRb; } else { uRb += SRb; cRb += SRb; }
  // c = sqrt(g p / r)
  // dc/dp = g / (2 c r), dc/dr = -c / (2 r) (c^2 = g p / r)
  const double hL = cLb / (2.0 * cL * rL), hR = cRb / (2.0 * cR * rR);
  pLb += hL * g;
  rLb -= hL * cL * cL;
  pRb += hR * g;
  rRb -= hR * cR * cR;
  WLb[0] += rLb;
  WLb[1] += uLb;
  WLb[NV - 1] += pLb;
  WRb[0] += rRb;
  WRb[1] += uRb;
  WRb[NV - 1] += pRb;
}

// Contributions of the flux adjoint of one face along `axis` to the
// primitive adjoints of its four stencil cells f-2 .. f+1 (primitive order,
// before any ghost fold): Cb[s][v] for cell f - 2 + s.  (cx, cy, cz) is a
// cell of the face's line (its coordinate along `axis` is not used); the
// flux adjoint is Fbar = scale (mu_f - mu_{f-1}) / dx, zero outside the
// interior.
template <int NDIM, int axis>
__device__ __forceinline__ void face_vjp(const double* __restrict__ X,
                                         const double* __restrict__ mu, double scale,
                                         const AdjGeo& g, int cx, int cy, int cz, int f,
                                         double (&Cb)[4][NDIM + 2]) {
  constexpr int NV = NDIM + 2;
  const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
  const long long N = (long long)nx * ny * nz;
  const int nd = g.n[axis];
  auto cell = [&](int q, bool& flip) -> long long {
    int c[3] = {cx, cy, cz};
    c[axis] = remap(q, nd, g.bc[axis][0], g.bc[axis][1], flip);
    return ((long long)c[2] * ny + c[1]) * nx + c[0];
  };
  // stencil primitives, cells f-2 .. f+1
  double W[4][NV];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    bool fl;
    long long ci = cell(f - 2 + s, fl);
    double u[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) u[v] = X[v * N + ci];
    prim_plain<NDIM>(u, g.gamma, W[s]);
    if (fl) W[s][1 + axis] = -W[s][1 + axis];
  }
  // face states (plain formula) and the minmod picks
  double WL[NV], WR[NV];
  int pl[NV], pr[NV];
  {
#pragma clang fp contract(off)
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      double sl = minmod_plain(W[1][v] - W[0][v], W[2][v] - W[1][v], pl[v]);
      double sr = minmod_plain(W[2][v] - W[1][v], W[3][v] - W[2][v], pr[v]);
      WL[v] = W[1][v] + 0.5 * sl;
      WR[v] = W[2][v] - 0.5 * sr;
    }
  }
  // flux adjoint: Fbar = scale (mu_f - mu_{f-1}) / dx (zero outside the interior)
  double Fb[NV];
  {
    bool fl;
    long long cr = cell(f, fl), cm = cell(f - 1, fl);
    const bool hasR = f < nd, hasL = f >= 1;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      double mr = hasR ? mu[v * N + cr] : 0.0;
      double ml = hasL ? mu[v * N + cm] : 0.0;
      Fb[v] = scale * (mr - ml) * g.inv_dx[axis];
    }
  }
  // rotate to the face's normal order (rho, u_n, u_t ascending, p)
  constexpr int t0 = axis == 0 ? 2 : 1;          // first transverse velocity slot
  constexpr int t1 = axis == 2 ? 2 : 3;          // second (3D only)
  constexpr int perm[5] = {0, 1 + axis, NDIM >= 2 ? t0 : NV - 1, NDIM == 3 ? t1 : NV - 1, NV - 1};
  double A[NV], B[NV], Fn[NV], Ab[NV], Bb[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    A[k] = WL[perm[k]];
    B[k] = WR[perm[k]];
    Fn[k] = Fb[perm[k]];
  }
  hllc_vjp<NDIM - 1>(A, B, g.gamma, Fn, Ab, Bb);
  double WLb[NV], WRb[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    WLb[perm[k]] = Ab[k];
    WRb[perm[k]] = Bb[k];
  }
  // face states -> stencil cells
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    Cb[0][v] = 0;
    Cb[1][v] = WLb[v];
    Cb[2][v] = WRb[v];
    Cb[3][v] = 0;
    const double slb = 0.5 * WLb[v];
    if (pl[v] == 1) { Cb[1][v] += slb; Cb[0][v] -= slb; }
    else if (pl[v] == 2) { Cb[2][v] += slb; Cb[1][v] -= slb; }
    const double srb = -0.5 * WRb[v];
    if (pr[v] == 1) { Cb[2][v] += srb; Cb[1][v] -= srb; }
    else if (pr[v] == 2) { Cb[3][v] += srb; Cb[2][v] -= srb; }
  }
}

// One face along `axis` per thread: its stencil contributions written to
// C[slot][var][face] (faces numbered x fastest) for adj_gather.
template <int NDIM, int axis>
__global__ __launch_bounds__(256) void adj_face(const double* __restrict__ X,
                                                const double* __restrict__ mu,
                                                const double* __restrict__ dt_dev, double factor,
                                                AdjGeo g, double* __restrict__ C) {
  constexpr int NV = NDIM + 2;
  const double scale = factor * *dt_dev;
  const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
  // faces form a grid of n + 1 positions along `axis` and n along the others,
  // x fastest (so that neighbouring threads touch neighbouring cells)
  const int m0 = nx + (axis == 0), m1 = ny + (axis == 1);
  const long long NF = (long long)m0 * m1 * (nz + (axis == 2));
  const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= NF) return;
  int c0[3];
  c0[0] = (int)(id % m0);
  c0[1] = (int)((id / m0) % m1);
  c0[2] = (int)(id / ((long long)m0 * m1));
  double Cb[4][NV];
  face_vjp<NDIM, axis>(X, mu, scale, g, c0[0], c0[1], c0[2], c0[axis], Cb);
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int v = 0; v < NV; ++v) C[(s * NV + v) * NF + id] = Cb[s][v];
}

// Per cell: sum the contributions of every face stencil that reads it along
// `axis`, directly or through a ghost whose source it is (normal velocity
// adjoint negated across a reflecting wall), in a fixed order.
template <int NDIM>
__global__ __launch_bounds__(256) void adj_gather(AdjGeo g, int axis, const double* __restrict__ C,
                                                  double* __restrict__ Wb, int accumulate) {
  constexpr int NV = NDIM + 2;
  const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
  const long long N = (long long)nx * ny * nz;
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= N) return;
  const int x = (int)(c % nx), y = (int)((c / nx) % ny), z = (int)(c / ((long long)nx * ny));
  const int nd = g.n[axis];
  const int j = axis == 0 ? x : (axis == 1 ? y : z);
  // the face grid of `axis` (see adj_face): index of face position f on this
  // cell's line, f = 0 .. nd
  const int m0 = nx + (axis == 0), m1 = ny + (axis == 1);
  const long long NF = (long long)m0 * m1 * (nz + (axis == 2));
  const long long fstride = axis == 0 ? 1 : (axis == 1 ? (long long)m0 : (long long)m0 * m1);
  const long long fbase = ((long long)z * m1 + y) * m0 + x - (long long)j * fstride;
  double acc[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) acc[v] = 0.0;
  const int qs[5] = {j, -2, -1, nd, nd + 1};
  for (int k = 0; k < 5; ++k) {
    const int q = qs[k];
    bool flip = false;
    if (k > 0) {
      int src = remap(q, nd, g.bc[axis][0], g.bc[axis][1], flip);
      if (src != j) continue;
    }
    const int f0 = q - 1 > 0 ? q - 1 : 0;
    const int f1 = q + 2 < nd ? q + 2 : nd;
    for (int f = f0; f <= f1; ++f) {
      const double* in = C + (long long)(q - f + 2) * NV * NF + fbase + f * fstride;
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        double val = in[v * NF];
        if (flip && v == 1 + axis) val = -val;
        acc[v] += val;
      }
    }
  }
#pragma unroll
  for (int v = 0; v < NV; ++v) Wb[v * N + c] = accumulate ? Wb[v * N + c] + acc[v] : acc[v];
}

// Conserved adjoint (dW/dU)^T wb of the primitive adjoint wb at the state u.
template <int NDIM>
__device__ __forceinline__ void prim_to_cons_adjoint(const double* u, const double* wb,
                                                     double gamma, double* ub) {
  constexpr int NV = NDIM + 2;
  // derivatives only (no branch depends on them): one reciprocal of rho
  const double rho = u[0], gm1 = gamma - 1.0;
  const double ir = 1.0 / rho, ir2 = ir * ir;
  double q = 0.0;
#pragma unroll
  for (int d = 0; d < NDIM; ++d) q += u[1 + d] * u[1 + d];
  ub[0] = wb[0] + wb[NV - 1] * gm1 * 0.5 * q * ir2;
#pragma unroll
  for (int d = 0; d < NDIM; ++d) {
    ub[0] -= wb[1 + d] * u[1 + d] * ir2;
    ub[1 + d] = wb[1 + d] * ir - wb[NV - 1] * gm1 * u[1 + d] * ir;
  }
  ub[NV - 1] = wb[NV - 1] * gm1;
}

// out = c0 lam + c1 lam1 + (dW/dU)^T Wb at X (lam1 may be NULL).
template <int NDIM>
__global__ __launch_bounds__(256) void adj_final(const double* __restrict__ X,
                                                 const double* __restrict__ Wb, double gamma,
                                                 long long N, const double* lam, double c0,
                                                 const double* lam1, double c1, double* out) {
  constexpr int NV = NDIM + 2;
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= N) return;
  double u[NV], wb[NV], ub[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    u[v] = X[v * N + c];
    wb[v] = Wb[v * N + c];
  }
  prim_to_cons_adjoint<NDIM>(u, wb, gamma, ub);
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    double r = c0 * lam[v * N + c] + ub[v];
    if (lam1) r += c1 * lam1[v * N + c];
    out[v * N + c] = r;
  }
}

// ---------------------------------------------------------------------------
// The whole product in one launch for 1D and 2D grids (adj_tile): one
// workgroup per tile of TX x TY cells
//   out = c0 lam + c1 lam1 + (dW/dU)^T (dL/dX)^T (factor dt mu)   at X.
// It computes every face whose stencil reaches a cell of the tile (TX + 3
// per row and axis, plus the up to four faces at the far end of a line
// whose ghost cells fold into the tile), one face per thread and batch, and
// adds each face's four stencil contributions to per-cell accumulators in
// LDS in eight rounds (axis, face index mod 4): faces of one round touch
// distinct cells.  Contributions to ghost positions are kept per (ghost,
// face) pair and folded into their source cells afterwards, in the order
// q = -2, -1, n, n + 1 (faces ascending), the normal velocity negated
// across a reflecting wall.  No face array goes through memory.
// ---------------------------------------------------------------------------
template <int NDIM>
struct AdjTileShape;
template <>
struct AdjTileShape<1> {
  static constexpr int TX = 256, TY = 1;
};
template <>
struct AdjTileShape<2> {
  static constexpr int TX = 16, TY = 16;
};

// The six (ghost position, face) pairs of a line: (-2, 0), (-1, 0), (-1, 1),
// (n, n-1), (n, n), (n+1, n); pair_of() maps a face and a ghost stencil slot
// to its pair.
__device__ __forceinline__ int pair_q(int k, int nd) {
  return k == 0 ? -2 : (k <= 2 ? -1 : (k <= 4 ? nd : nd + 1));
}
__device__ __forceinline__ int pair_f(int k, int nd) {
  return k <= 1 ? 0 : (k == 2 ? 1 : (k == 3 ? nd - 1 : nd));
}
__device__ __forceinline__ int pair_of(int q, int f, int nd) {
  if (q == -2) return 0;
  if (q == -1) return f == 0 ? 1 : 2;
  if (q == nd) return f == nd - 1 ? 3 : 4;
  return 5;
}

template <int NDIM>
__global__ __launch_bounds__(256) void adj_tile(const double* __restrict__ X,
                                                const double* __restrict__ mu,
                                                const double* __restrict__ dt_dev, double factor,
                                                AdjGeo g, const double* lam, double c0,
                                                const double* lam1, double c1, double* out) {
  constexpr int NV = NDIM + 2;
  constexpr int TX = AdjTileShape<NDIM>::TX, TY = AdjTileShape<NDIM>::TY;
  // own faces t0 - 1 .. t0 + T + 1 of every line, x items then y items, then
  // the far-end faces (four per line and axis), which only tiles at a grid
  // edge iterate.  Each region starts on a wave boundary, so that no wave
  // computes faces of both axes (the two face routines would run one after
  // the other) and interior tiles issue no lane for a far-end slot.
  constexpr int OX = TX + 3, OY = TY + 3;
  constexpr int NOX = TY * OX, NOY = NDIM == 2 ? TX * OY : 0;
  constexpr int NOXP = (NOX + 63) / 64 * 64;
  constexpr int NOWN = NOXP + NOY;
  constexpr int FAR0 = (NOWN + 63) / 64 * 64;
  constexpr int NFX = TY * 4, NFXP = (NFX + 63) / 64 * 64, NFY = NDIM == 2 ? TX * 4 : 0;
  constexpr int NI = FAR0 + NFXP + NFY;
  constexpr int NL = NDIM == 1 ? 1 : (TX > TY ? TX : TY);  // lines per axis, at most
  __shared__ double acc[NV][TY][TX];
  __shared__ double gbuf[NDIM][NL][6][NV];
  const int tid = threadIdx.x;
  const int nx = g.n[0], ny = g.n[1];
  const long long N = (long long)nx * ny;
  const int tiles_x = (nx + TX - 1) / TX;
  const int x0 = (int)(blockIdx.x % tiles_x) * TX, y0 = (int)(blockIdx.x / tiles_x) * TY;
  const double scale = factor * *dt_dev;
  const int lx = tid % TX, ly = tid / TX;         // this thread's cell (TX * TY == 256)
#pragma unroll
  for (int v = 0; v < NV; ++v) acc[v][ly][lx] = 0.0;
  __syncthreads();

  // the face of item i: axis, line (row y or column x of the tile), face index
  // f along the axis; false if the item carries no face
  auto item = [&](int i, int& ax, int& line, int& f, bool& own) -> bool {
    int slot;
    if (i < FAR0) {
      if (i < NOXP) {
        if (i >= NOX) return false;
        ax = 0; line = i / OX; slot = i % OX;
      } else {
        const int k = i - NOXP;
        if (k >= NOY) return false;
        ax = 1; line = k % TX; slot = k / TX;
      }
    } else if (i < FAR0 + NFXP) {
      const int k = i - FAR0;
      if (k >= NFX) return false;
      ax = 0; line = k / 4; slot = OX + k % 4;
    } else {
      const int k = i - FAR0 - NFXP;
      if (k >= NFY) return false;
      ax = 1; line = k % TX; slot = OY + k / TX;
    }
    int t0, T, nd, nother, origin_other;
    if (ax == 0) {
      t0 = x0; T = TX; nd = nx; nother = ny; origin_other = y0;
    } else {
      t0 = y0; T = TY; nd = ny; nother = nx; origin_other = x0;
    }
    if (origin_other + line >= nother) return false;
    const int t1 = t0 + T < nd ? t0 + T : nd;       // tile cells [t0, t1) along the axis
    const int fa = t0 - 1 > 0 ? t0 - 1 : 0, fb = t1 + 1 < nd ? t1 + 1 : nd;
    if (slot < T + 3) {
      f = t0 - 1 + slot;
      own = true;
      return f >= fa && f <= fb;
    }
    // far-end faces whose ghost contributions fold into this tile
    const int r = slot - (T + 3);
    const int cand[4] = {0, 1, nd - 1, nd};
    f = cand[r];
    own = false;
    if (f >= fa && f <= fb) return false;           // computed as an own face
    for (int e = 0; e < r; ++e)
      if (cand[e] == f) return false;               // duplicate (short lines)
    bool need = false;
    for (int k = 0; k < 6; ++k) {
      if (pair_f(k, nd) != f) continue;
      bool fl;
      const int src = remap(pair_q(k, nd), nd, g.bc[ax][0], g.bc[ax][1], fl);
      need = need || (src >= t0 && src < t1);
    }
    return need;
  };

  // a ghost's source cell is one of 0, 1, nd - 2, nd - 1: only a tile that
  // holds one of them (along either axis) has far-end faces to compute
  bool edge = x0 < 2 || x0 + TX > nx - 2;
  if constexpr (NDIM == 2) edge = edge || y0 < 2 || y0 + TY > ny - 2;
  const int ni = edge ? NI : NOWN;
  for (int base = 0; base < ni; base += 256) {
    const int i = base + tid;
    int ax = 0, line = 0, f = 0;
    bool own = false;
    const bool has = i < ni && item(i, ax, line, f, own);
    double Cb[4][NV];
    if (has) {
      if (ax == 0) face_vjp<NDIM, 0>(X, mu, scale, g, 0, y0 + line, 0, f, Cb);
      else if constexpr (NDIM == 2) face_vjp<NDIM, 1>(X, mu, scale, g, x0 + line, 0, 0, f, Cb);
      // ghost contributions whose source cell lies in the tile
      const int nd = g.n[ax], t0 = ax == 0 ? x0 : y0, T = ax == 0 ? TX : TY;
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int q = f - 2 + s;
        if (q >= 0 && q < nd) continue;
        bool fl;
        const int src = remap(q, nd, g.bc[ax][0], g.bc[ax][1], fl);
        if (src < t0 || src >= t0 + T) continue;
        const int k = pair_of(q, f, nd);
#pragma unroll
        for (int v = 0; v < NV; ++v) gbuf[ax][line][k][v] = Cb[s][v];
      }
    }
    // direct contributions, round by round; the rounds of an axis with no
    // own item in this batch are skipped (uniform over the workgroup)
    const bool xr = base < NOX;
    const bool yr = NDIM == 2 && base + 256 > NOXP && base < NOXP + NOY;
#pragma unroll
    for (int r = 0; r < 4 * NDIM; ++r) {
      if (!(r < 4 ? xr : yr)) continue;
      if (has && own && ax == r / 4 && (f & 3) == (r & 3)) {
        const int nd = g.n[ax], t0 = ax == 0 ? x0 : y0, T = ax == 0 ? TX : TY;
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const int q = f - 2 + s;
          if (q < 0 || q >= nd || q < t0 || q >= t0 + T) continue;
#pragma unroll
          for (int v = 0; v < NV; ++v) {
            if (ax == 0) acc[v][line][q - t0] += Cb[s][v];
            else acc[v][q - t0][line] += Cb[s][v];
          }
        }
      }
      __syncthreads();
    }
  }

  // the last batch may have run no round: its ghost contributions must be
  // visible before the folds
  __syncthreads();

  // ghost folds, then the conserved adjoint of this thread's cell
  const int gx = x0 + lx, gy = y0 + ly;
  if (gx >= nx || gy >= ny) return;
  double wb[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) wb[v] = acc[v][ly][lx];
#pragma unroll
  for (int ax = 0; ax < NDIM; ++ax) {
    const int nd = g.n[ax], j = ax == 0 ? gx : gy, line = ax == 0 ? ly : lx;
    if (j >= 2 && j < nd - 2) continue;             // no ghost has this cell as its source
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      bool fl;
      const int src = remap(pair_q(k, nd), nd, g.bc[ax][0], g.bc[ax][1], fl);
      if (src != j) continue;
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const double val = gbuf[ax][line][k][v];
        wb[v] += (fl && v == 1 + ax) ? -val : val;
      }
    }
  }
  const long long c = (long long)gy * nx + gx;
  double u[NV], ub[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) u[v] = X[v * N + c];
  prim_to_cons_adjoint<NDIM>(u, wb, g.gamma, ub);
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    double r = c0 * lam[v * N + c] + ub[v];
    if (lam1) r += c1 * lam1[v * N + c];
    out[v * N + c] = r;
  }
}

struct AdjLayout {
  size_t ctl, u1, lam1, wb, cbuf, total;
};

static AdjLayout adj_layout(const Grid& G) {
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
  AdjLayout L;
  const size_t state = (size_t)G.nvar * G.ncell * sizeof(double);
  size_t cmax = 0;
  for (int d = 0; d < G.ndim; ++d) {
    size_t faces = (size_t)(G.n[d] + 1) * (size_t)(G.ncell / G.n[d]);
    cmax = faces > cmax ? faces : cmax;
  }
  L.ctl = 0;
  L.u1 = 256;
  L.lam1 = L.u1 + al(state);
  L.wb = L.lam1 + al(state);
  L.cbuf = L.wb + al(state);
  L.total = L.cbuf + al(cmax * 4 * G.nvar * sizeof(double));
  return L;
}

// (dL/dX)^T (scale mu) into Wb (primitive adjoints), axes in the order x, y, z.
template <int NDIM, int AX>
static void launch_face(const Grid& G, const AdjGeo& g, const double* X, const double* mu,
                        const double* dt_dev, double factor, double* C, hipStream_t s) {
  long long nf = (long long)(G.n[AX] + 1) * (G.ncell / G.n[AX]);
  hipLaunchKernelGGL((adj_face<NDIM, AX>), dim3((unsigned)((nf + 255) / 256)), dim3(256), 0, s, X,
                     mu, dt_dev, factor, g, C);
}

// (dL/dX)^T (factor dt mu) into Wb (primitive adjoints), axes in the order x, y, z.
template <int NDIM>
static hipError_t adj_rhs(const Grid& G, const AdjGeo& g, const double* X, const double* mu,
                          const double* dt_dev, double factor, double* C, double* Wb,
                          hipStream_t s) {
  const long long N = G.ncell;
  for (int d = 0; d < NDIM; ++d) {
    if (d == 0) launch_face<NDIM, 0>(G, g, X, mu, dt_dev, factor, C, s);
    if constexpr (NDIM >= 2) if (d == 1) launch_face<NDIM, 1>(G, g, X, mu, dt_dev, factor, C, s);
    if constexpr (NDIM >= 3) if (d == 2) launch_face<NDIM, 2>(G, g, X, mu, dt_dev, factor, C, s);
    hipLaunchKernelGGL(adj_gather<NDIM>, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, g, d,
                       (const double*)C, Wb, d > 0 ? 1 : 0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <int NDIM>
static hipError_t adj_step(const Grid& G, const double* Un, const double* U1, const double* dt_dev,
                           double* lam, char* wb, const AdjLayout& L, hipStream_t s) {
  AdjGeo g;
  for (int d = 0; d < 3; ++d) {
    g.n[d] = G.n[d];
    g.bc[d][0] = G.bc[d][0];
    g.bc[d][1] = G.bc[d][1];
    g.inv_dx[d] = G.inv_dx[d];
  }
  g.gamma = G.gamma;
  double* lam1 = reinterpret_cast<double*>(wb + L.lam1);
  double* Wbuf = reinterpret_cast<double*>(wb + L.wb);
  double* C = reinterpret_cast<double*>(wb + L.cbuf);
  const long long N = G.ncell;
  const unsigned nb = (unsigned)((N + 255) / 256);
  hipError_t e;
  if constexpr (NDIM <= 2) {
    // one fused launch per product (adj_tile)
    using TS = AdjTileShape<NDIM>;
    const unsigned tiles = (unsigned)(((G.n[0] + TS::TX - 1) / TS::TX) *
                                      ((G.n[1] + TS::TY - 1) / TS::TY));
    // lam1 = lam/2 + (dL/dU1)^T (dt lam / 2)
    hipLaunchKernelGGL(adj_tile<NDIM>, dim3(tiles), dim3(256), 0, s, U1, (const double*)lam,
                       dt_dev, 0.5, g, (const double*)lam, 0.5, (const double*)nullptr, 0.0, lam1);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // lam0 = lam/2 + lam1 + (dL/dU)^T (dt lam1)
    hipLaunchKernelGGL(adj_tile<NDIM>, dim3(tiles), dim3(256), 0, s, Un, (const double*)lam1,
                       dt_dev, 1.0, g, (const double*)lam, 0.5, (const double*)lam1, 1.0, lam);
    return hipGetLastError();
  }
  // 3D: face kernels with their contributions through the workspace, a
  // gather per axis and the final map
  // lam1 = lam/2 + (dL/dU1)^T (dt lam / 2)
  if ((e = adj_rhs<NDIM>(G, g, U1, lam, dt_dev, 0.5, C, Wbuf, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(adj_final<NDIM>, dim3(nb), dim3(256), 0, s, (const double*)U1,
                     (const double*)Wbuf, G.gamma, N, (const double*)lam, 0.5,
                     (const double*)nullptr, 0.0, lam1);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // lam0 = lam/2 + lam1 + (dL/dU)^T (dt lam1)
  if ((e = adj_rhs<NDIM>(G, g, Un, lam1, dt_dev, 1.0, C, Wbuf, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(adj_final<NDIM>, dim3(nb), dim3(256), 0, s, Un, (const double*)Wbuf, G.gamma,
                     N, (const double*)lam, 0.5, (const double*)lam1, 1.0, lam);
  return hipGetLastError();
}

}  // namespace hard

using namespace hard;

extern "C" {

hard_status_t hard_adjoint_workspace_bytes(const hard_grid_t* g, size_t* bytes) {
  Grid G;
  hard_status_t st = check_grid(g, &G);
  if (st) return st;
  if (!bytes) return fail(HARD_ERR_INVALID_ARG, "bytes is NULL");
  if (G.dtype != HARD_F64) return fail(HARD_ERR_UNSUPPORTED, "the adjoint is built for HARD_F64");
  if (G.scheme != HARD_SCHEME_MUSCL_HLLC || G.rad)
    return fail(HARD_ERR_UNSUPPORTED, "the adjoint is built for HARD_SCHEME_MUSCL_HLLC without radiation");
  *bytes = adj_layout(G).total;
  return ok();
}

// Shared body of the two adjoint entry points: U_1 is the stage-1 state of
// U_n for this dt (NULL: recomputed into the workspace by the forward stage
// kernel).
static hard_status_t adjoint_step(const hard_grid_t* g, const void* U_n, const void* U_1,
                                  const double* dt_dev, void* lam, void* work, size_t work_bytes,
                                  void* stream, const char* name) {
  Grid G;
  hard_status_t st = check_grid(g, &G);
  if (st) return st;
  if (G.dtype != HARD_F64) return fail(HARD_ERR_UNSUPPORTED, "the adjoint is built for HARD_F64");
  if (G.scheme != HARD_SCHEME_MUSCL_HLLC || G.rad)
    return fail(HARD_ERR_UNSUPPORTED, "the adjoint is built for HARD_SCHEME_MUSCL_HLLC without radiation");
  if ((st = check_ptr(U_n, 8, "U_n"))) return st;
  if ((st = check_ptr(lam, 8, "lam"))) return st;
  if ((st = check_ptr(dt_dev, 8, "dt_dev"))) return st;
  if (U_1 && (st = check_ptr(U_1, 8, "U_1"))) return st;
  AdjLayout L = adj_layout(G);
  if ((st = check_work(work, work_bytes, L.total))) return st;
  hipStream_t s = (hipStream_t)stream;
  char* wb = static_cast<char*>(work);
  hipError_t e;
  const double* U1 = static_cast<const double*>(U_1);
  if (!U1) {
    // recompute U1 = U + dt L(U) with the forward stage kernel
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
    a.dt = dt_dev;
    a.ctl = reinterpret_cast<Control*>(wb + L.ctl);
    a.cz = stage_cz_override();
    a.src = U_n;
    a.un = U_n;
    a.dst = wb + L.u1;
    if ((e = launch_stage(G.ndim, G.dtype, a, 1, s)) != hipSuccess) return hip_fail(e, name);
    U1 = reinterpret_cast<const double*>(wb + L.u1);
  }
  const double* Un = static_cast<const double*>(U_n);
  double* lm = static_cast<double*>(lam);
  switch (G.ndim) {
    case 1: e = adj_step<1>(G, Un, U1, dt_dev, lm, wb, L, s); break;
    case 2: e = adj_step<2>(G, Un, U1, dt_dev, lm, wb, L, s); break;
    default: e = adj_step<3>(G, Un, U1, dt_dev, lm, wb, L, s); break;
  }
  if (e != hipSuccess) return hip_fail(e, name);
  return ok();
}

hard_status_t hard_hydro_step_adjoint(const hard_grid_t* g, const void* U_n, const double* dt_dev,
                                      void* lam, void* work, size_t work_bytes, void* stream) {
  return adjoint_step(g, U_n, nullptr, dt_dev, lam, work, work_bytes, stream,
                      "hard_hydro_step_adjoint");
}

hard_status_t hard_hydro_step_adjoint_given_u1(const hard_grid_t* g, const void* U_n,
                                               const void* U_1, const double* dt_dev, void* lam,
                                               void* work, size_t work_bytes, void* stream) {
  if (!U_1) return fail(HARD_ERR_INVALID_ARG, "U_1 is NULL");
  return adjoint_step(g, U_n, U_1, dt_dev, lam, work, work_bytes, stream,
                      "hard_hydro_step_adjoint_given_u1");
}

}  // extern "C"
