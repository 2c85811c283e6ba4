// The paper's own face scheme (section 2.2.2): WENO5-Z face states of the
// primitive variables (Borges, Carmona, Costa and Don 2008) with the HLL flux
// (Harten, Lax and van Leer 1983; Davis wave speeds), inside the same Heun
// stages as the MUSCL-HLLC path.  Three ghost layers per side.
//
// This path is a pipeline per stage, not the fused tile kernel:
//   weno_xface   one thread per x face: the primitives of the stage source
//                for a run of rows in LDS (each cell's also stored to W for
//                the other axes, with the status bits), then six cells along
//                x (ghosts by index remap), WENO5-Z left and right states,
//                HLL flux into the x face array;
//   weno_face    (3D) the same for the y faces, the six cells read from W;
//   weno_walk    (2D, 3D) the faces of the last axis and the update in one
//                pass: each thread walks a column along that axis, computes
//                its faces from a register window of W and updates each
//                cell with the other axes' fluxes from their arrays; no face
//                array of the last axis exists;
//   weno_update  (1D) grid-stride over the cells: L(U) = -(F+ - F-)/dx, the
//                stage combine, and in stage 2 the fused CFL step.
// Bytes per cell and stage: the fused MUSCL kernel moves 2-3 nvar words; this
// pipeline 3 + 2 + 5 (+ 1 in stage 2) nvar words in 3D, 3 + 4 (+ 1) in 2D
// (W and the face arrays of the other axes round-trip through memory).
//
// Arithmetic: the face kernels are bound by FP64 instruction issue (about
// 1100 VALU instructions per face, 0.8 of issue busy), so the WENO5-Z
// reconstruction and the HLL flux fuse multiply-adds within each expression
// and take refined reciprocals and the rsq-based sound speed (errors near
// 1e-16 relative; 7.5% of the step).  The primitives and the update keep
// plain IEEE division, no contraction, in the order of the formulas.  On the
// paper's Sod run (503 steps) every step stays within 5e-16 of the oracle's
// step from the same state and the whole run within 1e-11.

#include "hydro_device.hpp"
#include "launch.hpp"

namespace hard {

// WENO5-Z value at the right face of the middle cell of v0..v4 (cells
// i-2..i+2): third-order candidates on the three sub-stencils, Jiang-Shu
// smoothness indicators, tau5 = |beta0 - beta2|, weights
// d_k (1 + tau5 / (beta_k + eps)) with d = (1/10, 6/10, 3/10), eps = 1e-40,
// evaluated over their common denominator with a single (refined)
// reciprocal.
// Evaluated in double for both storage types: at a jump the weight ratios
// reach 1e40 and beyond, out of float range (and the FP64 vector rate of
// gfx950 equals its unpacked FP32 rate).
__device__ __forceinline__ double weno5z_d(double v0, double v1, double v2, double v3, double v4) {
  // 6 x the three third-order candidates
  double q0 = 2.0 * v0 - 7.0 * v1 + 11.0 * v2;
  double q1 = -v1 + 5.0 * v2 + 2.0 * v3;
  double q2 = 2.0 * v2 + 5.0 * v3 - v4;
  double s0 = v0 - 2.0 * v1 + v2, t0 = v0 - 4.0 * v1 + 3.0 * v2;
  double s1 = v1 - 2.0 * v2 + v3, t1 = v1 - v3;
  double s2 = v2 - 2.0 * v3 + v4, t2 = 3.0 * v2 - 4.0 * v3 + v4;
  const double c1 = 13.0 / 12.0, c2 = 0.25, eps = 1e-40;
  double b0 = c1 * s0 * s0 + c2 * t0 * t0;
  double b1 = c1 * s1 * s1 + c2 * t1 * t1;
  double b2 = c1 * s2 * s2 + c2 * t2 * t2;
  double tau = fabs(b0 - b2);
  // the weights over the common denominator (b0 + eps)(b1 + eps)(b2 + eps),
  // the 1/6 of the candidates folded into the normalisation: one reciprocal
  const double e0 = b0 + eps, e1 = b1 + eps, e2 = b2 + eps;
  double a0 = 0.1 * (e0 + tau) * (e1 * e2);
  double a1 = 0.6 * (e1 + tau) * (e0 * e2);
  double a2 = 0.3 * (e2 + tau) * (e0 * e1);
  return (a0 * q0 + a1 * q1 + a2 * q2) * fast_rcp(6.0 * (a0 + a1 + a2));
}
template <typename R>
__device__ __forceinline__ R weno5z(R v0, R v1, R v2, R v3, R v4) {
  return R(weno5z_d(v0, v1, v2, v3, v4));
}

// HLL flux of face states ordered (rho, u_n, u_t..., p); output (mass,
// normal momentum, transverse momenta, energy).  Davis wave speeds; F_L if
// S_L >= 0, F_R if S_R <= 0, else (S_R F_L - S_L F_R + S_L S_R (U_R - U_L)) /
// (S_R - S_L).
template <typename R, int NV>
__device__ __forceinline__ void hll_ordered(const R* WL, const R* WR, R gam, R gm1, R* F) {
  constexpr int NT = NV - 3;
  const R rL = WL[0], uL = WL[1], pL = WL[NV - 1];
  const R rR = WR[0], uR = WR[1], pR = WR[NV - 1];
  R cL = sound_speed(gam * pL, rL);
  R cR = sound_speed(gam * pR, rR);
  const R igm1 = R(1) / gm1;
  R qL = uL * uL, qR = uR * uR;
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    qL = qL + WL[2 + t] * WL[2 + t];
    qR = qR + WR[2 + t] * WR[2 + t];
  }
  const R EL = pL * igm1 + R(0.5) * rL * qL;
  const R ER = pR * igm1 + R(0.5) * rR * qR;
  R aL = uL - cL, bL = uR - cR;
  R SL = (aL <= bL) ? aL : bL;
  R aR = uL + cL, bR = uR + cR;
  R SR = (aR >= bR) ? aR : bR;
  const R mL = rL * uL, mR = rR * uR;
  R FL[NV], FR[NV], UL[NV], UR[NV];
  FL[0] = mL;
  FR[0] = mR;
  UL[0] = rL;
  UR[0] = rR;
  FL[1] = mL * uL + pL;
  FR[1] = mR * uR + pR;
  UL[1] = mL;
  UR[1] = mR;
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    FL[2 + t] = mL * WL[2 + t];
    FR[2 + t] = mR * WR[2 + t];
    UL[2 + t] = rL * WL[2 + t];
    UR[2 + t] = rR * WR[2 + t];
  }
  FL[NV - 1] = (EL + pL) * uL;
  FR[NV - 1] = (ER + pR) * uR;
  UL[NV - 1] = EL;
  UR[NV - 1] = ER;
  if (SL >= R(0)) {
#pragma unroll
    for (int v = 0; v < NV; ++v) F[v] = FL[v];
  } else if (SR <= R(0)) {
#pragma unroll
    for (int v = 0; v < NV; ++v) F[v] = FR[v];
  } else {
    const R id = fast_rcp(SR - SL);
#pragma unroll
    for (int v = 0; v < NV; ++v)
      F[v] = (SR * FL[v] - SL * FR[v] + SL * SR * (UR[v] - UL[v])) * id;
  }
}

// Primitives of one conserved state in the order of the formulas: ke =
// 0.5 |m|^2 / rho, e = E - ke, p = (gamma - 1) e, u_d = m_d / rho.  Float
// storage recovers e in double.
template <typename R, int NDIM>
__device__ __forceinline__ void primitives_plain(const R* u, double gamma, R* w) {
#pragma clang fp contract(off)
  const double rho = (double)u[0];
  double q = (double)u[1] * (double)u[1];
#pragma unroll
  for (int d = 1; d < NDIM; ++d) q = q + (double)u[1 + d] * (double)u[1 + d];
  const double ke = 0.5 * q / rho;
  const double e = (double)u[NDIM + 1] - ke;
  w[0] = u[0];
#pragma unroll
  for (int d = 0; d < NDIM; ++d) w[1 + d] = u[1 + d] / u[0];
  w[NDIM + 1] = R((gamma - 1.0) * e);
}

// x faces with the primitives of their stencils computed in the same pass
// (no separate primitive pass over the grid).  A block takes 256 consecutive faces of the x-face
// layout (f, j, k).  Face t of the block reads the six cells f - 3 .. f + 2
// of its row from LDS slots p(t) .. p(t) + 5, p(t) = t + 6 (r - r0) with r
// its row and r0 the block's first row: consecutive faces of a row share
// five slots, and each row starts six slots after the previous one.  Every
// slot is filled once: each face thread fills the slot of cell f (a ghost
// past the row's end by index remap, with the wall flip), the block's first
// face of a row also cells f - 3 .. f - 1, its last face cells f + 1 and
// f + 2.  The thread of face f < nx also stores the primitives of cell f to
// W (read by the y faces and the z walk) and its status bits.  Rows of at
// least 4 faces (nx >= 3) bound the rows a block touches to 65.
constexpr int WENO_XSLOTS = 256 + 5 + 6 * 64;

template <typename R, int NDIM>
__global__ __launch_bounds__(256) void weno_xface(WenoArgs a) {
  constexpr int NV = NDIM + 2;
  __shared__ R S[NV][WENO_XSLOTS];
  const int nx = a.n[0], ny = a.n[1], nz = a.n[2];
  const long long N = (long long)nx * ny * nz;
  const long long nface = N / nx * (nx + 1);
  const unsigned mx = (unsigned)nx + 1u;
  const long long base = (long long)xcd_tile(blockIdx.x, gridDim.x) * blockDim.x;
  const long long idx = base + threadIdx.x;
  const bool live = idx < nface;
  // the face count is below 2^32 (fewer than 2^31 cells): 32-bit splits
  const unsigned r0 = (unsigned)base / mx;
  const unsigned u = (unsigned)(live ? idx : base);
  const int f = (int)(u % mx);
  const unsigned r = u / mx;               // row (j, k) = (r % ny, r / ny)
  const int p = (int)threadIdx.x + 6 * (int)(r - r0);
  const R* U = static_cast<const R*>(a.src);
  R* W = static_cast<R*>(a.W);
  unsigned flags = 0;
  auto fill = [&](int q, int slot, bool own) {
    bool flip;
    const int qq = remap(q, nx, a.bc[0][0], a.bc[0][1], flip);
    const long long cell = (long long)r * nx + qq;
    R uc[NV], w[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) uc[v] = U[v * N + cell];
    primitives_plain<R, NDIM>(uc, a.gamma, w);
    if (own) {
      flags = cell_flags<R, NV>(uc, w[NV - 1]);
      if constexpr (NDIM >= 2) {
#pragma unroll
        for (int v = 0; v < NV; ++v) W[v * N + cell] = w[v];
      }
    }
    if (flip) w[1] = -w[1];
#pragma unroll
    for (int v = 0; v < NV; ++v) S[v][slot] = w[v];
  };
  if (live) {
    fill(f, p + 3, f < nx);
    if (f == 0 || idx == base)
      for (int s = 0; s < 3; ++s) fill(f - 3 + s, p + s, false);
    if (f == nx || idx == base + (long long)blockDim.x - 1 || idx == nface - 1)
      for (int s = 4; s < 6; ++s) fill(f - 3 + s, p + s, false);
  }
  __syncthreads();
  if (live) {
    R c[6][NV];
#pragma unroll
    for (int s = 0; s < 6; ++s)
#pragma unroll
      for (int v = 0; v < NV; ++v) c[s][v] = S[v][p + s];
    // face states ordered (rho, u_x, u_y, u_z, p): the x faces need no swap
    R WL[NV], WR[NV], Fn[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      WL[v] = weno5z<R>(c[0][v], c[1][v], c[2][v], c[3][v], c[4][v]);
      WR[v] = weno5z<R>(c[5][v], c[4][v], c[3][v], c[2][v], c[1][v]);
    }
    const R gam = R(a.gamma), gm1 = R(a.gamma - 1.0);
    hll_ordered<R, NV>(WL, WR, gam, gm1, Fn);
    R* F = static_cast<R*>(a.F[0]);
#pragma unroll
    for (int v = 0; v < NV; ++v) F[v * nface + idx] = Fn[v];
  }
  flags = wave_or(flags);
  if ((threadIdx.x & 63) == 0 && flags) atomicOr(&a.ctl->flags, flags);
}

// y faces of a 3D grid: face f (0..ny) lies between cells f-1 and f.
// Linear face index (the layout of the face array), x fastest: (i, f, k).
// A block takes 256 consecutive faces of that layout: the six cells of a
// face lie in its own plane, which the L2 holds.  The x faces are computed
// by weno_xface, the z faces (and the y faces of a 2D grid) inside
// weno_walk.

template <typename R, int NDIM, int AX>
__global__ __launch_bounds__(256) void weno_face(WenoArgs a) {
  constexpr int NV = NDIM + 2;
  const int nx = a.n[0], ny = a.n[1], nz = a.n[2];
  const long long N = (long long)nx * ny * nz;
  const long long nface = N / a.n[AX] * (a.n[AX] + 1);
  static_assert(AX == 1 && NDIM == 3, "x faces: weno_xface; the last axis: weno_walk");
  const long long idx = (long long)xcd_tile(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (idx >= nface) return;
  // the face count of an axis is below 2^32 (fewer than 2^31 cells), so the
  // index splits in 32-bit unsigned arithmetic
  const unsigned u = (unsigned)idx, my = (unsigned)ny + 1u;
  const int i = (int)(u % (unsigned)nx);
  const unsigned r = u / (unsigned)nx;
  const int f = (int)(r % my), k = (int)(r / my);
  const R* W = static_cast<const R*>(a.W);
  // six cells f-3 .. f+2 along AX, primitives with the wall flip applied
  R c[6][NV];
#pragma unroll
  for (int s = 0; s < 6; ++s) {
    bool flip;
    const int q = remap(f - 3 + s, a.n[AX], a.bc[AX][0], a.bc[AX][1], flip);
    const long long cell = ((long long)k * ny + q) * nx + i;
#pragma unroll
    for (int v = 0; v < NV; ++v) c[s][v] = W[v * N + cell];
    if (flip) c[s][1 + AX] = -c[s][1 + AX];
  }
  // face states ordered (rho, u_n, u_t in axis order, p)
  int perm[NV];
  perm[0] = 0;
  perm[1] = 1 + AX;
  {
    int t = 2;
#pragma unroll
    for (int d = 0; d < NDIM; ++d)
      if (d != AX) perm[t++] = 1 + d;
  }
  perm[NV - 1] = NV - 1;
  R WL[NV], WR[NV], Fn[NV];
#pragma unroll
  for (int m = 0; m < NV; ++m) {
    const int v = perm[m];
    WL[m] = weno5z<R>(c[0][v], c[1][v], c[2][v], c[3][v], c[4][v]);
    WR[m] = weno5z<R>(c[5][v], c[4][v], c[3][v], c[2][v], c[1][v]);
  }
  const R gam = R(a.gamma), gm1 = R(a.gamma - 1.0);
  hll_ordered<R, NV>(WL, WR, gam, gm1, Fn);
  R* F = static_cast<R*>(a.F[AX]);
#pragma unroll
  for (int m = 0; m < NV; ++m) F[perm[m] * nface + idx] = Fn[m];
}

template <typename R, int NDIM, int STAGE>
__global__ __launch_bounds__(256) void weno_update(WenoArgs a) {
#pragma clang fp contract(off)
  constexpr int NV = NDIM + 2;
  const int nx = a.n[0], ny = a.n[1], nz = a.n[2];
  const long long N = (long long)nx * ny * nz;
  const bool fuse = STAGE == 2 && a.fuse_cfl;
  double smax = 0.0;
  // grid-stride with a bounded grid: one CFL slot per workgroup
  for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < N;
       c += (long long)gridDim.x * blockDim.x) {
    // fewer than 2^31 cells: the cell index splits in 32-bit unsigned arithmetic
    const unsigned cu = (unsigned)c, r = cu / (unsigned)nx;
    const int i = (int)(cu % (unsigned)nx);
    const int j = (int)(r % (unsigned)ny), k = (int)(r / (unsigned)ny);
    const R* src = static_cast<const R*>(a.src);
    const R* un = static_cast<const R*>(a.un);
    R* dst = static_cast<R*>(a.dst);
    const R dt = R(*a.dt);
    long long fm[3], step[3], nf[3];
    fm[0] = ((long long)k * ny + j) * (nx + 1) + i;
    step[0] = 1;
    nf[0] = (long long)(nx + 1) * ny * nz;
    fm[1] = ((long long)k * (ny + 1) + j) * nx + i;
    step[1] = nx;
    nf[1] = (long long)nx * (ny + 1) * nz;
    fm[2] = ((long long)k * ny + j) * nx + i;
    step[2] = (long long)nx * ny;
    nf[2] = (long long)nx * ny * (nz + 1);
    R Out[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      R l = R(0);
#pragma unroll
      for (int d = 0; d < NDIM; ++d) {
        const R* F = static_cast<const R*>(a.F[d]) + v * nf[d];
        const R df = F[fm[d] + step[d]] - F[fm[d]];
        l = l - (a.dx_pow2 ? df * R(a.inv_dx[d]) : df / R(a.dx[d]));
      }
      const R u = src[v * N + c];
      if (STAGE == 1)
        Out[v] = u + dt * l;
      else
        Out[v] = R(0.5) * (un[v * N + c] + (u + dt * l));
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) dst[v * N + c] = Out[v];
    if (fuse) {
      double Ud[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) Ud[v] = (double)Out[v];
      smax = fmax(smax, cfl_signal<R, NDIM>(Ud, a.inv_dx, a.gamma));
    }
  }
  block_finish<256>(0u, smax, fuse, a.ctl, a.slots + blockIdx.x);
}


// 2D and 3D: the faces of the last axis (y in 2D, z in 3D) fused into the
// stage update.  A work unit is a tile of columns along that axis (64 x 4
// (i, j) columns in 3D, 256 i columns in 2D) and a chunk of WENO_WCHUNK
// cells along it (WENO_WCHUNK, halved while the launch would have fewer
// than about 1500 units, down to 4); each thread walks its column with the six cells of the
// current face in a register window (one new cell loaded per face) and
// carries the flux of the face below the current cell from the previous
// position, so no face array of that axis goes through memory (the face at
// a chunk's upper end is computed by both chunks that share it).  The other
// axes' face fluxes come from their arrays.  The face arithmetic is
// weno_face's and the update's weno_update's, in the same order.
// Grid-stride over the units, one CFL slot per workgroup.  In 3D, against a
// z face kernel plus a separate update: 4.44 against 5.27 ms per step of the
// 256^3 blast, the same bits; chunks of 16 or 64 cells 4.62 and 4.52 ms,
// loading the next window cell one face ahead 4.48 ms.
constexpr int WENO_ZTX = 64, WENO_ZTY = 4, WENO_WCHUNK = 32;

template <typename R, int NDIM, int STAGE>
__global__ __launch_bounds__(256) void weno_walk(WenoArgs a, long long units, int wchunk) {
  static_assert(NDIM >= 2, "1D grids use weno_update");
  constexpr int NV = NDIM + 2, WA = NDIM - 1;
  constexpr int CX = NDIM == 3 ? WENO_ZTX : 256, CY = NDIM == 3 ? WENO_ZTY : 1;
  const int nx = a.n[0], ny = a.n[1], nz = a.n[2];
  const int nw = a.n[WA];
  const long long N = (long long)nx * ny * nz;
  const long long WS = NDIM == 3 ? (long long)nx * ny : nx;  // stride along the walk axis
  const bool fuse = STAGE == 2 && a.fuse_cfl;
  const int tilesx = (nx + CX - 1) / CX;
  const int nchunk = (nw + wchunk - 1) / wchunk;
  const long long nf0 = (long long)(nx + 1) * ny * nz, nf1 = (long long)nx * (ny + 1) * nz;
  const R* W = static_cast<const R*>(a.W);
  const R* src = static_cast<const R*>(a.src);
  const R* un = static_cast<const R*>(a.un);
  R* dst = static_cast<R*>(a.dst);
  const R* Fx = static_cast<const R*>(a.F[0]);
  const R* Fy = static_cast<const R*>(a.F[1]);
  const R dt = R(*a.dt);
  const R gam = R(a.gamma), gm1 = R(a.gamma - 1.0);
  // face order along the walk axis: (rho, u_w, the other velocities, p)
  constexpr int perm3[5] = {0, 3, 1, 2, 4}, perm2[4] = {0, 2, 1, 3};
  double smax = 0.0;
  for (long long u = xcd_tile(blockIdx.x, gridDim.x); u < units; u += gridDim.x) {
    const int ch = (int)(u % nchunk);
    const long long t = u / nchunk;
    const int i = (int)(t % tilesx) * CX + (int)(threadIdx.x % CX);
    const int j = NDIM == 3 ? (int)(t / tilesx) * CY + (int)(threadIdx.x / CX) : 0;
    if (i >= nx || j >= ny) continue;
    const int k0 = ch * wchunk, k1 = min(k0 + wchunk, nw);
    const long long col = (long long)j * nx + i;
    auto load_cell = [&](int q, R* out) {
      bool flip;
      const int kk = remap(q, nw, a.bc[WA][0], a.bc[WA][1], flip);
      const long long cell = (long long)kk * WS + col;
#pragma unroll
      for (int v = 0; v < NV; ++v) out[v] = W[v * N + cell];
      if (flip) out[1 + WA] = -out[1 + WA];
    };
    R c[6][NV], Fm[NV];
#pragma unroll
    for (int s = 1; s < 6; ++s) load_cell(k0 - 4 + s, c[s]);
    for (int f = k0; f <= k1; ++f) {
      // window: cells f - 3 .. f + 2
#pragma unroll
      for (int s = 0; s < 5; ++s)
#pragma unroll
        for (int v = 0; v < NV; ++v) c[s][v] = c[s + 1][v];
      load_cell(f + 2, c[5]);
      R WL[NV], WR[NV], Fo[NV], Fn[NV];
#pragma unroll
      for (int m = 0; m < NV; ++m) {
        const int v = NDIM == 3 ? perm3[m] : perm2[m];
        WL[m] = weno5z<R>(c[0][v], c[1][v], c[2][v], c[3][v], c[4][v]);
        WR[m] = weno5z<R>(c[5][v], c[4][v], c[3][v], c[2][v], c[1][v]);
      }
      hll_ordered<R, NV>(WL, WR, gam, gm1, Fo);
#pragma unroll
      for (int m = 0; m < NV; ++m) Fn[NDIM == 3 ? perm3[m] : perm2[m]] = Fo[m];
      if (f > k0) {
#pragma clang fp contract(off)
        const int k = f - 1;  // the cell below face f along the walk axis
        const long long cidx = (long long)k * WS + col;
        // x face (i, j, k) in 3D, (i, k) in 2D; y face (i, k, j) ... of a 3D grid
        const long long fx = NDIM == 3 ? ((long long)k * ny + j) * (nx + 1) + i
                                       : (long long)k * (nx + 1) + i;
        const long long fy = ((long long)k * (ny + 1) + j) * nx + i;
        R Out[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          R dfs[NDIM];
          dfs[0] = Fx[v * nf0 + fx + 1] - Fx[v * nf0 + fx];
          if constexpr (NDIM == 3) dfs[1] = Fy[v * nf1 + fy + nx] - Fy[v * nf1 + fy];
          dfs[NDIM - 1] = Fn[v] - Fm[v];
          R l = R(0);
#pragma unroll
          for (int d = 0; d < NDIM; ++d) {
            const R df = dfs[d];
            l = l - (a.dx_pow2 ? df * R(a.inv_dx[d]) : df / R(a.dx[d]));
          }
          const R uc = src[v * N + cidx];
          if (STAGE == 1)
            Out[v] = uc + dt * l;
          else
            Out[v] = R(0.5) * (un[v * N + cidx] + (uc + dt * l));
        }
#pragma unroll
        for (int v = 0; v < NV; ++v) dst[v * N + cidx] = Out[v];
        if (fuse) {
          double Ud[NV];
#pragma unroll
          for (int v = 0; v < NV; ++v) Ud[v] = (double)Out[v];
          smax = fmax(smax, cfl_signal<R, NDIM>(Ud, a.inv_dx, a.gamma));
        }
      }
#pragma unroll
      for (int v = 0; v < NV; ++v) Fm[v] = Fn[v];
    }
  }
  block_finish<256>(0u, smax, fuse, a.ctl, a.slots + blockIdx.x);
}

template <typename R, int NDIM>
static hipError_t weno_stage_t(const WenoArgs& a, int stage, hipStream_t s) {
  const long long N = (long long)a.n[0] * a.n[1] * a.n[2];
  const bool fuse = stage == 2 && a.fuse_cfl;
  if (a.n[0] < 3) return hipErrorInvalidValue;  // weno_xface's slot bound
  auto faces = [&](int d) { return (unsigned)((N / a.n[d] * (a.n[d] + 1) + 255) / 256); };
  hipLaunchKernelGGL((weno_xface<R, NDIM>), dim3(faces(0)), dim3(256), 0, s, a);
  if constexpr (NDIM == 3) hipLaunchKernelGGL((weno_face<R, NDIM, 1>), dim3(faces(1)), dim3(256), 0, s, a);
  unsigned ng;
  if constexpr (NDIM >= 2) {
    const int cx = NDIM == 3 ? WENO_ZTX : 256, cy = NDIM == 3 ? WENO_ZTY : 1;
    const int nw = a.n[NDIM - 1];
    const long long cols = (long long)((a.n[0] + cx - 1) / cx) * (NDIM == 3 ? (a.n[1] + cy - 1) / cy : 1);
    int wchunk = WENO_WCHUNK;
    while (wchunk > 4 && cols * ((nw + wchunk - 1) / wchunk) < 1536) wchunk /= 2;
    const long long units = cols * ((nw + wchunk - 1) / wchunk);
    const long long cap = fuse ? a.nslots : GRID_STRIDE_MAX_BLOCKS;
    if (cap < 1) return hipErrorInvalidValue;
    ng = (unsigned)(units < cap ? units : cap);
    if (stage == 1)
      hipLaunchKernelGGL((weno_walk<R, NDIM, 1>), dim3(ng), dim3(256), 0, s, a, units, wchunk);
    else
      hipLaunchKernelGGL((weno_walk<R, NDIM, 2>), dim3(ng), dim3(256), 0, s, a, units, wchunk);
  } else {
    const unsigned nb = (unsigned)((N + 255) / 256);
    ng = nb < 2048u ? nb : 2048u;
    if (fuse && (int)ng > a.nslots) return hipErrorInvalidValue;
    if (stage == 1)
      hipLaunchKernelGGL((weno_update<R, NDIM, 1>), dim3(ng), dim3(256), 0, s, a);
    else
      hipLaunchKernelGGL((weno_update<R, NDIM, 2>), dim3(ng), dim3(256), 0, s, a);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !fuse) return e;
  return launch_cfl_final(a.slots, (int)ng, a.cfl, a.next_dt, s);
}

hipError_t launch_weno_stage(int ndim, int dtype, const WenoArgs& a, int stage, hipStream_t s) {
  if (dtype == 0) {
    switch (ndim) {
      case 1: return weno_stage_t<double, 1>(a, stage, s);
      case 2: return weno_stage_t<double, 2>(a, stage, s);
      case 3: return weno_stage_t<double, 3>(a, stage, s);
    }
  } else {
    switch (ndim) {
      case 1: return weno_stage_t<float, 1>(a, stage, s);
      case 2: return weno_stage_t<float, 2>(a, stage, s);
      case 3: return weno_stage_t<float, 3>(a, stage, s);
    }
  }
  return hipErrorInvalidValue;
}

}  // namespace hard
