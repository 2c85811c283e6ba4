// One tile of a Heun stage: the shared body of the single-grid stage kernel
// and the batched kernel (HARD paper section 2.2.2: finite-volume face
// difference, Heun's Butcher tableau in Shu-Osher form).
//
// A workgroup of TX x TY threads owns a TX x TY tile of cells in the x-y
// plane and walks the z planes [z0, z1) (3D).  For each plane it
//   1. builds the primitive states of the tile plus a two-cell x/y halo in
//      LDS (interior cells come from a per-thread register window along z,
//      halo cells are loaded and converted here; ghost cells are produced by
//      index remapping, so no ghost arrays exist in HBM),
//   2. computes every x and y face flux of the tile once, into LDS,
//   3. computes the z face above each cell from the register window (the face
//      below was computed in the previous plane),
//   4. forms L(U) and the stage combine, and stores the cell once.
// 2D grids use one plane (no z walk), 1D grids one row.
#pragma once

#include "hydro_device.hpp"

namespace hard {

struct TileArgs {
  const void* src;  // stencil source: U^n (stage 1) or U^1 (stage 2)
  const void* un;   // U^n for the stage-2 combine
  void* dst;        // U^1 (stage 1) or U^{n+1} (stage 2; may alias un)
  int n[3];
  int bc[3][2];
  double dx[3];
  double inv_dx[3];
  double gamma;
  double dt;
  int x0, y0, z0, z1;  // tile origin and z range
  int fuse_cfl;        // stage 2: accumulate the CFL signal max of the output
};

// LDS elements (of type R) one tile needs.
template <int NDIM, typename R, int TX, int TY>
struct TileShape {
  static constexpr int NV = NDIM + 2;
  static constexpr int LX = TX + 4;
  static constexpr int LY = NDIM >= 2 ? TY + 4 : 1;
  static constexpr int NF = (TX + 1) * TY + (NDIM >= 2 ? TX * (TY + 1) : 0);
  static constexpr int lds_elems = NV * (LX * LY + NF);
};

// Runs one tile; ORs status bits into `flags` and maxes the CFL signal sum of
// the stored cells into `smax` (when a.fuse_cfl).  Every thread of the
// workgroup must call it (it contains barriers).
//
// NTHR (>= TX*TY) is the workgroup size; threads beyond TX*TY own no cell but
// take part in the face and halo loops (a 1D tile of 255 cells has exactly
// 256 faces, one per thread of a 256-thread workgroup).
template <int NDIM, typename R, int STAGE, int TX, int TY, int NTHR = TX * TY>
__device__ __forceinline__ void run_tile(const TileArgs& a, R* lds, unsigned& flags, double& smax) {
  constexpr int NV = NDIM + 2;
  constexpr int NT = NTHR;
  static_assert(NTHR >= TX * TY, "one thread per cell at least");
  constexpr int OY = NDIM >= 2 ? 2 : 0;               // LDS row offset of the tile
  constexpr int LX = TX + 4;
  constexpr int LY = NDIM >= 2 ? TY + 4 : 1;
  constexpr int LXY = LX * LY;
  constexpr int NFX = (TX + 1) * TY;                  // x faces per plane
  constexpr int NFY = NDIM >= 2 ? TX * (TY + 1) : 0;  // y faces per plane
  constexpr int NF = NFX + NFY;
  constexpr int NHALO = NDIM >= 2 ? 4 * (TX + TY) : 4;
  static_assert(NDIM >= 2 || TY == 1, "1D tiles are one row");

  R* Ws = lds;            // NV * LXY: primitives of the plane (tile + halo)
  R* Fs = lds + NV * LXY; // NV * NF: in-plane face fluxes, x faces then y faces

  const int tid = threadIdx.x;
  const bool owner = tid < TX * TY;  // this thread owns a cell column of the tile
  const int tx = owner ? tid % TX : 0, ty = owner ? tid / TX : 0;
  const int nx = a.n[0], ny = a.n[1], nz = a.n[2];
  const long long N = (long long)nx * ny * nz;

  const int x0 = a.x0, y0 = a.y0;
  const int gx = x0 + tx, gy = y0 + ty;
  const bool inside = owner && gx < nx && gy < ny;
  const int z0 = a.z0, z1 = a.z1;

  const R* __restrict__ src = static_cast<const R*>(a.src);
  const R* __restrict__ un = static_cast<const R*>(a.un);
  R* __restrict__ dst = static_cast<R*>(a.dst);
  const double gm1 = a.gamma - 1.0;
  const R gam = R(a.gamma);
  const R inv_gm1 = R(1.0 / gm1);
  const R dt = R(a.dt);
  const R idx0 = R(a.inv_dx[0]), idx1 = R(a.inv_dx[1]), idx2 = R(a.inv_dx[2]);

  // this thread's column, clamped (and mirrored past reflecting walls) for
  // the overhang of ragged tiles; such threads never store
  bool fx_, fy_;
  const int cx = remap(gx, nx, a.bc[0][0], a.bc[0][1], fx_);
  const int cy = remap(gy, ny, a.bc[1][0], a.bc[1][1], fy_);
  const long long col = (long long)cy * nx + cx;

  auto zplane = [&](int q, bool& fz) -> long long {
    int z = NDIM == 3 ? remap(q, nz, a.bc[2][0], a.bc[2][1], fz) : 0;
    return (long long)z * nx * ny;
  };
  auto load_cons = [&](long long c, R* Uc) {
#pragma unroll
    for (int v = 0; v < NV; ++v) Uc[v] = src[v * N + c];
  };
  // primitive state of this thread's column from conserved values
  auto col_prim = [&](const R* Uc, bool fz, R* W) {
    to_primitive<R, NDIM>(Uc, W, gm1);
    if (fx_) W[1] = -W[1];
    if (NDIM >= 2 && fy_) W[2] = -W[2];
    if (NDIM == 3 && fz) W[3] = -W[3];
  };

  // z register window (3D): P0 = plane z, P1 = z+1, S0 = slope at z, Fm = flux
  // through the face z-1/2 (variables in the order rho, u_z, u_x, u_y, p)
  R P0[NV], P1[NV], S0[NV], Fm[NV];
  // conserved values of this column at planes z and z+1 (each cell is loaded
  // from memory once per stage; the combine uses them from registers)
  R Ucur[NV], Uc1[NV];
  if (NDIM < 3) load_cons(col, Ucur);
  if constexpr (NDIM == 3) {
    R Pm2[NV], Pm1[NV], Ut[NV];
    bool fz;
    long long zo;
    zo = zplane(z0 - 2, fz); load_cons(zo + col, Ut); col_prim(Ut, fz, Pm2);
    zo = zplane(z0 - 1, fz); load_cons(zo + col, Ut); col_prim(Ut, fz, Pm1);
    zo = zplane(z0, fz);     load_cons(zo + col, Ucur); col_prim(Ucur, fz, P0);
    zo = zplane(z0 + 1, fz); load_cons(zo + col, Uc1); col_prim(Uc1, fz, P1);
    R WL[NV], WR[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      R d0 = Pm1[v] - Pm2[v], d1 = P0[v] - Pm1[v], d2 = P1[v] - P0[v];
      R sm1 = minmod(d0, d1);
      S0[v] = minmod(d1, d2);
      WL[v] = Pm1[v] + R(0.5) * sm1;
      WR[v] = P0[v] - R(0.5) * S0[v];
    }
    R A[NV], B[NV], Fn[NV];
    A[0] = WL[0]; A[1] = WL[3]; A[2] = WL[1]; A[3] = WL[2]; A[4] = WL[4];
    B[0] = WR[0]; B[1] = WR[3]; B[2] = WR[1]; B[3] = WR[2]; B[4] = WR[4];
    hllc_ordered<R, NV>(A, B, gam, inv_gm1, Fn);
    Fm[0] = Fn[0]; Fm[1] = Fn[2]; Fm[2] = Fn[3]; Fm[3] = Fn[1]; Fm[4] = Fn[4];
  }

  // Halo slot of this thread: NHALO <= NT, so each thread owns at most one
  // halo cell of the plane, at the same x-y position on every plane.
  static_assert(NHALO <= NT, "one halo cell per thread at most");
  const bool has_halo = tid < NHALO;
  int hlx = 0, hly = 0;
  bool hflx = false, hfly = false;
  long long hcol = 0;
  if (has_halo) {
    const int h = tid;
    if (NDIM >= 2) {
      if (h < 4 * TY) {
        int side = h / (2 * TY), r = h % (2 * TY);
        hly = r / 2 + 2;
        hlx = side ? TX + 2 + (r % 2) : (r % 2);
      } else {
        int hh = h - 4 * TY;
        int side = hh / (2 * TX), r = hh % (2 * TX);
        hlx = r % TX + 2;
        hly = side ? TY + 2 + r / TX : r / TX;
      }
    } else {
      hly = 0;
      hlx = h < 2 ? h : TX + h;
    }
    int qx = remap(x0 + hlx - 2, nx, a.bc[0][0], a.bc[0][1], hflx);
    int qy = NDIM >= 2 ? remap(y0 + hly - 2, ny, a.bc[1][0], a.bc[1][1], hfly) : 0;
    hcol = (long long)qy * nx + qx;
  }
  // conserved values of this thread's halo cell on the current plane; the
  // next plane's are loaded while the current plane's faces are computed
  R Hc[NV];
  if (has_halo) {
    bool f;
    load_cons(zplane(z0, f) + hcol, Hc);
  }

  for (int z = z0; z < z1; ++z) {
    // ---- 0. issue the z+2 plane's column load early
    R Unext[NV];
    bool fz_next = false;
    if (NDIM == 3) {
      long long zn = zplane(z + 2, fz_next);
      load_cons(zn + col, Unext);
    }
    if (NDIM < 3) {
      col_prim(Ucur, false, P0);
    }
    // ---- 1. primitives of plane z: interior from the window, halo from Hc
    R Hn[NV];
    if (has_halo) {
      R Wh[NV];
      to_primitive<R, NDIM>(Hc, Wh, gm1);
      if (hflx) Wh[1] = -Wh[1];
      if (NDIM >= 2 && hfly) Wh[2] = -Wh[2];
#pragma unroll
      for (int v = 0; v < NV; ++v) Ws[v * LXY + hly * LX + hlx] = Wh[v];
      if (NDIM == 3 && z + 1 < z1) {
        bool f;
        load_cons(zplane(z + 1, f) + hcol, Hn);
      }
    }
    if (owner) {
#pragma unroll
      for (int v = 0; v < NV; ++v) Ws[v * LXY + (ty + OY) * LX + tx + 2] = P0[v];
    }
    if (inside) flags |= cell_flags<R, NV>(Ucur, P0[NV - 1]);
    __syncthreads();

    // ---- 2. in-plane faces.  The normal velocity of a y face is variable
    // slot 2 and its first transverse velocity slot 1: the swap is done in
    // the LDS addresses, so one code path serves both axes.
    for (int f = tid; f < NF; f += NT) {
      int base, stride;
      bool yface = f >= NFX;
      if (!yface) {
        int fxx = f % (TX + 1), fyy = f / (TX + 1);
        base = (fyy + OY) * LX + fxx;
        stride = 1;
      } else {
        int g = f - NFX;
        int fxx = g % TX, fyy = g / TX;
        base = fyy * LX + fxx + 2;
        stride = LX;
      }
      int slot[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) slot[v] = v;
      if (NDIM >= 2) {
        slot[1] = yface ? 2 : 1;
        slot[2] = yface ? 1 : 2;
      }
      R WL[NV], WR[NV], Fn[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const R* w = Ws + slot[v] * LXY + base;
        muscl_pair(w[0], w[stride], w[2 * stride], w[3 * stride], WL[v], WR[v]);
      }
      hllc_ordered<R, NV>(WL, WR, gam, inv_gm1, Fn);
#pragma unroll
      for (int v = 0; v < NV; ++v) Fs[slot[v] * NF + f] = Fn[v];
    }

    // ---- 3. face z+1/2 from the register window
    R Fp[NV];
    R P2[NV];
    if constexpr (NDIM == 3) {
      col_prim(Unext, fz_next, P2);
      R S1[NV], A[NV], B[NV], Fn[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        R d1 = P1[v] - P0[v], d2 = P2[v] - P1[v];
        S1[v] = minmod(d1, d2);
      }
      // reorder to (rho, u_z, u_x, u_y, p)
      const int perm[5] = {0, 3, 1, 2, 4};
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        int q = perm[v];
        A[v] = P0[q] + R(0.5) * S0[q];
        B[v] = P1[q] - R(0.5) * S1[q];
      }
      hllc_ordered<R, NV>(A, B, gam, inv_gm1, Fn);
#pragma unroll
      for (int v = 0; v < NV; ++v) Fp[perm[v]] = Fn[v];
#pragma unroll
      for (int v = 0; v < NV; ++v) S0[v] = S1[v];
    }
    __syncthreads();

    // ---- 4. flux difference and stage combine
    if (inside) {
      long long c = (long long)z * nx * ny + (long long)gy * nx + gx;
      const int fxl = ty * (TX + 1) + tx;
      const int fyl = NFX + ty * TX + tx;
      R Out[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        R l = R(0) - (Fs[v * NF + fxl + 1] - Fs[v * NF + fxl]) * idx0;
        if (NDIM >= 2) l = l - (Fs[v * NF + fyl + TX] - Fs[v * NF + fyl]) * idx1;
        if (NDIM == 3) l = l - (Fp[v] - Fm[v]) * idx2;
        if (STAGE == 1) {
          Out[v] = Ucur[v] + dt * l;
        } else {
          R u0 = un[v * N + c];
          Out[v] = R(0.5) * (u0 + (Ucur[v] + dt * l));
        }
      }
#pragma unroll
      for (int v = 0; v < NV; ++v) dst[v * N + c] = Out[v];
      if (STAGE == 2 && a.fuse_cfl) {
        double Ud[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) Ud[v] = (double)Out[v];
        smax = fmax(smax, signal_sum<NDIM>(Ud, a.dx, a.gamma));
      }
    }

    // ---- 5. slide the window
    if (NDIM == 3) {
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        Fm[v] = Fp[v];
        P0[v] = P1[v];
        P1[v] = P2[v];
        Ucur[v] = Uc1[v];
        Uc1[v] = Unext[v];
        Hc[v] = Hn[v];
      }
    }
  }

}

}  // namespace hard
