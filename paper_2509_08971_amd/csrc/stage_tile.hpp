// One tile of a Heun stage: the shared body of the single-grid stage kernel
// and the batched kernels (HARD paper section 2.2.2: finite-volume face
// difference, Heun's Butcher tableau in Shu-Osher form).
//
// A tile is a plane of cells held in LDS that walks along the last axis:
//   1D: a row of TX cells in x (no walk);
//   2D: a row of TX cells in x walking along y over [w0, w1) (TY = 1), or a
//       TX x TY tile in x-y that does not walk (TY > 1: small grids, which
//       the walk would cut into too few waves);
//   3D: a TX x TY tile in x-y walking along z over [w0, w1).
// For each position of the walk it
//   1. puts the primitive states of the plane plus a two-cell halo in LDS
//      (the thread's own cell comes from a register window along the walk
//      axis, the halo cells were loaded during the previous position; ghost
//      cells are produced by index remapping, so no ghost arrays exist),
//   2. computes every in-plane face flux once, into LDS,
//   3. computes the face ahead along the walk axis from the register window
//      (the face behind was computed at the previous position),
//   4. forms L(U) and the stage combine, and stores the cell once.
// Each cell is read from memory once per stage (plus the halo re-reads of
// neighbouring tiles, which are served by L2), written once.
#pragma once

#include <type_traits>

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
  int dx_pow2;      // every dx is a power of two: x / dx == x * (1/dx) exactly
  double gamma;
  double dt;
  int x0, y0;       // tile origin (y0: 3D only)
  int w0, w1;       // walk range (y in 2D, z in 3D; [0, 1) in 1D)
  int fuse_cfl;     // stage 2: accumulate the CFL signal max of the output
  int exchange;     // stage 2 with RAD: the heating/cooling exchange of each
                    // new cell state before it is stored
  double kappa, mu;
};

// Streams that no other workgroup reads again within the launch -- the
// stored result and, in stage 2, U^n of the own cell -- can go through the
// cache as non-temporal accesses (NTS), so that they do not push the halo
// lines that neighbouring tiles re-read out of the XCD's L2.  That pays for
// 3D tiles, whose rows are whole 128-byte lines; the batched kernels store
// 63-cell rows that straddle lines, which the L2 must merge before they
// reach memory, so they keep ordinary stores.
template <bool NTS, typename R>
__device__ __forceinline__ R stream_load(const R* p) {
  if constexpr (NTS) return __builtin_nontemporal_load(p);
  else return *p;
}
template <bool NTS, typename R>
__device__ __forceinline__ void stream_store(R* p, R v) {
  if constexpr (NTS) __builtin_nontemporal_store(v, p);
  else *p = v;
}

// RAD: the state carries the radiation energy density E_r as field NDIM + 2,
// advected in the same pass (see rusanov_er).
template <int NDIM, typename R, int TX, int TY, bool RAD = false>
struct TileShape {
  static constexpr int NH = NDIM + 2;            // hydro fields
  static constexpr int NV = NH + (RAD ? 1 : 0);  // fields carried through the tile
  static constexpr int PD = (NDIM == 3 || TY > 1) ? 2 : 1;  // dimensions of the plane in LDS
  static constexpr bool WALK = NDIM == 3 || (NDIM == 2 && TY == 1);
  static constexpr int LX = TX + 4;
  static constexpr int LY = PD == 2 ? TY + 4 : 1;
  static constexpr int LXY = LX * LY;
  static constexpr int NFX = (TX + 1) * TY;                // x faces per plane
  static constexpr int NFY = PD == 2 ? TX * (TY + 1) : 0;  // y faces per plane (3D)
  static constexpr int NF = NFX + NFY;
  static constexpr int NHALO = PD == 2 ? 4 * (TX + TY) : 4;
  // FP64 3D: the flux through the face below each cell along the walk axis
  // lives in LDS instead of registers (10 VGPRs fewer at the peak)
  static constexpr bool FZ_LDS = WALK && PD == 2 && sizeof(R) == 8;
  static constexpr int lds_elems = NV * (LXY + NF) + (FZ_LDS ? NV * TX * TY : 0);
  static_assert(NDIM >= 2 || TY == 1, "1D planes are one row");
};

// Runs one tile; ORs status bits into `flags` and maxes the CFL signal sum of
// the stored cells into `smax` (when a.fuse_cfl).  Every thread of the
// workgroup must call it (it contains barriers).  NTHR (>= TX*TY) is the
// workgroup size; threads beyond TX*TY own no cell but take part in the face
// and halo loops (a row of 63 cells has exactly 64 faces, one per lane).
template <int NDIM, typename R, int STAGE, int TX, int TY, int NTHR = TX * TY, bool NTS = false,
          bool RAD = false>
__device__ __forceinline__ void run_tile(const TileArgs& a, R* lds, unsigned& flags, double& smax) {
  using S = TileShape<NDIM, R, TX, TY, RAD>;
  constexpr int NV = S::NV, NH = S::NH, PD = S::PD, LX = S::LX, LXY = S::LXY;
  constexpr int NFX = S::NFX, NF = S::NF, NHALO = S::NHALO;
  constexpr bool WALK = S::WALK;
  constexpr int WA = NDIM - 1;          // walk axis
  constexpr int OY = PD == 2 ? 2 : 0;   // LDS row of the tile's first row
  constexpr int NT = NTHR;
  static_assert(NTHR >= TX * TY, "one thread per cell at least");
  static_assert(NHALO <= NT, "one halo cell per thread at most");

  R* Ws = lds;             // NV * LXY: primitives of the plane (tile + halo)
  R* Fs = lds + NV * LXY;  // NV * NF: in-plane face fluxes, x faces then y faces
  // (FZ_LDS) the walk-axis flux below each owner cell; each thread reads and
  // writes only its own slots, so no barrier guards them
  R* Fz = lds + NV * (LXY + NF);
  constexpr bool FZ_LDS = S::FZ_LDS;

  const int tid = threadIdx.x;
  const bool owner = NT == TX * TY || tid < TX * TY;  // this thread owns a cell column of the tile
  const int tx = owner ? tid % TX : 0, ty = owner ? tid / TX : 0;
  const int nx = a.n[0], ny = a.n[1], nz = a.n[2];
  const long long N = (long long)nx * ny * nz;
  const int nwalk = NDIM == 3 ? nz : (NDIM == 2 ? ny : 1);
  const long long WS = NDIM == 3 ? (long long)nx * ny : nx;  // stride along the walk axis

  const int x0 = a.x0, y0 = a.y0;
  const int gx = x0 + tx, gy = PD == 2 ? y0 + ty : 0;
  const bool inside = owner && gx < nx && (PD == 1 || gy < ny);
  const int w0 = a.w0, w1 = a.w1;

  // src never aliases dst (the stage state lives in its own buffer); un and
  // dst may be the same array, each thread reading its own cell before
  // storing it, so neither of them is restrict.
  const R* __restrict__ src = static_cast<const R*>(a.src);
  const R* un = static_cast<const R*>(a.un);
  R* dst = static_cast<R*>(a.dst);
  const double gm1 = a.gamma - 1.0;
  const R gam = R(a.gamma);
  const R inv_gm1 = R(1.0 / gm1);
  const R dt = R(a.dt);
  const R idx0 = R(a.inv_dx[0]), idx1 = R(a.inv_dx[1]), idxw = R(a.inv_dx[WA]);

  // this thread's column, clamped (and mirrored past reflecting walls) for
  // the overhang of ragged tiles; such threads never store
  bool fx_ = false, fy_ = false;
  const int cx = remap(gx, nx, a.bc[0][0], a.bc[0][1], fx_);
  const int cy = PD == 2 ? remap(gy, ny, a.bc[1][0], a.bc[1][1], fy_) : 0;
  const long long col = (long long)cy * nx + cx;

  // offset of walk position q (ghost-mapped along the walk axis)
  auto wplane = [&](int q, bool& fw) -> long long {
    fw = false;
    if constexpr (!WALK) {
      return 0;
    } else {
      int w = remap(q, nwalk, a.bc[WA][0], a.bc[WA][1], fw);
      return (long long)w * WS;
    }
  };
  auto load_cons = [&](long long c, R* Uc) {
#pragma unroll
    for (int v = 0; v < NV; ++v) Uc[v] = src[v * N + c];
  };
  // primitive state of this thread's column from conserved values (E_r, if
  // carried, is its own primitive)
  auto col_prim = [&](const R* Uc, bool fw, R* W) {
    to_primitive<R, NDIM>(Uc, W, gm1);
    if constexpr (RAD) W[NH] = Uc[NH];
    if (fx_) W[1] = -W[1];
    if (PD == 2 && fy_) W[2] = -W[2];
    if (WALK && fw) W[1 + WA] = -W[1 + WA];
  };
  // variable order of a face normal to the walk axis: (rho, u_n, u_t..., p
  // [, E_r])
  constexpr int wperm[6] = {0, 1 + WA, 1, NDIM == 3 ? 2 : NH - 1, NDIM == 3 ? NH - 1 : NH, NH};
  // flux of a face from its states in face order: HLLC for the hydro fields,
  // the Rusanov flux of E_r beside it
  auto face_flux = [&](const R* A, const R* B, R* Fn) {
    hllc_ordered<R, NH>(A, B, gam, inv_gm1, Fn);
    if constexpr (RAD) Fn[NH] = rusanov_er<R, NH>(A, B, gam);
  };

  // walk-axis register window: P0 = position w, P1 = w+1, S0 = slope at w,
  // Fm = flux through the face w-1/2; conserved values Ucur (w) and Uc1 (w+1)
  R P0[NV], P1[NV], S0[NV], Fm[FZ_LDS ? 1 : NV];
  auto fz_get = [&](int v) -> R {
    if constexpr (FZ_LDS) return Fz[v * (TX * TY) + tid];
    else return Fm[v];
  };
  auto fz_set = [&](int v, R x) {
    if constexpr (FZ_LDS) {
      if (owner) Fz[v * (TX * TY) + tid] = x;
    } else {
      Fm[v] = x;
    }
  };
  R Ucur[NV], Uc1[NV];
  if constexpr (!WALK) load_cons(col, Ucur);
  if constexpr (WALK) {
    R Pm2[NV], Pm1[NV], Ut[NV];
    bool fw;
    long long wo;
    wo = wplane(w0 - 2, fw); load_cons(wo + col, Ut); col_prim(Ut, fw, Pm2);
    wo = wplane(w0 - 1, fw); load_cons(wo + col, Ut); col_prim(Ut, fw, Pm1);
    wo = wplane(w0, fw);     load_cons(wo + col, Ucur); col_prim(Ucur, fw, P0);
    wo = wplane(w0 + 1, fw); load_cons(wo + col, Uc1); col_prim(Uc1, fw, P1);
    R A[NV], B[NV], Fn[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) S0[v] = minmod(P0[v] - Pm1[v], P1[v] - P0[v]);
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      const int q = wperm[k];
      R sm1 = minmod(Pm1[q] - Pm2[q], P0[q] - Pm1[q]);
      A[k] = Pm1[q] + R(0.5) * sm1;
      B[k] = P0[q] - R(0.5) * S0[q];
    }
    face_flux(A, B, Fn);
#pragma unroll
    for (int k = 0; k < NV; ++k) fz_set(wperm[k], Fn[k]);
  }

  // Halo slot of this thread: NHALO <= NT, so each thread owns at most one
  // halo cell of the plane, at the same in-plane position on every plane.
  const bool has_halo = tid < NHALO;
  int hlx = 0, hly = 0;
  bool hflx = false, hfly = false;
  long long hcol = 0;
  if (has_halo) {
    const int h = tid;
    if constexpr (PD == 2) {
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
    int qy = PD == 2 ? remap(y0 + hly - 2, ny, a.bc[1][0], a.bc[1][1], hfly) : 0;
    hcol = (long long)qy * nx + qx;
  }
  // conserved values of this thread's halo cell at the current position; the
  // next position's are loaded while the current plane's faces are computed
  R Hc[NV];
  if (has_halo) {
    bool f;
    load_cons(wplane(w0, f) + hcol, Hc);
  }

  for (int w = w0; w < w1; ++w) {
    // ---- 0. issue the loads this position needs later: the column two
    // positions ahead, and (stage 2) U^n of this thread's cell
    R Unext[NV], Un0[NV];
    bool fw_next = false;
    if constexpr (WALK) load_cons(wplane(w + 2, fw_next) + col, Unext);
    const long long cidx = (long long)w * WS + col;
    if (STAGE == 2 && inside) {
#pragma unroll
      for (int v = 0; v < NV; ++v) Un0[v] = stream_load<NTS>(un + v * N + cidx);
    }
    if constexpr (!WALK) col_prim(Ucur, false, P0);

    // ---- 1. primitives of the plane: own cell from the window, halo from Hc
    R Hn[NV];
    if (has_halo) {
      R Wh[NV];
      to_primitive<R, NDIM>(Hc, Wh, gm1);
      if constexpr (RAD) Wh[NH] = Hc[NH];
      if (hflx) Wh[1] = -Wh[1];
      if (PD == 2 && hfly) Wh[2] = -Wh[2];
#pragma unroll
      for (int v = 0; v < NV; ++v) Ws[v * LXY + hly * LX + hlx] = Wh[v];
      if (WALK && w + 1 < w1) {
        bool f;
        load_cons(wplane(w + 1, f) + hcol, Hn);
      }
    }
    if (owner) {
#pragma unroll
      for (int v = 0; v < NV; ++v) Ws[v * LXY + (ty + OY) * LX + tx + 2] = P0[v];
    }
    if (inside) flags |= cell_flags<R, NV>(Ucur, P0[NH - 1]);
    __syncthreads();
    // The in-plane faces are the phase every wave of the workgroup waits on
    // at the next barrier: they issue at a raised priority over the waves of
    // the other workgroups on the SIMD, which are between barriers of their
    // own (measured 1.4% faster per FP64 step, 0.8% FP32).
    __builtin_amdgcn_s_setprio(2);

    // ---- 2. in-plane faces.  Each owner thread takes the low x face of
    // its cell (and, in 3D, the low y face); the far faces (x = TX of every
    // row, y = TY of every column) go to the threads that own no cell, or to
    // a short third round.  In 3D the normal velocity of a y face is
    // variable slot 2 and its first transverse velocity slot 1: the swap is
    // done in the LDS addresses, so one code path serves both axes.
    auto face = [&](int base, int fidx, auto yface_c) {
      constexpr bool YF = decltype(yface_c)::value;
      constexpr int stride = YF ? LX : 1;
      R WL[NV], WR[NV], Fn[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const int sv = (PD == 2 && YF && (v == 1 || v == 2)) ? 3 - v : v;
        const R* wp = Ws + sv * LXY + base;
        muscl_pair(wp[0], wp[stride], wp[2 * stride], wp[3 * stride], WL[v], WR[v]);
      }
      face_flux(WL, WR, Fn);
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const int sv = (PD == 2 && YF && (v == 1 || v == 2)) ? 3 - v : v;
        Fs[sv * NF + fidx] = Fn[v];
      }
    };
    using XF = std::integral_constant<bool, false>;
    using YF = std::integral_constant<bool, true>;
    if constexpr (PD == 1) {
      // a row: TX + 1 faces, face f between tile cells f - 1 and f
      for (int f = tid; f < TX + 1; f += NT) face(f, f, XF{});
    } else {
      constexpr int NSPARE = NT - TX * TY;
      const int sp = tid - TX * TY;  // spare-thread index (< 0 for owners)
      if (owner) face((ty + OY) * LX + tx, ty * (TX + 1) + tx, XF{});
      else if (sp < TY) face((sp + OY) * LX + TX, sp * (TX + 1) + TX, XF{});
      if (owner) face(ty * LX + tx + 2, NFX + ty * TX + tx, YF{});
      else if (sp < TX) face(TY * LX + sp + 2, NFX + TY * TX + sp, YF{});
      if constexpr (NSPARE < TY || NSPARE < TX) {
        // far faces the spare threads did not cover
        constexpr int RX = NSPARE < TY ? TY - NSPARE : 0;
        constexpr int RY = NSPARE < TX ? TX - NSPARE : 0;
        const int wv = tid >> 6, ln = tid & 63;
        if constexpr (RX + RY <= 64 && sizeof(R) == 8) {
          // FP64: all far faces on wave 0 in one pass, the axis chosen per
          // lane (x faces on the first RX lanes): one wave computes one extra
          // face (measured 2% faster per step than one wave per axis)
          if (wv == 0 && ln < RX + RY) {
            const bool yf = ln >= RX;
            const int j = NSPARE + (yf ? ln - RX : ln);
            const int base = yf ? TY * LX + j + 2 : (j + OY) * LX + TX;
            const int fidx = yf ? NFX + TY * TX + j : j * (TX + 1) + TX;
            const int stride = yf ? LX : 1;
            R WL[NV], WR[NV], Fn[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) {
              const int sv = (PD == 2 && yf && (v == 1 || v == 2)) ? 3 - v : v;
              const R* wp = Ws + sv * LXY + base;
              muscl_pair(wp[0], wp[stride], wp[2 * stride], wp[3 * stride], WL[v], WR[v]);
            }
            face_flux(WL, WR, Fn);
#pragma unroll
            for (int v = 0; v < NV; ++v) {
              const int sv = (PD == 2 && yf && (v == 1 || v == 2)) ? 3 - v : v;
              Fs[sv * NF + fidx] = Fn[v];
            }
          }
        } else {
          // the x far faces on wave 0, the y far faces on wave 1: no wave
          // computes two faces in this round (the others would wait for it at
          // the barrier), and only two waves spend the round's instructions.
          // FP32 keeps this form: the per-lane axis choice costs it registers
          // (128 instead of 96, one wave per SIMD fewer).
          constexpr int NW = NT / 64;
          static_assert(NW >= 2, "far-face split needs two waves");
          constexpr int FW = 2;  // waves that take far faces
          constexpr int PX = (RX + FW / 2 - 1) / (FW / 2), PY = (RY + FW / 2 - 1) / (FW / 2);
          static_assert(PX <= 64 && PY <= 64, "one far face per lane");
          if (wv < FW / 2) {
            const int r = wv * PX + ln;
            if (ln < PX && r < RX) {
              const int j = NSPARE + r;
              face((j + OY) * LX + TX, j * (TX + 1) + TX, XF{});
            }
          } else if (wv < FW) {
            const int r = (wv - FW / 2) * PY + ln;
            if (ln < PY && r < RY) {
              const int j = NSPARE + r;
              face(TY * LX + j + 2, NFX + TY * TX + j, YF{});
            }
          }
        }
      }
    }

    __builtin_amdgcn_s_setprio(0);
    // ---- 3. face w+1/2 from the register window
    R Fp[NV];
    R P2[NV];
    if constexpr (WALK) {
      col_prim(Unext, fw_next, P2);
      R S1[NV], A[NV], B[NV], Fn[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) S1[v] = minmod(P1[v] - P0[v], P2[v] - P1[v]);
#pragma unroll
      for (int k = 0; k < NV; ++k) {
        const int q = wperm[k];
        A[k] = P0[q] + R(0.5) * S0[q];
        B[k] = P1[q] - R(0.5) * S1[q];
      }
      face_flux(A, B, Fn);
#pragma unroll
      for (int k = 0; k < NV; ++k) Fp[wperm[k]] = Fn[k];
#pragma unroll
      for (int v = 0; v < NV; ++v) S0[v] = S1[v];
    }
    __syncthreads();

    // ---- 4. flux difference (x, then y, then z) and stage combine
    if (inside) {
      const int fxl = ty * (TX + 1) + tx;
      const int fyl = NFX + ty * TX + tx;
      R Out[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        R l = R(0) - (Fs[v * NF + fxl + 1] - Fs[v * NF + fxl]) * idx0;
        if (PD == 2) l = l - (Fs[v * NF + fyl + TX] - Fs[v * NF + fyl]) * idx1;
        if (WALK) l = l - (Fp[v] - fz_get(v)) * idxw;
        if (STAGE == 1) {
          Out[v] = Ucur[v] + dt * l;
        } else {
          Out[v] = R(0.5) * (Un0[v] + (Ucur[v] + dt * l));
        }
      }
      // RAD, stage 2: the heating/cooling exchange of the new state before
      // it is stored (and before its CFL signal)
      if constexpr (RAD && STAGE == 2) {
        if (a.exchange) flags |= exchange_cell<R, NDIM>(Out, a.dt, a.gamma, a.kappa, a.mu);
      }
#pragma unroll
      for (int v = 0; v < NV; ++v) stream_store<NTS>(dst + v * N + cidx, Out[v]);
      if (STAGE == 2 && a.fuse_cfl) {
        double Ud[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) Ud[v] = (double)Out[v];
        smax = fmax(smax, cfl_signal<R, NDIM>(Ud, a.inv_dx, a.gamma));
      }
    }

    // ---- 5. slide the window
    if constexpr (WALK) {
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        fz_set(v, Fp[v]);
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
