// Implicit flux-limited radiation diffusion solved by geometric multigrid
// (section 2.2.1: the diffusion term of the radiation energy equation with
// D = c lambda / (kappa rho) and the Levermore limiter; section 2.2.2: the
// multigrid solver of A u = f, the residual equation on the coarse grids and
// the V-cycle).
//
// One call advances E_r by one backward-Euler step of d_t E = div(D grad E)
// with D frozen at the start of the step, so that
//     A E_new = E_old,   (A x)_c = x_c + sum_faces a_f (x_c - x_nb),
//     a_f = dt (D_c + D_nb)/2 / dx_d^2
// (zero-flux walls on non-periodic sides), and solves it by `ncycles`
// V-cycles from E_old:
//
//   fld_setup      per cell: grad E by central differences, R, lambda, D;
//                  b = x = E_old; status bits
//   fld_coarsen_D  per coarse cell: D = mean of its children's D
//   fld_relax      one red-black half-sweep (Gauss-Seidel on one colour:
//                  every cell of a colour depends only on the other colour,
//                  so the half-sweep is one parallel pass in any order)
//   fld_restrict   per coarse cell: the fine residual b - A x averaged over
//                  the children -> coarse b; coarse x = 0 (fld_restrict_tile
//                  and fld_restrict_red: the same from an LDS tile of fine
//                  residuals; the latter computes only the red ones, the black
//                  residuals being zero after a black half-sweep)
//   fld_prolong    per fine cell: x += linear interpolation of the coarse x
//                  (weights 3/4, 1/4 along each halved axis, the edge value
//                  repeated beyond a wall); fld_prolong_colour: the black
//                  cells only, when a red half-sweep follows
//   fld_vcycle_tail  the V-cycle below the first level that fits in one
//                  workgroup's LDS, in one launch
//   fld_store      the finest x back into the state's E_r field
//   fld_resid_sq   per tile the sum of (b - A x)^2; fld_resid_final adds the
//                  tile sums in a fixed order (deterministic)
//
// Every level keeps x, b and D colour-split (the red cells, then the black
// ones, each colour packed two-to-one along x), so that a half-sweep reads
// the other colour's x, its own b and both colours' D as contiguous streams
// and writes its own x: 20 bytes per cell instead of the 32 that the natural
// layout costs (every line of x, b and D is touched to update half of them).

// Coarsening halves every axis whose size is even; a periodic axis only
// while the half is even or one, so that the red-black colouring stays
// consistent across the periodic seam.  The coarsest level is relaxed
// `ncoarse` sweeps from zero (one cell: A = [1], exact in one sweep).
//
// Plain arithmetic throughout (IEEE division and square root, no
// contraction), in the order the formulas above are written; the zero black
// residuals of fld_restrict_red are the one departure from evaluating each
// formula as written.  These kernels
// stream a few arrays and do a handful of flops per cell: they are bound by
// memory, not by arithmetic.

#include <algorithm>
#include <cmath>
#include <cstring>
#include <type_traits>

#include "../../include/hard.h"
#include "api_internal.hpp"
#include "hydro_device.hpp"

namespace hard {

constexpr double FLD_C_LIGHT = 2.99792458e10;  // cm/s
constexpr int FLD_MAX_LEVELS = 40;

// One multigrid level.  Every array (x, b, D) is stored colour-split: the
// red cells (i + j + k even) of all rows first, then the black ones; within
// a colour, row (j, k) holds its cells i at slot i / 2 (hx = ceil(nx / 2)
// slots per row; when nx is odd one colour leaves the last slot unused).
// A red-black half-sweep then streams contiguous arrays: the cells it
// updates, their right-hand sides, and the other colour's values.
// Indices are 32-bit: a level has fewer than 2^31 cells, so a colour-split
// array has fewer than 2^32 elements.
struct FldLevel {
  int n[3];
  int halved[3];   // axis halved from the next finer level
  unsigned hx;     // slots per row and colour
  unsigned cs;     // elements per colour: n[1] n[2] hx
  double dx[3];    // cell width
  double dx2[3];   // dx_d * dx_d
  const double* K; // device: K_d = (dt/2) / dx_d^2 of this level (3 doubles)
  double* x;
  double* b;
  double* D;
};

struct FldCommon {
  int per[3];          // periodic axis
  const double* dt;    // device dt
};

// Neighbour of p on an axis of n cells on side s (0 low, 1 high), or -1 when
// the face carries no flux (a wall, or a periodic axis of one cell).
__device__ __forceinline__ int fld_nb(int p, int n, int s, int periodic) {
  if (s == 0) {
    if (p > 0) return p - 1;
    return periodic && n > 1 ? n - 1 : -1;
  }
  if (p < n - 1) return p + 1;
  return periodic && n > 1 ? 0 : -1;
}

// Colour-split index of cell (i, j, k).
__device__ __forceinline__ unsigned fld_at(const FldLevel& L, int i, int j, int k) {
  return (((i + j + k) & 1) ? L.cs : 0u) + ((unsigned)k * (unsigned)L.n[1] + (unsigned)j) * L.hx +
         ((unsigned)i >> 1);
}

// Natural-order cell index -> (i, j, k)
__device__ __forceinline__ void fld_cell(const FldLevel& L, unsigned c, int* p) {
  const unsigned nx = L.n[0], ny = L.n[1];
  const unsigned row = c / nx;
  p[0] = (int)(c - row * nx);
  p[1] = (int)(row % ny);
  p[2] = (int)(row / ny);
}

__device__ __forceinline__ unsigned fld_cells(const FldLevel& L) {
  return (unsigned)L.n[0] * (unsigned)L.n[1] * (unsigned)L.n[2];
}

// The 2 NDIM face neighbours of cell (i, j, k) (row = k n1 + j), all of the
// other colour: their colour-split indices, read straight from the layout
// (x: slot (i -+ 1)/2 of the same row; y, z: slot i/2 of the rows +-1 and
// +-n1), and whether each face is open.  A closed face (wall, or a periodic
// axis of one cell) still gets an in-range index, so every load is
// unconditional and a cell's loads are all in flight together; the
// coefficient of a closed face is zeroed by a select.
template <int NDIM>
__device__ __forceinline__ void fld_faces(const FldLevel& L, const FldCommon& cm, int i, int j,
                                          int k, unsigned row, unsigned* nb, bool* open) {
  const unsigned hx = L.hx;
  const unsigned ob = (((i + j + k) & 1) ? 0u : L.cs) + row * hx;  // other colour, this row
  const unsigned o = ob + ((unsigned)i >> 1);
  const int nx = L.n[0];
  {
    const bool lo = i > 0, hi = i < nx - 1, wrap = cm.per[0] && nx > 1;
    nb[0] = ob + (lo ? (unsigned)(i - 1) >> 1 : (unsigned)(nx - 1) >> 1);
    nb[1] = ob + (hi ? (unsigned)(i + 1) >> 1 : 0u);
    open[0] = lo || wrap;
    open[1] = hi || wrap;
  }
  if (NDIM > 1) {
    const int ny = L.n[1];
    const bool lo = j > 0, hi = j < ny - 1, wrap = cm.per[1] && ny > 1;
    const unsigned span = (unsigned)(ny - 1) * hx;
    nb[2] = lo ? o - hx : o + span;
    nb[3] = hi ? o + hx : o - span;
    open[2] = lo || wrap;
    open[3] = hi || wrap;
  }
  if (NDIM > 2) {
    const int nz = L.n[2];
    const unsigned ps = (unsigned)L.n[1] * hx;
    const bool lo = k > 0, hi = k < nz - 1, wrap = cm.per[2] && nz > 1;
    const unsigned span = (unsigned)(nz - 1) * ps;
    nb[4] = lo ? o - ps : o + span;
    nb[5] = hi ? o + ps : o - span;
    open[4] = lo || wrap;
    open[5] = hi || wrap;
  }
}

// (A x) at cell p = (i, j, k) of level L: x_c + sum over open faces, in the
// order x low, x high, y low, ..., of a_f (x_c - x_nb), a_f = (D_c + D_nb) K_d.
// A closed face adds exactly zero.
template <int NDIM>
__device__ __forceinline__ double fld_apply_row(const FldLevel& L, const FldCommon& cm,
                                                const int* p) {
#pragma clang fp contract(off)
  constexpr int NF = 2 * NDIM;
  const unsigned row = (unsigned)p[2] * (unsigned)L.n[1] + (unsigned)p[1];
  const unsigned c = (((p[0] + p[1] + p[2]) & 1) ? L.cs : 0u) + row * L.hx + ((unsigned)p[0] >> 1);
  unsigned nb[NF];
  bool open[NF];
  fld_faces<NDIM>(L, cm, p[0], p[1], p[2], row, nb, open);
  const double xc = L.x[c], Dc = L.D[c];
  double Dn[NF], xn[NF];
#pragma unroll
  for (int f = 0; f < NF; ++f) {
    Dn[f] = L.D[nb[f]];
    xn[f] = L.x[nb[f]];
  }
  double Ax = xc;
#pragma unroll
  for (int f = 0; f < NF; ++f) {
    const double a = open[f] ? (Dc + Dn[f]) * L.K[f >> 1] : 0.0;
    Ax += a * (open[f] ? xc - xn[f] : 0.0);
  }
  return Ax;
}

// Gauss-Seidel update of cell (i, j, k) of colour `colour` (row = k n1 + j,
// slot h = i / 2): x_c = (b_c + sum_faces a_f x_nb) / (1 + sum_faces a_f),
// open faces in the order x low, x high, y low, ...; a closed face adds
// exactly zero.
template <int NDIM>
__device__ __forceinline__ void fld_relax_cell(const FldLevel& L, const FldCommon& cm, int colour,
                                               int i, int j, int k, unsigned row) {
#pragma clang fp contract(off)
  constexpr int NF = 2 * NDIM;
  const unsigned c = (colour ? L.cs : 0u) + row * L.hx + ((unsigned)i >> 1);
  unsigned nb[NF];
  bool open[NF];
  fld_faces<NDIM>(L, cm, i, j, k, row, nb, open);
  const double Dc = L.D[c];
  const double bc = L.b[c];
  double Dn[NF], xn[NF];
#pragma unroll
  for (int f = 0; f < NF; ++f) {
    Dn[f] = L.D[nb[f]];
    xn[f] = L.x[nb[f]];
  }
  double num = bc;
  double den = 1.0;
#pragma unroll
  for (int f = 0; f < NF; ++f) {
    const double a = open[f] ? (Dc + Dn[f]) * L.K[f >> 1] : 0.0;
    num += a * (open[f] ? xn[f] : 0.0);
    den += a;
  }
  L.x[c] = num / den;
}

// The cell at slot t of colour `colour` (t = row hx + h).
template <int NDIM>
__device__ __forceinline__ void fld_relax_slot(const FldLevel& L, const FldCommon& cm, int colour,
                                               unsigned t) {
  const unsigned h = t % L.hx;
  const unsigned row = t / L.hx;
  const int j = (int)(row % (unsigned)L.n[1]), k = (int)(row / (unsigned)L.n[1]);
  const int i = 2 * (int)h + ((j + k + colour) & 1);
  if (i >= L.n[0]) return;
  fld_relax_cell<NDIM>(L, cm, colour, i, j, k, row);
}

// Children of a coarse cell: along a halved axis 2I and 2I+1, else I.
__device__ __forceinline__ void fld_children(const FldLevel& C, const int* P, int* lo, int* cnt) {
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    lo[d] = C.halved[d] ? 2 * P[d] : P[d];
    cnt[d] = C.halved[d] ? 2 : 1;
  }
}

// Coarse cell P: b = mean over the children of the fine residual, x = 0.
template <int NDIM>
__device__ __forceinline__ void fld_restrict_cell(const FldLevel& F, const FldLevel& C,
                                                  const FldCommon& cm, double inv, const int* P) {
#pragma clang fp contract(off)
  int lo[3], cnt[3];
  fld_children(C, P, lo, cnt);
  double s = 0.0;
  for (int dz = 0; dz < cnt[2]; ++dz)
    for (int dy = 0; dy < cnt[1]; ++dy)
      for (int dx = 0; dx < cnt[0]; ++dx) {
        const int p[3] = {lo[0] + dx, lo[1] + dy, lo[2] + dz};
        const double r = F.b[fld_at(F, p[0], p[1], p[2])] - fld_apply_row<NDIM>(F, cm, p);
        s += r;
      }
  const unsigned cc = fld_at(C, P[0], P[1], P[2]);
  C.b[cc] = s * inv;
  C.x[cc] = 0.0;
}

// Fine cell f: x += linear interpolation of the coarse x.
__device__ __forceinline__ void fld_prolong_cell(const FldLevel& F, const FldLevel& C,
                                                 const FldCommon& cm, const int* f) {
#pragma clang fp contract(off)
  int nr[3], fr[3], cnt[3];
  double wn[3], wf[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    if (!C.halved[d]) {
      nr[d] = fr[d] = f[d];
      wn[d] = 1.0;
      wf[d] = 0.0;
      cnt[d] = 1;
      continue;
    }
    const int I = f[d] >> 1;
    int q = fld_nb(I, C.n[d], f[d] & 1, cm.per[d]);
    if (q < 0) q = I;
    nr[d] = I;
    fr[d] = q;
    wn[d] = 0.75;
    wf[d] = 0.25;
    cnt[d] = 2;
  }
  double v = 0.0;
  for (int cz = 0; cz < cnt[2]; ++cz)
    for (int cy = 0; cy < cnt[1]; ++cy)
      for (int cx = 0; cx < cnt[0]; ++cx) {
        const double w = (cx ? wf[0] : wn[0]) * (cy ? wf[1] : wn[1]) * (cz ? wf[2] : wn[2]);
        const double xc = C.x[fld_at(C, cx ? fr[0] : nr[0], cy ? fr[1] : nr[1], cz ? fr[2] : nr[2])];
        v += w * xc;
      }
  F.x[fld_at(F, f[0], f[1], f[2])] += v;
}

// fld_prolong_cell when every active axis is halved: the 2^NDIM coarse
// values are loaded together, then summed in the same order and with the
// same weights.
template <int NDIM>
__device__ __forceinline__ void fld_prolong_cell_all(const FldLevel& F, const FldLevel& C,
                                                     const FldCommon& cm, const int* f) {
#pragma clang fp contract(off)
  constexpr int NC = 1 << NDIM;
  int nr[3] = {0, 0, 0}, fr[3] = {0, 0, 0};
#pragma unroll
  for (int d = 0; d < NDIM; ++d) {
    const int I = f[d] >> 1;
    const int q = fld_nb(I, C.n[d], f[d] & 1, cm.per[d]);
    nr[d] = I;
    fr[d] = q < 0 ? I : q;
  }
  double xc[NC];
#pragma unroll
  for (int m = 0; m < NC; ++m)
    xc[m] = C.x[fld_at(C, (m & 1) ? fr[0] : nr[0], (m & 2) ? fr[1] : nr[1], (m & 4) ? fr[2] : nr[2])];
  double v = 0.0;
#pragma unroll
  for (int m = 0; m < NC; ++m) {
    const double w = ((m & 1) ? 0.25 : 0.75) * (NDIM > 1 ? ((m & 2) ? 0.25 : 0.75) : 1.0) *
                     (NDIM > 2 ? ((m & 4) ? 0.25 : 0.75) : 1.0);
    v += w * xc[m];
  }
  const unsigned c = fld_at(F, f[0], f[1], f[2]);
  F.x[c] += v;
}

// Block tile of the natural-order kernels: 256 cells, TX x TY x TZ.
template <int NDIM> struct FldTile;
template <> struct FldTile<1> { static constexpr int TX = 256, TY = 1, TZ = 1; };
template <> struct FldTile<2> { static constexpr int TX = 64, TY = 4, TZ = 1; };
template <> struct FldTile<3> { static constexpr int TX = 32, TY = 4, TZ = 2; };

// Tile rows (along y) of one panel: tile ids run x fastest, then y inside the
// panel, then z, then panel.  The z neighbours of a tile were then touched one
// panel slab earlier (TX*tx x TY*FLD_PANEL x TZ cells, about 0.2 MB of x, b
// and D at 256 cells in x), well inside one XCD's 4 MB L2; in plain x-y-z
// order they were a full x-y slab earlier and came from HBM again.
constexpr unsigned FLD_PANEL = 4;

// Tiles of 512 cells for the kernels that work on one colour (half-sweep,
// red residuals, prolongation into the black cells): one thread per cell of
// that colour, so a wave covers 32 slots of two rows.
template <int NDIM> struct FldColourTile;
template <> struct FldColourTile<1> { static constexpr int TX = 512, TY = 1, TZ = 1; };
template <> struct FldColourTile<2> { static constexpr int TX = 64, TY = 8, TZ = 1; };
template <> struct FldColourTile<3> { static constexpr int TX = 64, TY = 4, TZ = 2; };

// Tiles of the kernels that take two cells of a colour (or four cells of a
// row) per thread with 16-byte accesses: 32 threads take a row of 128 cells.
struct FldPairTile {
  static constexpr int TX = 128, TY = 4, TZ = 2;
};

__device__ __forceinline__ double2 fld_ld2(const double* p) {
  return *reinterpret_cast<const double2*>(p);
}

// Origin (in cells) of this workgroup's TX x TY x TZ tile of level L: tile ids
// dealt XCD-contiguously, in y panels.
template <class T>
__device__ __forceinline__ void fld_tile_origin(const FldLevel& L, int* o) {
  const unsigned tx = (L.n[0] + T::TX - 1) / T::TX, ty = (L.n[1] + T::TY - 1) / T::TY;
  const unsigned tz = (L.n[2] + T::TZ - 1) / T::TZ;
  const unsigned b = (unsigned)xcd_tile(blockIdx.x, gridDim.x);
  // panel pn holds tile rows [pn*FLD_PANEL, pn*FLD_PANEL + py); the last may be short
  const unsigned pn = b / (tx * FLD_PANEL * tz), rem = b - pn * (tx * FLD_PANEL * tz);
  const unsigned py = min(FLD_PANEL, ty - pn * FLD_PANEL);
  const unsigned bx = rem % tx, r = rem / tx;
  const unsigned by = pn * FLD_PANEL + r % py, bz = r / py;
  o[0] = (int)bx * T::TX;
  o[1] = (int)by * T::TY;
  o[2] = (int)bz * T::TZ;
}

template <class T>
unsigned fld_tiles_of(const FldLevel& L) {
  return (unsigned)(((L.n[0] + T::TX - 1) / T::TX) * ((L.n[1] + T::TY - 1) / T::TY) *
                    ((L.n[2] + T::TZ - 1) / T::TZ));
}

// Cell (i, j, k) of this thread in the tile grid of level L; false if
// outside the level.
template <int NDIM>
__device__ __forceinline__ bool fld_tile_cell(const FldLevel& L, int* p) {
  using T = FldTile<NDIM>;
  fld_tile_origin<T>(L, p);
  const int t = threadIdx.x;
  p[0] += t % T::TX;
  p[1] += (t / T::TX) % T::TY;
  p[2] += t / (T::TX * T::TY);
  return p[0] < L.n[0] && p[1] < L.n[1] && p[2] < L.n[2];
}

template <int NDIM>
unsigned fld_tiles(const FldLevel& L) {
  return fld_tiles_of<FldTile<NDIM>>(L);
}

// Cell (i, j, k) of colour `colour` of this thread in the colour tile grid of
// level L (the tile origin is even along x, so the colour fixes i's parity);
// false if outside the level.
template <int NDIM>
__device__ __forceinline__ bool fld_colour_cell(const FldLevel& L, int colour, int* p) {
  using T = FldColourTile<NDIM>;
  fld_tile_origin<T>(L, p);
  const int t = threadIdx.x;
  constexpr int SX = T::TX / 2;
  p[1] += (t / SX) % T::TY;
  p[2] += t / (SX * T::TY);
  p[0] += 2 * (t % SX) + ((p[1] + p[2] + colour) & 1);
  return p[0] < L.n[0] && p[1] < L.n[1] && p[2] < L.n[2];
}

// Finest level from the state: D, b = E, x = E (a float state is widened:
// the solve itself is in double for both storage types).
template <int NDIM, typename T>
__global__ __launch_bounds__(256) void fld_setup(FldLevel L, FldCommon cm, const T* rho,
                                                 const T* E, double kappa, int limiter,
                                                 Control* ctl) {
#pragma clang fp contract(off)
  int p[3];
  unsigned flags = 0;
  if (fld_tile_cell<NDIM>(L, p)) {
    const unsigned stride[3] = {1u, (unsigned)L.n[0], (unsigned)L.n[0] * (unsigned)L.n[1]};
    const unsigned c = (unsigned)p[0] + (unsigned)p[1] * stride[1] + (unsigned)p[2] * stride[2];
    double g2 = 0.0;
#pragma unroll
    for (int d = 0; d < NDIM; ++d) {
      const int qlo = fld_nb(p[d], L.n[d], 0, cm.per[d]);
      const int qhi = fld_nb(p[d], L.n[d], 1, cm.per[d]);
      const unsigned lo = qlo < 0 ? c : c + (unsigned)(qlo - p[d]) * stride[d];
      const unsigned hi = qhi < 0 ? c : c + (unsigned)(qhi - p[d]) * stride[d];
      const double g = ((double)E[hi] - (double)E[lo]) / (2.0 * L.dx[d]);
      g2 += g * g;
    }
    const double r = (double)rho[c], e = (double)E[c];
    double lam = 1.0 / 3.0;
    if (limiter) {
      const double R = sqrt(g2) / (r * kappa * e);
      lam = (2.0 + R) / (6.0 + 3.0 * R + R * R);
    }
    const double D = FLD_C_LIGHT * lam / (kappa * r);
    const unsigned s = fld_at(L, p[0], p[1], p[2]);
    L.D[s] = D;
    L.b[s] = e;
    L.x[s] = e;
    if (!(r > 0.0)) flags |= FLAG_DENSITY;
    if (!(e > 0.0) || !isfinite(D)) flags |= FLAG_RADIATION;
  }
  block_finish<256>(flags, 0.0, false, ctl, nullptr);
}

// fld_setup for FP64 3D states with nx a multiple of 4: four cells of a row
// per thread (x = i0 .. i0 + 3, i0 a multiple of 4).  E and rho come as
// 16-byte pairs, the six neighbour values per cell from the row itself, one
// value beyond each end and the pairs of the rows above and below: 14 loads
// per four cells instead of 32.  Cells i0 and i0 + 2 share a colour, as do
// i0 + 1 and i0 + 3, each pair at two consecutive slots: x, b and D go out as
// six 16-byte stores instead of twelve.  Per cell the arithmetic is
// fld_setup's, in the same order.
__global__ __launch_bounds__(256) void fld_setup_quad(FldLevel L, FldCommon cm, const double* rho,
                                                      const double* E, double kappa, int limiter,
                                                      Control* ctl) {
#pragma clang fp contract(off)
  int o[3];
  fld_tile_origin<FldPairTile>(L, o);
  const int t = threadIdx.x;
  const int j = o[1] + (t / 32) % FldPairTile::TY, k = o[2] + t / (32 * FldPairTile::TY);
  const int i0 = o[0] + 4 * (t % 32);
  const int n0 = L.n[0], n1 = L.n[1], n2 = L.n[2];
  unsigned flags = 0;
  if (i0 < n0 && j < n1 && k < n2) {
    const unsigned sy = (unsigned)n0, sz = (unsigned)n0 * (unsigned)n1;
    const unsigned c = (unsigned)i0 + (unsigned)j * sy + (unsigned)k * sz;
    // a wall side uses the cell itself, as fld_nb's -1 does in fld_setup
    const int xl = fld_nb(i0, n0, 0, cm.per[0]), xh = fld_nb(i0 + 3, n0, 1, cm.per[0]);
    const int jl = fld_nb(j, n1, 0, cm.per[1]), jh = fld_nb(j, n1, 1, cm.per[1]);
    const int kl = fld_nb(k, n2, 0, cm.per[2]), kh = fld_nb(k, n2, 1, cm.per[2]);
    const unsigned cxl = xl < 0 ? c : c - (unsigned)i0 + (unsigned)xl;
    const unsigned cxh = xh < 0 ? c + 3u : c - (unsigned)i0 + (unsigned)xh;
    const unsigned cyl = jl < 0 ? c : c + (unsigned)(jl - j) * sy;
    const unsigned cyh = jh < 0 ? c : c + (unsigned)(jh - j) * sy;
    const unsigned czl = kl < 0 ? c : c + (unsigned)(kl - k) * sz;
    const unsigned czh = kh < 0 ? c : c + (unsigned)(kh - k) * sz;
    const double2 e01 = fld_ld2(E + c), e23 = fld_ld2(E + c + 2);
    const double2 r01 = fld_ld2(rho + c), r23 = fld_ld2(rho + c + 2);
    const double exl = E[cxl], exh = E[cxh];
    const double2 yl01 = fld_ld2(E + cyl), yl23 = fld_ld2(E + cyl + 2);
    const double2 yh01 = fld_ld2(E + cyh), yh23 = fld_ld2(E + cyh + 2);
    const double2 zl01 = fld_ld2(E + czl), zl23 = fld_ld2(E + czl + 2);
    const double2 zh01 = fld_ld2(E + czh), zh23 = fld_ld2(E + czh + 2);
    const double ev[4] = {e01.x, e01.y, e23.x, e23.y};
    const double rv[4] = {r01.x, r01.y, r23.x, r23.y};
    const double ylv[4] = {yl01.x, yl01.y, yl23.x, yl23.y}, yhv[4] = {yh01.x, yh01.y, yh23.x, yh23.y};
    const double zlv[4] = {zl01.x, zl01.y, zl23.x, zl23.y}, zhv[4] = {zh01.x, zh01.y, zh23.x, zh23.y};
    double Dv[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const double lo[3] = {q == 0 ? exl : ev[q - 1], ylv[q], zlv[q]};
      const double hi[3] = {q == 3 ? exh : ev[q + 1], yhv[q], zhv[q]};
      double g2 = 0.0;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const double g = (hi[d] - lo[d]) / (2.0 * L.dx[d]);
        g2 += g * g;
      }
      const double r = rv[q], e = ev[q];
      double lam = 1.0 / 3.0;
      if (limiter) {
        const double R = sqrt(g2) / (r * kappa * e);
        lam = (2.0 + R) / (6.0 + 3.0 * R + R * R);
      }
      Dv[q] = FLD_C_LIGHT * lam / (kappa * r);
      if (!(r > 0.0)) flags |= FLAG_DENSITY;
      if (!(e > 0.0) || !isfinite(Dv[q])) flags |= FLAG_RADIATION;
    }
    // colour of cell i0 and its partner i0 + 2 at slots i0/2, i0/2 + 1; the
    // other colour holds i0 + 1 and i0 + 3 at the same slots
    const unsigned row = (unsigned)k * (unsigned)n1 + (unsigned)j;
    const unsigned base = row * L.hx + (unsigned)(i0 >> 1);
    const int c0 = (i0 + j + k) & 1;
    const unsigned s0 = (c0 ? L.cs : 0u) + base, s1 = (c0 ? 0u : L.cs) + base;
    *reinterpret_cast<double2*>(L.D + s0) = make_double2(Dv[0], Dv[2]);
    *reinterpret_cast<double2*>(L.b + s0) = make_double2(ev[0], ev[2]);
    *reinterpret_cast<double2*>(L.x + s0) = make_double2(ev[0], ev[2]);
    *reinterpret_cast<double2*>(L.D + s1) = make_double2(Dv[1], Dv[3]);
    *reinterpret_cast<double2*>(L.b + s1) = make_double2(ev[1], ev[3]);
    *reinterpret_cast<double2*>(L.x + s1) = make_double2(ev[1], ev[3]);
  }
  block_finish<256>(flags, 0.0, false, ctl, nullptr);
}

// The finest x back into the state's E_r field (rounded to float for a
// float state).
template <int NDIM, typename R>
__global__ __launch_bounds__(256) void fld_store(FldLevel L, R* E) {
  int p[3];
  if (!fld_tile_cell<NDIM>(L, p)) return;
  const unsigned c = ((unsigned)p[2] * (unsigned)L.n[1] + (unsigned)p[1]) * (unsigned)L.n[0] +
                     (unsigned)p[0];
  E[c] = R(L.x[fld_at(L, p[0], p[1], p[2])]);
}

// fld_store for FP64 3D states with nx a multiple of 4: four cells of a row
// per thread, the two colour pairs (slots i0/2, i0/2 + 1 of each colour) and
// E as 16-byte accesses, the same words as fld_store writes.
__global__ __launch_bounds__(256) void fld_store_quad(FldLevel L, double* E) {
  int o[3];
  fld_tile_origin<FldPairTile>(L, o);
  const int t = threadIdx.x;
  const int j = o[1] + (t / 32) % FldPairTile::TY, k = o[2] + t / (32 * FldPairTile::TY);
  const int i0 = o[0] + 4 * (t % 32);
  if (i0 >= L.n[0] || j >= L.n[1] || k >= L.n[2]) return;
  const unsigned row = (unsigned)k * (unsigned)L.n[1] + (unsigned)j;
  const unsigned base = row * L.hx + (unsigned)(i0 >> 1);
  const int c0 = (i0 + j + k) & 1;  // colour of cells i0 and i0 + 2
  const double2 a = fld_ld2(L.x + (c0 ? L.cs : 0u) + base);
  const double2 b = fld_ld2(L.x + (c0 ? 0u : L.cs) + base);
  double* e = E + row * (unsigned)L.n[0] + (unsigned)i0;
  *reinterpret_cast<double2*>(e) = make_double2(a.x, b.x);
  *reinterpret_cast<double2*>(e + 2) = make_double2(a.y, b.y);
}

__global__ __launch_bounds__(256) void fld_coarsen_D(FldLevel F, FldLevel C, double inv) {
#pragma clang fp contract(off)
  const unsigned c = (unsigned)blockIdx.x * 256u + threadIdx.x;
  if (c >= fld_cells(C)) return;
  int P[3], lo[3], cnt[3];
  fld_cell(C, c, P);
  fld_children(C, P, lo, cnt);
  double s = 0.0;
  for (int dz = 0; dz < cnt[2]; ++dz)
    for (int dy = 0; dy < cnt[1]; ++dy)
      for (int dx = 0; dx < cnt[0]; ++dx) s += F.D[fld_at(F, lo[0] + dx, lo[1] + dy, lo[2] + dz)];
  C.D[fld_at(C, P[0], P[1], P[2])] = s * inv;
}

// One red-black half-sweep of level L: every cell of colour `colour`, one
// thread per cell of a colour tile.
template <int NDIM>
__global__ __launch_bounds__(256) void fld_relax(FldLevel L, FldCommon cm, int colour) {
  int p[3];
  if (!fld_colour_cell<NDIM>(L, colour, p)) return;
  fld_relax_cell<NDIM>(L, cm, colour, p[0], p[1], p[2],
                       (unsigned)p[2] * (unsigned)L.n[1] + (unsigned)p[1]);
}

// The 3D half-sweep with two cells of the colour per thread (slots h and
// h + 1 of a row, h even) and 16-byte loads.  The half-sweep's neighbour
// loads hit the L1, but each 64-lane load instruction still occupies the L1's
// address and data units for tens of cycles (about 26 measured for 8-byte
// words), so with six neighbour rows of x and D per cell that path, not HBM,
// set the time.  Here one 16-byte load brings a neighbour row's values for
// both cells: 14 loads and one store per two cells instead of 28 loads and
// two stores.  Needs hx even (the pairs and both colour halves 16-byte
// aligned), hence nx a multiple of 4.  Faces, order and arithmetic are those
// of fld_relax_cell.

// The neighbourhood of the pair of cells of colour `colour` at slots h, h+1 of
// row (j, k): both cells' own D and b (and x when want_x), and for each cell
// the other colour's x and D across its six faces (x low, x high, y low, y
// high, z low, z high) with the faces' open flags, as fld_faces names them.
struct FldPair {
  unsigned own;          // index of slot h of the own colour
  int i0;                // x of the first cell; the second is i0 + 2
  double D[2], b[2], x[2];
  double xn[2][6], Dn[2][6];
  bool open[2][6];
};

__device__ __forceinline__ void fld_pair_load(const FldLevel& L, const FldCommon& cm, int colour,
                                              int h, int j, int k, bool want_x, FldPair& q) {
  const int n0 = L.n[0], n1 = L.n[1], n2 = L.n[2], hx = (int)L.hx;
  const int par = (j + k + colour) & 1;
  q.i0 = 2 * h + par;
  const unsigned row = (unsigned)k * (unsigned)n1 + (unsigned)j;
  const unsigned ob = colour ? 0u : L.cs;  // other colour
  q.own = (colour ? L.cs : 0u) + row * L.hx + (unsigned)h;
  const unsigned oth = ob + row * L.hx + (unsigned)h;
  // the in-row slot beyond the pair: h - 1 below the first cell (par 0) or
  // h + 2 above the second (par 1), wrapped on a periodic axis, clamped on a
  // wall (where the face is closed and the value unused)
  int he = par ? h + 2 : h - 1;
  if (he < 0) he = cm.per[0] ? hx - 1 : 0;
  if (he >= hx) he = cm.per[0] ? 0 : hx - 1;
  const int jm = j > 0 ? j - 1 : (cm.per[1] ? n1 - 1 : j);
  const int jp = j < n1 - 1 ? j + 1 : (cm.per[1] ? 0 : j);
  const int km = k > 0 ? k - 1 : (cm.per[2] ? n2 - 1 : k);
  const int kp = k < n2 - 1 ? k + 1 : (cm.per[2] ? 0 : k);
  auto at = [&](int jj, int kk) {
    return ob + ((unsigned)kk * (unsigned)n1 + (unsigned)jj) * L.hx + (unsigned)h;
  };
  const double2 Dc = fld_ld2(L.D + q.own), bc = fld_ld2(L.b + q.own);
  const double2 xc = want_x ? fld_ld2(L.x + q.own) : make_double2(0.0, 0.0);
  const double2 xr = fld_ld2(L.x + oth), Dr = fld_ld2(L.D + oth);
  const double xe = L.x[oth - (unsigned)h + (unsigned)he], De = L.D[oth - (unsigned)h + (unsigned)he];
  const double2 xym = fld_ld2(L.x + at(jm, k)), Dym = fld_ld2(L.D + at(jm, k));
  const double2 xyp = fld_ld2(L.x + at(jp, k)), Dyp = fld_ld2(L.D + at(jp, k));
  const double2 xzm = fld_ld2(L.x + at(j, km)), Dzm = fld_ld2(L.D + at(j, km));
  const double2 xzp = fld_ld2(L.x + at(j, kp)), Dzp = fld_ld2(L.D + at(j, kp));
  const bool wx = cm.per[0] && n0 > 1, wy = cm.per[1] && n1 > 1, wz = cm.per[2] && n2 > 1;
  q.D[0] = Dc.x; q.D[1] = Dc.y;
  q.b[0] = bc.x; q.b[1] = bc.y;
  q.x[0] = xc.x; q.x[1] = xc.y;
  // first cell: x low is xe (par 0) or slot h (par 1), x high slot h (par 0)
  // or h + 1 (par 1); second cell: x low slot h or h + 1, x high h + 1 or xe
  q.xn[0][0] = par ? xr.x : xe;   q.Dn[0][0] = par ? Dr.x : De;
  q.xn[0][1] = par ? xr.y : xr.x; q.Dn[0][1] = par ? Dr.y : Dr.x;
  q.xn[1][0] = par ? xr.y : xr.x; q.Dn[1][0] = par ? Dr.y : Dr.x;
  q.xn[1][1] = par ? xe : xr.y;   q.Dn[1][1] = par ? De : Dr.y;
  q.xn[0][2] = xym.x; q.xn[1][2] = xym.y; q.Dn[0][2] = Dym.x; q.Dn[1][2] = Dym.y;
  q.xn[0][3] = xyp.x; q.xn[1][3] = xyp.y; q.Dn[0][3] = Dyp.x; q.Dn[1][3] = Dyp.y;
  q.xn[0][4] = xzm.x; q.xn[1][4] = xzm.y; q.Dn[0][4] = Dzm.x; q.Dn[1][4] = Dzm.y;
  q.xn[0][5] = xzp.x; q.xn[1][5] = xzp.y; q.Dn[0][5] = Dzp.x; q.Dn[1][5] = Dzp.y;
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const int i = q.i0 + 2 * c;
    q.open[c][0] = i > 0 || wx;
    q.open[c][1] = i < n0 - 1 || wx;
    q.open[c][2] = j > 0 || wy;
    q.open[c][3] = j < n1 - 1 || wy;
    q.open[c][4] = k > 0 || wz;
    q.open[c][5] = k < n2 - 1 || wz;
  }
}

__global__ __launch_bounds__(256) void fld_relax_pair(FldLevel L, FldCommon cm, int colour) {
#pragma clang fp contract(off)
  int o[3];
  fld_tile_origin<FldPairTile>(L, o);
  const int t = threadIdx.x;
  const int j = o[1] + (t / 32) % FldPairTile::TY, k = o[2] + t / (32 * FldPairTile::TY);
  const int h = (o[0] >> 1) + 2 * (t % 32);
  if (j >= L.n[1] || k >= L.n[2] || h >= (int)L.hx) return;
  FldPair q;
  fld_pair_load(L, cm, colour, h, j, k, false, q);
  double res[2];
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    double num = q.b[c];
    double den = 1.0;
#pragma unroll
    for (int f = 0; f < 6; ++f) {
      const double a = q.open[c][f] ? (q.D[c] + q.Dn[c][f]) * L.K[f >> 1] : 0.0;
      num += a * (q.open[c][f] ? q.xn[c][f] : 0.0);
      den += a;
    }
    res[c] = num / den;
  }
  *reinterpret_cast<double2*>(L.x + q.own) = make_double2(res[0], res[1]);
}

// fld_restrict_red with two red cells per thread and 16-byte loads (3D, hx
// even, every axis halved): the residuals b - A x of the pair in the order of
// fld_apply_row, the black cells' entries zero, then the tile's 128 coarse
// cells add their children from LDS in the order of fld_restrict_cell.
__global__ __launch_bounds__(256) void fld_restrict_red_pair(FldLevel F, FldLevel C, FldCommon cm,
                                                             double inv) {
#pragma clang fp contract(off)
  using T = FldPairTile;
  __shared__ double r[T::TZ][T::TY][T::TX];
  int o[3];
  fld_tile_origin<T>(F, o);
  const int t = threadIdx.x;
  const int dy = (t / 32) % T::TY, dz = t / (32 * T::TY), sx = t % 32;
  const int j = o[1] + dy, k = o[2] + dz;
  const int h = (o[0] >> 1) + 2 * sx;
  const int par = (j + k) & 1;  // red: i + j + k even
  double rv[2] = {0.0, 0.0};
  if (j < F.n[1] && k < F.n[2] && h < (int)F.hx) {
    FldPair q;
    fld_pair_load(F, cm, 0, h, j, k, true, q);
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      double Ax = q.x[c];
#pragma unroll
      for (int f = 0; f < 6; ++f) {
        const double a = q.open[c][f] ? (q.D[c] + q.Dn[c][f]) * F.K[f >> 1] : 0.0;
        Ax += a * (q.open[c][f] ? q.x[c] - q.xn[c][f] : 0.0);
      }
      rv[c] = q.b[c] - Ax;
    }
  }
  // this thread's four cells of the row: 4 sx + par and 4 sx + 2 + par are red
  r[dz][dy][4 * sx + par] = rv[0];
  r[dz][dy][4 * sx + 2 + par] = rv[1];
  r[dz][dy][4 * sx + 1 - par] = 0.0;
  r[dz][dy][4 * sx + 3 - par] = 0.0;
  __syncthreads();
  constexpr int CX = T::TX / 2, CY = T::TY / 2, CZ = T::TZ / 2;
  if (t >= CX * CY * CZ) return;
  const int cx = t % CX, cy = (t / CX) % CY, cz = t / (CX * CY);
  const int P[3] = {(o[0] >> 1) + cx, (o[1] >> 1) + cy, (o[2] >> 1) + cz};
  if (P[0] >= C.n[0] || P[1] >= C.n[1] || P[2] >= C.n[2]) return;
  double sum = 0.0;
  for (int ez = 0; ez < 2; ++ez)
    for (int ey = 0; ey < 2; ++ey)
      for (int ex = 0; ex < 2; ++ex) sum += r[2 * cz + ez][2 * cy + ey][2 * cx + ex];
  const unsigned cc = fld_at(C, P[0], P[1], P[2]);
  C.b[cc] = sum * inv;
  C.x[cc] = 0.0;
}

// Restriction, one thread per coarse cell (any halving pattern).
template <int NDIM>
__global__ __launch_bounds__(256) void fld_restrict(FldLevel F, FldLevel C, FldCommon cm,
                                                    double inv) {
  const unsigned c = (unsigned)xcd_tile(blockIdx.x, gridDim.x) * 256u + threadIdx.x;
  if (c >= fld_cells(C)) return;
  int P[3];
  fld_cell(C, c, P);
  fld_restrict_cell<NDIM>(F, C, cm, inv, P);
}

// Restriction when every active axis is halved: one thread per fine cell of
// an even-aligned tile computes its residual; the tile's coarse cells then
// sum their children from LDS in the same order as fld_restrict_cell.
template <int NDIM>
__global__ __launch_bounds__(256) void fld_restrict_tile(FldLevel F, FldLevel C, FldCommon cm,
                                                         double inv) {
#pragma clang fp contract(off)
  using T = FldTile<NDIM>;
  __shared__ double r[256];
  int p[3];
  const bool in = fld_tile_cell<NDIM>(F, p);
  double rv = 0.0;
  if (in) rv = F.b[fld_at(F, p[0], p[1], p[2])] - fld_apply_row<NDIM>(F, cm, p);
  r[threadIdx.x] = rv;
  __syncthreads();
  constexpr int CX = T::TX / 2, CY = NDIM > 1 ? T::TY / 2 : 1, CZ = NDIM > 2 ? T::TZ / 2 : 1;
  const int t = threadIdx.x;
  if (t >= CX * CY * CZ) return;
  const int cx = t % CX, cy = (t / CX) % CY, cz = t / (CX * CY);
  // tile origin in fine cells, from this thread's own fine cell
  const int fx0 = p[0] - t % T::TX, fy0 = p[1] - (t / T::TX) % T::TY, fz0 = p[2] - t / (T::TX * T::TY);
  const int P[3] = {(fx0 >> 1) + cx, NDIM > 1 ? (fy0 >> 1) + cy : 0, NDIM > 2 ? (fz0 >> 1) + cz : 0};
  if (P[0] >= C.n[0] || P[1] >= C.n[1] || P[2] >= C.n[2]) return;
  double s = 0.0;
  for (int dz = 0; dz < (NDIM > 2 ? 2 : 1); ++dz)
    for (int dy = 0; dy < (NDIM > 1 ? 2 : 1); ++dy)
      for (int dx = 0; dx < 2; ++dx)
        s += r[(2 * cz + dz) * T::TX * T::TY + (2 * cy + dy) * T::TX + 2 * cx + dx];
  const unsigned cc = fld_at(C, P[0], P[1], P[2]);
  C.b[cc] = s * inv;
  C.x[cc] = 0.0;
}

// Restriction after a pre-smoothing that ended with a black half-sweep.  A
// black cell's neighbours are all red and have not changed since that
// half-sweep set the cell so that its equation holds, so its residual is zero
// in exact arithmetic (what the fine arithmetic would leave is rounding of
// order eps |b|).  Only the red cells' residuals are computed, one thread per
// red cell of a colour tile (even-aligned on every axis); the black ones enter
// the child sums as zeros, in the same order as fld_restrict_cell.
template <int NDIM>
__global__ __launch_bounds__(256) void fld_restrict_red(FldLevel F, FldLevel C, FldCommon cm,
                                                        double inv) {
#pragma clang fp contract(off)
  using T = FldColourTile<NDIM>;
  static_assert(T::TX * T::TY * T::TZ == 512, "two fine cells per thread");
  __shared__ double r[512];
  int o[3];
  fld_tile_origin<T>(F, o);
  const int t = threadIdx.x;
  constexpr int SX = T::TX / 2;
  const int ly = (t / SX) % T::TY, lz = t / (SX * T::TY);
  const int j = o[1] + ly, k = o[2] + lz;
  // red: i + j + k even (o[0] is even)
  const int li = 2 * (t % SX) + ((j + k) & 1);
  const int p[3] = {o[0] + li, j, k};
  double rv = 0.0;
  if (p[0] < F.n[0] && p[1] < F.n[1] && p[2] < F.n[2])
    rv = F.b[fld_at(F, p[0], p[1], p[2])] - fld_apply_row<NDIM>(F, cm, p);
  const int row = (lz * T::TY + ly) * T::TX;
  r[row + li] = rv;
  r[row + (li ^ 1)] = 0.0;
  __syncthreads();
  constexpr int CX = T::TX / 2, CY = NDIM > 1 ? T::TY / 2 : 1, CZ = NDIM > 2 ? T::TZ / 2 : 1;
  if (t >= CX * CY * CZ) return;
  const int cx = t % CX, cy = (t / CX) % CY, cz = t / (CX * CY);
  const int P[3] = {(o[0] >> 1) + cx, NDIM > 1 ? (o[1] >> 1) + cy : 0, NDIM > 2 ? (o[2] >> 1) + cz : 0};
  if (P[0] >= C.n[0] || P[1] >= C.n[1] || P[2] >= C.n[2]) return;
  double sum = 0.0;
  for (int dz = 0; dz < (NDIM > 2 ? 2 : 1); ++dz)
    for (int dy = 0; dy < (NDIM > 1 ? 2 : 1); ++dy)
      for (int dx = 0; dx < 2; ++dx)
        sum += r[(2 * cz + dz) * T::TX * T::TY + (2 * cy + dy) * T::TX + 2 * cx + dx];
  const unsigned cc = fld_at(C, P[0], P[1], P[2]);
  C.b[cc] = sum * inv;
  C.x[cc] = 0.0;
}

template <int NDIM>
__global__ __launch_bounds__(256) void fld_prolong(FldLevel F, FldLevel C, FldCommon cm) {
  int f[3];
  if (!fld_tile_cell<NDIM>(F, f)) return;
  fld_prolong_cell(F, C, cm, f);
}

template <int NDIM>
__global__ __launch_bounds__(256) void fld_prolong_all(FldLevel F, FldLevel C, FldCommon cm) {
  int f[3];
  if (!fld_tile_cell<NDIM>(F, f)) return;
  fld_prolong_cell_all<NDIM>(F, C, cm, f);
}

// Prolongation into the cells of one colour only, one thread per cell of a
// colour tile.  When post-smoothing follows, its first half-sweep (red) recomputes
// every red cell from b and the black neighbours alone, so the correction of
// the red cells is never read and only the black ones (colour 1) need it; the
// result is the same, bit for bit, as correcting every cell.
template <int NDIM, bool ALL>
__global__ __launch_bounds__(256) void fld_prolong_colour(FldLevel F, FldLevel C, FldCommon cm,
                                                          int colour) {
  int f[3];
  if (!fld_colour_cell<NDIM>(F, colour, f)) return;
  if (ALL)
    fld_prolong_cell_all<NDIM>(F, C, cm, f);
  else
    fld_prolong_cell(F, C, cm, f);
}

// fld_prolong_colour for the black cells of a 3D level with every axis halved
// and hx even: two black cells of a row per thread (slots h, h + 1).  Their
// parents along x are three consecutive coarse cells (h - 1, h, h + 1 when the
// row's black cells are even, h, h + 1, h + 2 when odd, the outer one wrapped
// or clamped as fld_nb says), so each of the four coarse rows gives its three
// values once; the fine pair is one 16-byte load and store.  Per cell the
// weights, the order of the eight terms and the sum are those of
// fld_prolong_cell_all.
__global__ __launch_bounds__(256) void fld_prolong_pair(FldLevel F, FldLevel C, FldCommon cm) {
#pragma clang fp contract(off)
  int o[3];
  fld_tile_origin<FldPairTile>(F, o);
  const int t = threadIdx.x;
  const int j = o[1] + (t / 32) % FldPairTile::TY, k = o[2] + t / (32 * FldPairTile::TY);
  const int h = (o[0] >> 1) + 2 * (t % 32);
  if (j >= F.n[1] || k >= F.n[2] || h >= (int)F.hx) return;
  const int par = (j + k + 1) & 1;  // black: i + j + k odd
  // the three coarse x positions; the first cell takes (near, far) = (1, 0)
  // of them for even black cells and (0, 1) for odd, the second (2, 1) and
  // (1, 2)
  int xs[3];
  if (par == 0) {
    const int a = fld_nb(h, C.n[0], 0, cm.per[0]);
    xs[0] = a < 0 ? h : a; xs[1] = h; xs[2] = h + 1;
  } else {
    const int c = fld_nb(h + 1, C.n[0], 1, cm.per[0]);
    xs[0] = h; xs[1] = h + 1; xs[2] = c < 0 ? h + 1 : c;
  }
  const int J = j >> 1, K = k >> 1;
  const int jq = fld_nb(J, C.n[1], j & 1, cm.per[1]), kq = fld_nb(K, C.n[2], k & 1, cm.per[2]);
  const int Jf = jq < 0 ? J : jq, Kf = kq < 0 ? K : kq;
  // coarse values: row r = (y far) | (z far) << 1, three x positions each
  double xc[4][3];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int jj = (r & 1) ? Jf : J, kk = (r & 2) ? Kf : K;
#pragma unroll
    for (int q = 0; q < 3; ++q) xc[r][q] = C.x[fld_at(C, xs[q], jj, kk)];
  }
  // selects on the parity keep xc in registers (a run-time index would not)
  double cn[2][4], cf[2][4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    cn[0][r] = par ? xc[r][0] : xc[r][1];
    cf[0][r] = par ? xc[r][1] : xc[r][0];
    cn[1][r] = par ? xc[r][1] : xc[r][2];
    cf[1][r] = par ? xc[r][2] : xc[r][1];
  }
  double v[2];
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    double s = 0.0;
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      const double w = ((m & 1) ? 0.25 : 0.75) * ((m & 2) ? 0.25 : 0.75) * ((m & 4) ? 0.25 : 0.75);
      s += w * ((m & 1) ? cf[c][m >> 1] : cn[c][m >> 1]);
    }
    v[c] = s;
  }
  double* xf = F.x + F.cs + ((unsigned)k * (unsigned)F.n[1] + (unsigned)j) * F.hx + (unsigned)h;
  const double2 x = fld_ld2(xf);
  *reinterpret_cast<double2*>(xf) = make_double2(x.x + v[0], x.y + v[1]);
}

// Residual norm, two deterministic passes: per-tile sums of r^2 in a fixed
// order, then one workgroup adds the tile sums in a fixed order.
template <int NDIM>
__global__ __launch_bounds__(256) void fld_resid_sq(FldLevel L, FldCommon cm, double* part) {
#pragma clang fp contract(off)
  __shared__ double w[4];
  int p[3];
  double r2 = 0.0;
  if (fld_tile_cell<NDIM>(L, p)) {
    const double r = L.b[fld_at(L, p[0], p[1], p[2])] - fld_apply_row<NDIM>(L, cm, p);
    r2 = r * r;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) r2 += __shfl_xor(r2, o, 64);
  if ((threadIdx.x & 63) == 0) w[threadIdx.x >> 6] = r2;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = (w[0] + w[1]) + (w[2] + w[3]);
}

// K_d = (dt/2) / dx_d^2 of every level (dx2 from the host, dt on the device).
struct FldDx2 {
  double v[FLD_MAX_LEVELS][3];
};
__global__ void fld_coeffs(FldDx2 dx2, int nlev, const double* dt, double* K) {
#pragma clang fp contract(off)
  const int t = threadIdx.x;
  if (t < 3 * nlev) K[t] = (0.5 * *dt) / dx2.v[t / 3][t % 3];
}

__global__ __launch_bounds__(1024) void fld_resid_final(const double* part, unsigned n, double* out) {
#pragma clang fp contract(off)
  __shared__ double w[16];
  double s = 0.0;
  for (unsigned i = threadIdx.x; i < n; i += 1024) s += part[i];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if ((threadIdx.x & 63) == 0) w[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int i = 0; i < 16; ++i) t += w[i];
    *out = sqrt(t);
  }
}

// The V-cycle below a level small enough for one workgroup: the arrays of
// those levels are copied into LDS (x, b and D of the first one, D of the
// rest; the coarse x and b are written by the restriction before they are
// read), every phase (half-sweep, restriction, prolongation) is a loop of
// the workgroup over the level's cells separated by barriers, and x of the
// first level is copied back at the end.  Same per-cell arithmetic as the
// multi-workgroup kernels; LDS latency instead of L2 latency for the ~50
// short phases of a cycle.
constexpr int FLD_TAIL_LEVELS = 16;

struct FldTail {
  FldLevel lv[FLD_TAIL_LEVELS];       // global arrays
  double inv[FLD_TAIL_LEVELS];        // 1 / children of level m (from level m - 1)
  unsigned lds_off[FLD_TAIL_LEVELS];  // element offset of level m's arrays in LDS
  int nlev;
  int nu1, nu2, ncoarse;
};

// Level m of the tail with x, b, D in LDS (each 2 cs elements, in that order).
__device__ __forceinline__ FldLevel fld_lds_level(const FldTail& T, int m, double* lds) {
  FldLevel L = T.lv[m];
  const unsigned e = 2u * L.cs;
  L.x = lds + T.lds_off[m];
  L.b = L.x + e;
  L.D = L.b + e;
  return L;
}

template <int NDIM>
__device__ void fld_tail_relax(const FldLevel& L, const FldCommon& cm, int sweeps) {
  // A level of one cell has every face closed: one sweep sets x = b / 1 = b,
  // and every further sweep computes the same bits again, over a black colour
  // with no cell.  Its phases (each ending in a barrier of the workgroup) are
  // skipped; the result is that of `sweeps` sweeps.
  if (fld_cells(L) == 1) {
    if (sweeps > 0 && threadIdx.x == 0) fld_relax_slot<NDIM>(L, cm, 0, 0);
    __syncthreads();
    return;
  }
  for (int sw = 0; sw < sweeps; ++sw)
    for (int colour = 0; colour < 2; ++colour) {
      for (unsigned t = threadIdx.x; t < L.cs; t += 1024) fld_relax_slot<NDIM>(L, cm, colour, t);
      __syncthreads();
    }
}

template <int NDIM>
__global__ __launch_bounds__(1024) void fld_vcycle_tail(FldTail T, FldCommon cm) {
  extern __shared__ double lds[];
  for (int m = 0; m < T.nlev; ++m) {
    const FldLevel& G = T.lv[m];
    const FldLevel L = fld_lds_level(T, m, lds);
    const unsigned e = 2u * G.cs;
    for (unsigned t = threadIdx.x; t < e; t += 1024) {
      L.D[t] = G.D[t];
      if (m == 0) {
        L.x[t] = G.x[t];
        L.b[t] = G.b[t];
      }
    }
  }
  __syncthreads();
  const int last = T.nlev - 1;
  for (int l = 0; l < last; ++l) {
    const FldLevel F = fld_lds_level(T, l, lds);
    fld_tail_relax<NDIM>(F, cm, T.nu1);
    const FldLevel C = fld_lds_level(T, l + 1, lds);
    for (unsigned c = threadIdx.x; c < fld_cells(C); c += 1024) {
      int P[3];
      fld_cell(C, c, P);
      fld_restrict_cell<NDIM>(F, C, cm, T.inv[l + 1], P);
    }
    __syncthreads();
  }
  fld_tail_relax<NDIM>(fld_lds_level(T, last, lds), cm, T.ncoarse);
  for (int l = last - 1; l >= 0; --l) {
    const FldLevel F = fld_lds_level(T, l, lds);
    const FldLevel C = fld_lds_level(T, l + 1, lds);
    for (unsigned c = threadIdx.x; c < fld_cells(F); c += 1024) {
      int f[3];
      fld_cell(F, c, f);
      fld_prolong_cell(F, C, cm, f);
    }
    __syncthreads();
    fld_tail_relax<NDIM>(F, cm, T.nu2);
  }
  const FldLevel& G = T.lv[0];
  const FldLevel L = fld_lds_level(T, 0, lds);
  for (unsigned t = threadIdx.x; t < 2u * G.cs; t += 1024) G.x[t] = L.x[t];
}

// One double from device slot to device slot (the step size of a time loop
// handed to the diffusion before the hydro step overwrites its slot with the
// next CFL step).
__global__ void fld_copy_dt(const double* from, double* to) {
  if (threadIdx.x == 0) *to = *from;
}

hipError_t launch_fld_copy_dt(const double* from, double* to, hipStream_t s) {
  fld_copy_dt<<<1, 64, 0, s>>>(from, to);
  return hipGetLastError();
}

// ---------------------------------------------------------------- host side

namespace {

struct Hierarchy {
  int nlev;
  int n[FLD_MAX_LEVELS][3];
  int halved[FLD_MAX_LEVELS][3];
  double dx[FLD_MAX_LEVELS][3];
};

Hierarchy hierarchy_of(const Grid& G) {
  Hierarchy H;
  H.nlev = 1;
  for (int d = 0; d < 3; ++d) {
    H.n[0][d] = G.n[d];
    H.halved[0][d] = 0;
    H.dx[0][d] = G.dx[d];
  }
  while (H.nlev < FLD_MAX_LEVELS) {
    const int l = H.nlev;
    int any = 0;
    for (int d = 0; d < 3; ++d) {
      const int m = H.n[l - 1][d];
      const int periodic = G.bc[d][0] == BC_PERIODIC;
      int h = d < G.ndim && m % 2 == 0;
      if (h && periodic) h = (m / 2) % 2 == 0 || m / 2 == 1;
      H.halved[l][d] = h;
      H.n[l][d] = h ? m / 2 : m;
      H.dx[l][d] = h ? 2.0 * H.dx[l - 1][d] : H.dx[l - 1][d];
      any |= h;
    }
    if (!any) break;
    ++H.nlev;
  }
  return H;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

long long cells(const Hierarchy& H, int l) {
  return (long long)H.n[l][0] * H.n[l][1] * H.n[l][2];
}

// Elements of one colour-split array of level l: 2 colours x rows x slots.
long long split_elems(const Hierarchy& H, int l) {
  return 2LL * H.n[l][1] * H.n[l][2] * ((H.n[l][0] + 1) / 2);
}

// Tile-sum slots of the residual norm: one per 256-cell tile of the finest
// level (the tile counts of the 1D, 2D and 3D tilings never exceed this).
size_t resid_slots(const Hierarchy& H) {
  const long long a = (H.n[0][0] + 31) / 32, b = (H.n[0][1] + 3) / 4, c = (H.n[0][2] + 1) / 2;
  const long long t3 = a * b * c;
  const long long t2 = ((H.n[0][0] + 63) / 64) * b * H.n[0][2];
  const long long t1 = ((H.n[0][0] + 255) / 256) * H.n[0][1] * H.n[0][2];
  return (size_t)std::max(t3, std::max(t2, t1));
}

// Workspace: control block | K of every level | residual tile sums | per
// level: x, b, D (colour-split)
constexpr size_t FLD_K_BYTES = 1024;  // FLD_MAX_LEVELS x 3 doubles, rounded up
static_assert(FLD_MAX_LEVELS * 3 * sizeof(double) <= FLD_K_BYTES, "K slots");

size_t fld_workspace(const Hierarchy& H) {
  size_t total = 256 + FLD_K_BYTES + align256(resid_slots(H) * sizeof(double));
  for (int l = 0; l < H.nlev; ++l) total += 3 * align256(split_elems(H, l) * sizeof(double));
  return total;
}

hard_status_t check_fld_grid(const hard_grid_t* g, Grid* G) {
  hard_status_t st = check_grid(g, G);
  if (st) return st;
  if (!G->rad) return fail(HARD_ERR_INVALID_ARG, "radiation diffusion needs rad = 1");
  if (!(G->kappa > 0.0)) return fail(HARD_ERR_INVALID_ARG, "radiation diffusion needs kappa > 0");
  for (int d = 0; d < G->ndim; ++d)
    if (G->bc[d][0] == BC_PERIODIC && G->n[d] % 2)
      return fail(HARD_ERR_UNSUPPORTED,
                  "radiation diffusion: periodic axis %d has an odd size (%d); red-black "
                  "relaxation needs an even one", d, G->n[d]);
  return HARD_OK;
}

unsigned blocks_for(long long threads) { return (unsigned)((threads + 255) / 256); }

struct Solver {
  const Grid& G;
  const Hierarchy& H;
  FldLevel lv[FLD_MAX_LEVELS];
  double inv_children[FLD_MAX_LEVELS];
  FldCommon cm;
  int nu1, nu2, ncoarse;
  int tail;         // first level solved by the one-workgroup kernel
  double* part;     // residual tile sums
  double* Kbuf;     // K_d of every level
  hipStream_t s;

  bool all_halved(int l) const {  // every active axis halved from level l - 1
    for (int d = 0; d < G.ndim; ++d)
      if (!H.halved[l][d]) return false;
    return true;
  }

  template <int NDIM>
  hipError_t relax(int l, int sweeps) {
    const FldLevel& L = lv[l];
    const unsigned tiles = fld_tiles_of<FldColourTile<NDIM>>(L);
    const bool pair = NDIM == 3 && L.hx % 2 == 0;
    const unsigned ptiles = fld_tiles_of<FldPairTile>(L);
    for (int sw = 0; sw < sweeps; ++sw)
      for (int colour = 0; colour < 2; ++colour) {
        if (pair)
          fld_relax_pair<<<ptiles, 256, 0, s>>>(L, cm, colour);
        else
          fld_relax<NDIM><<<tiles, 256, 0, s>>>(L, cm, colour);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
      }
    return hipSuccess;
  }

  template <int NDIM>
  hipError_t vcycle(int l) {
    hipError_t e;
    if (l < 0 || l >= H.nlev) return hipErrorInvalidValue;
    if (l == tail) {
      FldTail T;
      T.nlev = H.nlev - l;
      for (int m = 0; m < T.nlev; ++m) {
        T.lv[m] = lv[l + m];
        T.inv[m] = inv_children[l + m];
      }
      T.nu1 = nu1;
      T.nu2 = nu2;
      T.ncoarse = ncoarse;
      unsigned off = 0;
      for (int m = 0; m < T.nlev; ++m) {
        T.lds_off[m] = off;
        off += 6u * lv[l + m].cs;
      }
      const size_t bytes = (size_t)off * sizeof(double);
      hipError_t e2 = hipFuncSetAttribute(reinterpret_cast<const void*>(&fld_vcycle_tail<NDIM>),
                                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
      if (e2 != hipSuccess) return e2;
      fld_vcycle_tail<NDIM><<<1, 1024, bytes, s>>>(T, cm);
      return hipGetLastError();
    }
    if (l + 1 == H.nlev) return relax<NDIM>(l, ncoarse);  // coarsest level
    if (l + 1 > H.nlev) return hipErrorInvalidValue;
    if ((e = relax<NDIM>(l, nu1)) != hipSuccess) return e;
    if (NDIM == 3 && all_halved(l + 1) && nu1 > 0 && lv[l].hx % 2 == 0)
      fld_restrict_red_pair<<<fld_tiles_of<FldPairTile>(lv[l]), 256, 0, s>>>(
          lv[l], lv[l + 1], cm, inv_children[l + 1]);
    else if (all_halved(l + 1) && nu1 > 0)
      fld_restrict_red<NDIM><<<fld_tiles_of<FldColourTile<NDIM>>(lv[l]), 256, 0, s>>>(
          lv[l], lv[l + 1], cm, inv_children[l + 1]);
    else if (all_halved(l + 1))
      fld_restrict_tile<NDIM><<<fld_tiles<NDIM>(lv[l]), 256, 0, s>>>(lv[l], lv[l + 1], cm,
                                                                    inv_children[l + 1]);
    else
      fld_restrict<NDIM><<<blocks_for(cells(H, l + 1)), 256, 0, s>>>(lv[l], lv[l + 1], cm,
                                                                     inv_children[l + 1]);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = vcycle<NDIM>(l + 1)) != hipSuccess) return e;
    if (NDIM == 3 && nu2 > 0 && all_halved(l + 1) && lv[l].hx % 2 == 0) {
      fld_prolong_pair<<<fld_tiles_of<FldPairTile>(lv[l]), 256, 0, s>>>(lv[l], lv[l + 1], cm);
    } else if (nu2 > 0) {
      const unsigned tiles = fld_tiles_of<FldColourTile<NDIM>>(lv[l]);
      if (all_halved(l + 1))
        fld_prolong_colour<NDIM, true><<<tiles, 256, 0, s>>>(lv[l], lv[l + 1], cm, 1);
      else
        fld_prolong_colour<NDIM, false><<<tiles, 256, 0, s>>>(lv[l], lv[l + 1], cm, 1);
    } else if (all_halved(l + 1)) {
      fld_prolong_all<NDIM><<<fld_tiles<NDIM>(lv[l]), 256, 0, s>>>(lv[l], lv[l + 1], cm);
    } else {
      fld_prolong<NDIM><<<fld_tiles<NDIM>(lv[l]), 256, 0, s>>>(lv[l], lv[l + 1], cm);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    return relax<NDIM>(l, nu2);
  }

  template <int NDIM>
  hipError_t resid_norm(double* out) {
    const unsigned nt = fld_tiles<NDIM>(lv[0]);
    fld_resid_sq<NDIM><<<nt, 256, 0, s>>>(lv[0], cm, part);
    fld_resid_final<<<1, 1024, 0, s>>>(part, nt, out);
    return hipGetLastError();
  }

  template <int NDIM, typename R>
  hipError_t run(R* U, int limiter, int ncycles, double* resid, Control* ctl) {
    hipError_t e;
    const long long N = cells(H, 0);
    const R* rho = U;
    R* E = U + (long long)(G.nvar - 1) * N;
    if (NDIM == 3 && std::is_same<R, double>::value && G.n[0] % 4 == 0 &&
        ((uintptr_t)rho | (uintptr_t)E) % 16 == 0)
      fld_setup_quad<<<fld_tiles_of<FldPairTile>(lv[0]), 256, 0, s>>>(
          lv[0], cm, reinterpret_cast<const double*>(rho), reinterpret_cast<const double*>(E),
          G.kappa, limiter, ctl);
    else
      fld_setup<NDIM, R><<<fld_tiles<NDIM>(lv[0]), 256, 0, s>>>(lv[0], cm, rho, E, G.kappa, limiter,
                                                               ctl);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    FldDx2 dx2;
    for (int l = 0; l < H.nlev; ++l)
      for (int d = 0; d < 3; ++d) dx2.v[l][d] = lv[l].dx2[d];
    fld_coeffs<<<1, 3 * FLD_MAX_LEVELS, 0, s>>>(dx2, H.nlev, cm.dt, Kbuf);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    for (int l = 1; l < H.nlev; ++l) {
      fld_coarsen_D<<<blocks_for(cells(H, l)), 256, 0, s>>>(lv[l - 1], lv[l], inv_children[l]);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (resid && (e = resid_norm<NDIM>(resid)) != hipSuccess) return e;
    for (int c = 0; c < ncycles; ++c) {
      if ((e = vcycle<NDIM>(0)) != hipSuccess) return e;
      if (resid && (e = resid_norm<NDIM>(resid + c + 1)) != hipSuccess) return e;
    }
    if (NDIM == 3 && std::is_same<R, double>::value && G.n[0] % 4 == 0 && (uintptr_t)E % 16 == 0)
      fld_store_quad<<<fld_tiles_of<FldPairTile>(lv[0]), 256, 0, s>>>(
          lv[0], reinterpret_cast<double*>(E));
    else
      fld_store<NDIM, R><<<fld_tiles<NDIM>(lv[0]), 256, 0, s>>>(lv[0], E);
    return hipGetLastError();
  }
};

}  // namespace
}  // namespace hard

using namespace hard;

extern "C" {

hard_status_t hard_gmg_levels(const hard_grid_t* g, int32_t max_levels, int64_t* levels_n,
                              int32_t* nlevels) {
  Grid G;
  hard_status_t st = check_fld_grid(g, &G);
  if (st) return st;
  if (!nlevels) return fail(HARD_ERR_INVALID_ARG, "nlevels is NULL");
  if (max_levels > 0 && !levels_n) return fail(HARD_ERR_INVALID_ARG, "levels_n is NULL");
  const Hierarchy H = hierarchy_of(G);
  for (int l = 0; l < H.nlev && l < max_levels; ++l)
    for (int d = 0; d < 3; ++d) levels_n[3 * l + d] = H.n[l][d];
  *nlevels = H.nlev;
  return ok();
}

hard_status_t hard_rad_diffuse_workspace_bytes(const hard_grid_t* g, size_t* bytes) {
  Grid G;
  hard_status_t st = check_fld_grid(g, &G);
  if (st) return st;
  if (!bytes) return fail(HARD_ERR_INVALID_ARG, "bytes is NULL");
  *bytes = fld_workspace(hierarchy_of(G));
  return ok();
}

hard_status_t hard_rad_diffuse(const hard_grid_t* g, void* U, const double* dt_dev,
                               const hard_gmg_opts_t* opts, double* resid_dev, void* work,
                               size_t work_bytes, void* stream) {
  Grid G;
  hard_status_t st = check_fld_grid(g, &G);
  if (st) return st;
  if ((st = check_ptr(U, G.wsize, "U"))) return st;
  if ((st = check_ptr(dt_dev, 8, "dt_dev"))) return st;
  if (resid_dev && (st = check_ptr(resid_dev, 8, "resid_dev"))) return st;
  if (!opts) return fail(HARD_ERR_INVALID_ARG, "opts is NULL");
  if (opts->limiter != HARD_FLD_EDDINGTON && opts->limiter != HARD_FLD_LEVERMORE)
    return fail(HARD_ERR_INVALID_ARG, "limiter must be HARD_FLD_EDDINGTON or HARD_FLD_LEVERMORE");
  if (opts->ncycles < 0 || opts->ncycles > 1000)
    return fail(HARD_ERR_INVALID_ARG, "ncycles must be in [0, 1000]");
  if (opts->nu1 < 0 || opts->nu1 > 64 || opts->nu2 < 0 || opts->nu2 > 64)
    return fail(HARD_ERR_INVALID_ARG, "nu1 and nu2 must be in [0, 64]");
  if (opts->ncoarse < 1 || opts->ncoarse > 1024)
    return fail(HARD_ERR_INVALID_ARG, "ncoarse must be in [1, 1024]");
  const Hierarchy H = hierarchy_of(G);
  if ((st = check_work(work, work_bytes, fld_workspace(H)))) return st;

  char* wb = static_cast<char*>(work);
  Solver S{G, H, {}, {}, {}, opts->nu1, opts->nu2, opts->ncoarse, 0, nullptr, nullptr,
           (hipStream_t)stream};
  // the one-workgroup tail starts at the first level from which all the
  // coarser levels' arrays (x, b, D: 48 bytes per colour slot) fit in the
  // workgroup's LDS and in the tail's table
  int dev = 0, lds_max = 0;
  hipError_t he;
  if ((he = hipGetDevice(&dev)) != hipSuccess ||
      (he = hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev)) !=
          hipSuccess)
    return hip_fail(he, "hard_rad_diffuse: device LDS size");
  S.tail = H.nlev;
  for (int l = 0; l < H.nlev; ++l) {
    long long need = 0;
    for (int m = l; m < H.nlev; ++m) need += 48LL * (split_elems(H, m) / 2);
    if (need <= (long long)lds_max && H.nlev - l <= FLD_TAIL_LEVELS) {
      S.tail = l;
      break;
    }
  }
  // (no level fits: every level, the coarsest included, runs in the
  // multi-workgroup kernels)
  S.Kbuf = reinterpret_cast<double*>(wb + 256);
  S.part = reinterpret_cast<double*>(wb + 256 + FLD_K_BYTES);
  size_t off = 256 + FLD_K_BYTES + align256(resid_slots(H) * sizeof(double));
  for (int l = 0; l < H.nlev; ++l) {
    FldLevel& L = S.lv[l];
    const size_t bytes = align256(split_elems(H, l) * sizeof(double));
    for (int d = 0; d < 3; ++d) {
      L.n[d] = H.n[l][d];
      L.halved[d] = H.halved[l][d];
      L.dx[d] = H.dx[l][d];
      L.dx2[d] = H.dx[l][d] * H.dx[l][d];
    }
    L.K = S.Kbuf + 3 * l;
    L.hx = (unsigned)((H.n[l][0] + 1) / 2);
    L.cs = (unsigned)H.n[l][1] * (unsigned)H.n[l][2] * L.hx;
    L.x = reinterpret_cast<double*>(wb + off);
    L.b = reinterpret_cast<double*>(wb + off + bytes);
    L.D = reinterpret_cast<double*>(wb + off + 2 * bytes);
    off += 3 * bytes;
    const int nch = (H.halved[l][0] ? 2 : 1) * (H.halved[l][1] ? 2 : 1) * (H.halved[l][2] ? 2 : 1);
    S.inv_children[l] = 1.0 / (double)nch;
  }
  for (int d = 0; d < 3; ++d) S.cm.per[d] = G.bc[d][0] == BC_PERIODIC;
  S.cm.dt = dt_dev;
  Control* ctl = reinterpret_cast<Control*>(wb);
  hipError_t e;
  if (G.dtype == HARD_F64) {
    double* Ud = static_cast<double*>(U);
    switch (G.ndim) {
      case 1: e = S.run<1>(Ud, opts->limiter, opts->ncycles, resid_dev, ctl); break;
      case 2: e = S.run<2>(Ud, opts->limiter, opts->ncycles, resid_dev, ctl); break;
      default: e = S.run<3>(Ud, opts->limiter, opts->ncycles, resid_dev, ctl); break;
    }
  } else {
    float* Uf = static_cast<float*>(U);
    switch (G.ndim) {
      case 1: e = S.run<1>(Uf, opts->limiter, opts->ncycles, resid_dev, ctl); break;
      case 2: e = S.run<2>(Uf, opts->limiter, opts->ncycles, resid_dev, ctl); break;
      default: e = S.run<3>(Uf, opts->limiter, opts->ncycles, resid_dev, ctl); break;
    }
  }
  if (e != hipSuccess) return hip_fail(e, "hard_rad_diffuse launch");
  return ok();
}

}  // extern "C"
