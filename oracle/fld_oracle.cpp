// Plain CPU oracle for the implicit flux-limited radiation diffusion step and
// its geometric multigrid solver.
//
// TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
// benchmark's CPU-baseline leg may load this code.  It shares nothing with
// the HIP path: no headers, no helpers, no tables.
//
// What it computes (HARD paper, sections 2.2.1 and 2.2.2):
//   * the diffusive part of the radiation energy equation (the paper's
//     equation "radiation"): d_t E = div(D grad E) with D = c lambda/(kappa rho);
//   * lambda from the Levermore flux limiter, lambda = (2+R)/(6+3R+R^2) with
//     R = |grad E|/(rho kappa E) (the bridge law of section 2.2.1), or the
//     constant 1/3 of the optically thick (Eddington) limit that the same
//     section derives from it;
//   * one backward-Euler step of that equation with D taken from the state at
//     the start of the step, so that the operator is linear, as the multigrid
//     discussion of section 2.2.2 requires:  (I - dt div D grad) E_new = E_old;
//   * solved by geometric multigrid V-cycles with regular coarsening (section
//     2.2.2: the residual equation A e = r solved on every grid coarser than
//     the solution grid with initial guess zero, the correction carried back
//     to the finer grid, relaxation before and after, and a relaxation method
//     on the coarsest grid).
//
// Readings where the paper gives no detail (each one is a choice, stated):
//   * grad E at a cell centre by central differences; a non-periodic side
//     takes the edge cell itself as its neighbour (zero normal gradient);
//   * the face coefficient is dt * (D_i + D_j)/2 / dx^2 (arithmetic mean of
//     the two cells); non-periodic domain faces carry no flux (zero-flux
//     walls), and a periodic axis of one cell carries none either (the face
//     joins the cell to itself);
//   * the smoother is red-black Gauss-Seidel (cells with i+j+k even first);
//     one sweep is a red half-sweep followed by a black one;
//   * coarsening halves every axis whose size is even; a periodic axis is
//     halved only when the half is even or one (so red-black colouring stays
//     consistent across the periodic seam); coarsening stops when no axis can
//     be halved;
//   * coarse D is the mean of D over the children; coarse faces are built from
//     it with the same formula and the coarse spacing (rediscretisation);
//   * restriction averages the residual over the children; prolongation is
//     linear interpolation (weights 3/4 and 1/4 along each halved axis),
//     with the edge value repeated beyond a non-periodic side;
//   * the finest grid starts from x = E_old; the coarsest grid is relaxed
//     `ncoarse` sweeps from zero (exact after one sweep when it is one cell).
//
// Everything is FP64, compiled with -ffp-contract=off, in the loop order the
// code shows.  OpenMP splits the loops over the slowest axis; within a colour
// every cell depends only on cells of the other colour, so the result does
// not depend on the thread count.

#include <cmath>
#include <cstdint>
#include <vector>

namespace fld_oracle {

constexpr double C_LIGHT = 2.99792458e10;  // cm/s (CGS, as the paper's tests)

struct Level {
  int64_t n[3];
  double dx[3];
  int halved[3];  // axis halved from the next finer level
  std::vector<double> x, b, D;
  int64_t cells() const { return n[0] * n[1] * n[2]; }
  int64_t at(int64_t i, int64_t j, int64_t k) const { return (k * n[1] + j) * n[0] + i; }
};

struct Problem {
  int ndim;
  int bc[3][2];
  double dt;
};

// Neighbour of position p on an axis of size n on side s (0 low, 1 high);
// -1 when the face carries no flux.
inline int64_t neighbour(int64_t p, int64_t n, int s, const int* bc) {
  const int periodic = bc[0] == 0;
  if (s == 0) {
    if (p > 0) return p - 1;
    if (periodic && n > 1) return n - 1;
    return -1;
  }
  if (p < n - 1) return p + 1;
  if (periodic && n > 1) return 0;
  return -1;
}

// Index of the neighbour across face (d, s) of cell (i,j,k), or -1.
inline int64_t face_neighbour(const Level& L, const Problem& P, int64_t i, int64_t j,
                              int64_t k, int d, int s) {
  int64_t c[3] = {i, j, k};
  const int64_t q = neighbour(c[d], L.n[d], s, P.bc[d]);
  if (q < 0) return -1;
  c[d] = q;
  return L.at(c[0], c[1], c[2]);
}

// a_f = dt D_f / dx_d^2 with the face value D_f = (D_a + D_b)/2.
inline double face_coeff(const Level& L, const Problem& P, int d, int64_t a, int64_t b) {
  const double Dface = 0.5 * (L.D[a] + L.D[b]);
  return P.dt * Dface / (L.dx[d] * L.dx[d]);
}

// (A x)_c = x_c + sum over faces a_f (x_c - x_nb)
double apply_row(const Level& L, const Problem& P, const std::vector<double>& x, int64_t i,
                 int64_t j, int64_t k) {
  const int64_t c = L.at(i, j, k);
  double Ax = x[c];
  for (int d = 0; d < P.ndim; ++d)
    for (int s = 0; s < 2; ++s) {
      const int64_t nb = face_neighbour(L, P, i, j, k, d, s);
      if (nb < 0) continue;
      const double a = face_coeff(L, P, d, c, nb);
      Ax += a * (x[c] - x[nb]);
    }
  return Ax;
}

// Gauss-Seidel update of one cell: x_c = (b_c + sum a_f x_nb)/(1 + sum a_f)
void relax_cell(Level& L, const Problem& P, int64_t i, int64_t j, int64_t k) {
  const int64_t c = L.at(i, j, k);
  double num = L.b[c];
  double den = 1.0;
  for (int d = 0; d < P.ndim; ++d)
    for (int s = 0; s < 2; ++s) {
      const int64_t nb = face_neighbour(L, P, i, j, k, d, s);
      if (nb < 0) continue;
      const double a = face_coeff(L, P, d, c, nb);
      num += a * L.x[nb];
      den += a;
    }
  L.x[c] = num / den;
}

void relax(Level& L, const Problem& P, int sweeps) {
  for (int sw = 0; sw < sweeps; ++sw)
    for (int colour = 0; colour < 2; ++colour) {
#pragma omp parallel for schedule(static)
      for (int64_t k = 0; k < L.n[2]; ++k)
        for (int64_t j = 0; j < L.n[1]; ++j)
          for (int64_t i = 0; i < L.n[0]; ++i)
            if (((i + j + k) & 1) == colour) relax_cell(L, P, i, j, k);
    }
}

// Children of coarse cell (I,J,K) in finer level F: along a halved axis the
// two cells 2I, 2I+1, otherwise the cell I itself.  Visits them x fastest.
template <class Fn>
void for_children(const Level& C, int64_t I, int64_t J, int64_t K, Fn fn) {
  const int64_t c[3] = {I, J, K};
  int64_t lo[3], cnt[3];
  for (int d = 0; d < 3; ++d) {
    lo[d] = C.halved[d] ? 2 * c[d] : c[d];
    cnt[d] = C.halved[d] ? 2 : 1;
  }
  for (int64_t dz = 0; dz < cnt[2]; ++dz)
    for (int64_t dy = 0; dy < cnt[1]; ++dy)
      for (int64_t dxx = 0; dxx < cnt[0]; ++dxx) fn(lo[0] + dxx, lo[1] + dy, lo[2] + dz);
}

inline double nchildren(const Level& C) {
  return double((C.halved[0] ? 2 : 1) * (C.halved[1] ? 2 : 1) * (C.halved[2] ? 2 : 1));
}

// Coarse D: mean over the children.
void coarsen_D(const Level& F, Level& C) {
  const double inv = 1.0 / nchildren(C);
#pragma omp parallel for schedule(static)
  for (int64_t K = 0; K < C.n[2]; ++K)
    for (int64_t J = 0; J < C.n[1]; ++J)
      for (int64_t I = 0; I < C.n[0]; ++I) {
        double s = 0.0;
        for_children(C, I, J, K, [&](int64_t i, int64_t j, int64_t k) { s += F.D[F.at(i, j, k)]; });
        C.D[C.at(I, J, K)] = s * inv;
      }
}

// Coarse right-hand side: the fine residual averaged over the children;
// coarse initial guess zero.
void restrict_residual(const Level& F, const Problem& P, Level& C) {
  const double inv = 1.0 / nchildren(C);
#pragma omp parallel for schedule(static)
  for (int64_t K = 0; K < C.n[2]; ++K)
    for (int64_t J = 0; J < C.n[1]; ++J)
      for (int64_t I = 0; I < C.n[0]; ++I) {
        double s = 0.0;
        for_children(C, I, J, K, [&](int64_t i, int64_t j, int64_t k) {
          const double r = F.b[F.at(i, j, k)] - apply_row(F, P, F.x, i, j, k);
          s += r;
        });
        const int64_t c = C.at(I, J, K);
        C.b[c] = s * inv;
        C.x[c] = 0.0;
      }
}

// x_fine += linear interpolation of the coarse correction.
void prolong_add(Level& F, const Problem& P, const Level& C) {
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < F.n[2]; ++k)
    for (int64_t j = 0; j < F.n[1]; ++j)
      for (int64_t i = 0; i < F.n[0]; ++i) {
        const int64_t f[3] = {i, j, k};
        int64_t near[3], far[3];
        double wn[3], wf[3];
        int cnt[3];
        for (int d = 0; d < 3; ++d) {
          if (!C.halved[d]) {
            near[d] = far[d] = f[d];
            wn[d] = 1.0;
            wf[d] = 0.0;
            cnt[d] = 1;
            continue;
          }
          const int64_t I = f[d] >> 1;
          const int side = int(f[d] & 1);  // 0: low child -> far cell below
          int64_t q = neighbour(I, C.n[d], side, P.bc[d]);
          if (q < 0) q = I;  // beyond a wall: repeat the edge value
          near[d] = I;
          far[d] = q;
          wn[d] = 0.75;
          wf[d] = 0.25;
          cnt[d] = 2;
        }
        double v = 0.0;
        for (int cz = 0; cz < cnt[2]; ++cz)
          for (int cy = 0; cy < cnt[1]; ++cy)
            for (int cx = 0; cx < cnt[0]; ++cx) {
              const double w = (cx ? wf[0] : wn[0]) * (cy ? wf[1] : wn[1]) * (cz ? wf[2] : wn[2]);
              const double xc = C.x[C.at(cx ? far[0] : near[0], cy ? far[1] : near[1],
                                          cz ? far[2] : near[2])];
              v += w * xc;
            }
        F.x[F.at(i, j, k)] += v;
      }
}

void vcycle(std::vector<Level>& lv, const Problem& P, size_t l, int nu1, int nu2, int ncoarse) {
  Level& L = lv[l];
  if (l + 1 == lv.size()) {
    relax(L, P, ncoarse);
    return;
  }
  relax(L, P, nu1);
  restrict_residual(L, P, lv[l + 1]);
  vcycle(lv, P, l + 1, nu1, nu2, ncoarse);
  prolong_add(L, P, lv[l + 1]);
  relax(L, P, nu2);
}

double residual_norm(const Level& L, const Problem& P) {
  double s = 0.0;
  for (int64_t k = 0; k < L.n[2]; ++k)
    for (int64_t j = 0; j < L.n[1]; ++j)
      for (int64_t i = 0; i < L.n[0]; ++i) {
        const double r = L.b[L.at(i, j, k)] - apply_row(L, P, L.x, i, j, k);
        s += r * r;
      }
  return std::sqrt(s);
}

// The level sizes of the hierarchy (regular coarsening rule above).
std::vector<Level> hierarchy(int ndim, const int64_t* n, const double* dx, const Problem& P) {
  std::vector<Level> lv(1);
  for (int d = 0; d < 3; ++d) {
    lv[0].n[d] = d < ndim ? n[d] : 1;
    lv[0].dx[d] = d < ndim ? dx[d] : 1.0;
    lv[0].halved[d] = 0;
  }
  for (;;) {
    const Level& F = lv.back();
    Level C;
    int any = 0;
    for (int d = 0; d < 3; ++d) {
      const int64_t m = F.n[d];
      const int periodic = P.bc[d][0] == 0;
      int h = d < ndim && m % 2 == 0;
      if (h && periodic) h = (m / 2) % 2 == 0 || m / 2 == 1;
      C.halved[d] = h;
      C.n[d] = h ? m / 2 : m;
      C.dx[d] = h ? 2.0 * F.dx[d] : F.dx[d];
      any |= h;
    }
    if (!any) break;
    lv.push_back(C);
  }
  for (Level& L : lv) {
    L.x.assign(L.cells(), 0.0);
    L.b.assign(L.cells(), 0.0);
    L.D.assign(L.cells(), 0.0);
  }
  return lv;
}

double levermore(double R) { return (2.0 + R) / (6.0 + 3.0 * R + R * R); }

// D per cell of the finest grid from rho and E; returns 1 if some cell is
// non-physical (rho <= 0, E <= 0 or a non-finite D).
int fld_coefficient(Level& L, const Problem& P, const double* rho, const double* E,
                    double kappa, int limiter) {
  int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
  for (int64_t k = 0; k < L.n[2]; ++k)
    for (int64_t j = 0; j < L.n[1]; ++j)
      for (int64_t i = 0; i < L.n[0]; ++i) {
        const int64_t c = L.at(i, j, k);
        double g2 = 0.0;
        for (int d = 0; d < P.ndim; ++d) {
          int64_t lo = face_neighbour(L, P, i, j, k, d, 0);
          int64_t hi = face_neighbour(L, P, i, j, k, d, 1);
          if (lo < 0) lo = c;
          if (hi < 0) hi = c;
          const double g = (E[hi] - E[lo]) / (2.0 * L.dx[d]);
          g2 += g * g;
        }
        double lam = 1.0 / 3.0;
        if (limiter) {
          const double R = std::sqrt(g2) / (rho[c] * kappa * E[c]);
          lam = levermore(R);
        }
        const double D = C_LIGHT * lam / (kappa * rho[c]);
        L.D[c] = D;
        if (!(rho[c] > 0.0) || !(E[c] > 0.0) || !std::isfinite(D)) bad = 1;
      }
  return bad;
}

int setup(std::vector<Level>& lv, const Problem& P, const double* U, int nvar, double kappa,
          int limiter) {
  Level& L = lv[0];
  const int64_t N = L.cells();
  const double* rho = U;
  const double* E = U + (nvar - 1) * N;
  const int bad = fld_coefficient(L, P, rho, E, kappa, limiter);
  for (size_t l = 1; l < lv.size(); ++l) coarsen_D(lv[l - 1], lv[l]);
  for (int64_t c = 0; c < N; ++c) {
    L.b[c] = E[c];
    L.x[c] = E[c];
  }
  return bad;
}

Problem make_problem(int ndim, const int* bc, double dt) {
  Problem P;
  P.ndim = ndim;
  for (int d = 0; d < 3; ++d) {
    P.bc[d][0] = d < ndim ? bc[2 * d] : 0;
    P.bc[d][1] = d < ndim ? bc[2 * d + 1] : 0;
  }
  P.dt = dt;
  return P;
}

// A periodic axis of odd size above one cannot be coloured red-black.
int valid(int ndim, const int64_t* n, const int* bc) {
  for (int d = 0; d < ndim; ++d)
    if (bc[2 * d] == 0 && n[d] > 1 && n[d] % 2) return 0;
  return 1;
}

}  // namespace fld_oracle

using namespace fld_oracle;

extern "C" {

double oracle_levermore(double R) { return levermore(R); }

// Number of levels and their sizes (levels_n: 3 per level, at most max_levels).
int oracle_gmg_levels(int ndim, const int64_t* n, const double* dx, const int* bc, int max_levels,
                      int64_t* levels_n) {
  const Problem P = make_problem(ndim, bc, 0.0);
  std::vector<Level> lv = hierarchy(ndim, n, dx, P);
  for (size_t l = 0; l < lv.size() && int(l) < max_levels; ++l)
    for (int d = 0; d < 3; ++d) levels_n[3 * l + d] = lv[l].n[d];
  return int(lv.size());
}

// D of every finest-grid cell; returns 1 on a non-physical cell, -1 on a bad grid.
int oracle_fld_coefficient(int ndim, const int64_t* n, const double* dx, const int* bc,
                           double kappa, int limiter, const double* U, int nvar, double* D) {
  if (!valid(ndim, n, bc)) return -1;
  const Problem P = make_problem(ndim, bc, 0.0);
  std::vector<Level> lv = hierarchy(ndim, n, dx, P);
  const int64_t N = lv[0].cells();
  const int bad = fld_coefficient(lv[0], P, U, U + (nvar - 1) * N, kappa, limiter);
  for (int64_t c = 0; c < N; ++c) D[c] = lv[0].D[c];
  return bad;
}

// y = A x on the finest grid, A = I - dt div D grad with D from U.
int oracle_fld_apply(int ndim, const int64_t* n, const double* dx, const int* bc, double kappa,
                     int limiter, double dt, const double* U, int nvar, const double* x,
                     double* y) {
  if (!valid(ndim, n, bc)) return -1;
  const Problem P = make_problem(ndim, bc, dt);
  std::vector<Level> lv = hierarchy(ndim, n, dx, P);
  Level& L = lv[0];
  const int64_t N = L.cells();
  const int bad = fld_coefficient(L, P, U, U + (nvar - 1) * N, kappa, limiter);
  std::vector<double> xv(x, x + N);
  for (int64_t k = 0; k < L.n[2]; ++k)
    for (int64_t j = 0; j < L.n[1]; ++j)
      for (int64_t i = 0; i < L.n[0]; ++i) y[L.at(i, j, k)] = apply_row(L, P, xv, i, j, k);
  return bad;
}

// One implicit diffusion step of the radiation field (last field of U, in
// place) by `ncycles` V(nu1, nu2) cycles.  resid (or null) receives the
// finest-grid residual 2-norm before the first cycle and after each one.
int oracle_rad_diffuse(int ndim, const int64_t* n, const double* dx, const int* bc, double kappa,
                       int limiter, double dt, int ncycles, int nu1, int nu2, int ncoarse,
                       double* U, int nvar, double* resid) {
  if (!valid(ndim, n, bc)) return -1;
  const Problem P = make_problem(ndim, bc, dt);
  std::vector<Level> lv = hierarchy(ndim, n, dx, P);
  const int bad = setup(lv, P, U, nvar, kappa, limiter);
  if (resid) resid[0] = residual_norm(lv[0], P);
  for (int c = 0; c < ncycles; ++c) {
    vcycle(lv, P, 0, nu1, nu2, ncoarse);
    if (resid) resid[c + 1] = residual_norm(lv[0], P);
  }
  const int64_t N = lv[0].cells();
  double* E = U + (nvar - 1) * N;
  for (int64_t c = 0; c < N; ++c) E[c] = lv[0].x[c];
  return bad;
}

}  // extern "C"
