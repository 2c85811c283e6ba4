"""The diffusion oracle's pins catch plausible mistakes.

Each case plants one typical mistake in a copy of fld_oracle.cpp (a wrong
limiter coefficient, a dropped factor in the face coefficient or the
gradient, a wrong sign in the operator, a wrong transfer weight, a coarse
spacing that is not doubled, ...), builds it on the CPU and checks that at
least one quick pin fails, while every pin passes for the unmodified oracle.
The pins are the same kinds of facts as in test_oracle_fld.py: closed forms
of the limiter, D on constant-R states, the operator's symmetry, A 1 = 1 and
its Fourier eigenvalues, the dense solve, the closed-form decay of a mode and
a mesh-independent contraction per V-cycle.
"""
import numpy as np
import pytest

import oracle
from oracle import build as obuild
from oracle import fld

P, O, R = oracle.PERIODIC, oracle.OUTFLOW, oracle.REFLECT
C_LIGHT = 2.99792458e10
KAPPA = 0.4


def grid(n, bc, dx=None):
    return oracle.Grid(n, bc=bc, dx=dx, rad=(KAPPA, 0.6))


def rstate(g, seed):
    rng = np.random.default_rng(seed)
    U = np.zeros(g.shape)
    U[0] = 0.5 + rng.random(g.shape[1:])
    U[-1] = 1.0 + rng.random(g.shape[1:])
    return U


def dense(g, U, dt, limiter):
    N = int(np.prod(g.n))
    A = np.empty((N, N))
    for j in range(N):
        e = np.zeros(N)
        e[j] = 1.0
        A[:, j] = fld.fld_apply(g, U, dt, e.reshape(g.shape[1:]), limiter)[0].ravel()
    return A


def quick_pins():
    failed = []
    lam = {1.0: 0.3, 2.0: 0.25, 4.0: 6.0 / 34.0}
    if any(abs(fld.levermore(r) - v) > 1e-15 for r, v in lam.items()):
        failed.append("levermore")
    # D with R = 1 at interior cells
    g = grid((12, 10), (O, O, R, R), dx=(0.1, 0.1))
    xs = (np.arange(12) + 0.5) * 0.1
    ys = (np.arange(10) + 0.5) * 0.1
    x, y = xs[None, :], ys[:, None]
    E = 2.0 + 3.0 * x + 4.0 * y
    rho = 5.0 / (KAPPA * E)
    U = np.zeros(g.shape)
    U[0], U[-1] = rho, E
    D, _ = fld.fld_coefficient(g, U)
    if not np.allclose(D[1:-1, 1:-1], (C_LIGHT * 0.3 / (KAPPA * rho))[1:-1, 1:-1], rtol=1e-13):
        failed.append("coefficient")
    # wall cells see half the gradient
    g1 = grid((8,), (O, O), dx=(1.0,))
    E1 = 10.5 + np.arange(8.0)
    U1 = np.zeros(g1.shape)
    U1[0], U1[-1] = 1.0, E1
    D1, _ = fld.fld_coefficient(g1, U1)
    Rw = 0.5 / (KAPPA * E1[0])
    if abs(D1[0] - C_LIGHT * (2 + Rw) / (6 + 3 * Rw + Rw * Rw) / KAPPA) > 1e-13 * D1[0]:
        failed.append("wall gradient")
    # operator structure and eigenvalues
    for n, bc in (((6, 4), (P, P, O, O)), ((4, 2, 3), (R, R, P, P, O, O))):
        gs = grid(n, bc)
        A = dense(gs, rstate(gs, 3), 2e-12, fld.LEVERMORE)
        N = A.shape[0]
        if not (np.allclose(A, A.T, rtol=0, atol=1e-15 * np.abs(A).max())
                and np.allclose(A @ np.ones(N), 1.0, rtol=0, atol=1e-13 * np.abs(A).max())):
            failed.append(f"operator {n}")
    n = 32
    gp = grid((n, n), (P, P, P, P))
    xc = (np.arange(n) + 0.5) / n
    v = np.cos(2 * np.pi * 3 * xc)[None, :] * np.cos(2 * np.pi * 5 * xc)[:, None]
    Up = np.zeros(gp.shape)
    Up[0], Up[-1] = 2.0, 1.0
    Dc, dt = C_LIGHT / (3.0 * KAPPA * 2.0), 1e-12
    lam_v = 1.0 + 4.0 * dt * Dc * n * n * (np.sin(np.pi * 3 / n) ** 2 + np.sin(np.pi * 5 / n) ** 2)
    Av, _ = fld.fld_apply(gp, Up, dt, v, fld.EDDINGTON)
    if not np.allclose(Av, lam_v * v, rtol=0, atol=1e-12 * lam_v):
        failed.append("fourier eigenvalue")
    # mode decay through the multigrid solve (walls in x, periodic in y)
    gw = grid((32, 16), (O, O, P, P))
    xw = (np.arange(32) + 0.5) / 32
    yw = (np.arange(16) + 0.5) / 16
    mode = np.cos(np.pi * 2 * xw)[None, :] * np.cos(2 * np.pi * 1 * yw)[:, None]
    Uw = np.zeros(gw.shape)
    Uw[0], Uw[-1] = 2.0, 10.0 + mode
    lam_w = 1.0 + 4.0 * dt * Dc * (32 * 32 * np.sin(np.pi * 2 / 64) ** 2
                                   + 16 * 16 * np.sin(np.pi * 1 / 16) ** 2)
    X, _, res = fld.rad_diffuse(gw, Uw, dt, ncycles=24, limiter=fld.EDDINGTON)
    if not (np.all(np.isfinite(X[-1])) and np.allclose(X[-1], 10.0 + mode / lam_w, rtol=0,
                                                        atol=1e-11)):
        failed.append("mode decay")
    # dense solve of the operator and contraction per cycle
    gd = grid((8, 4), (P, P, O, O))
    Ud = rstate(gd, 4)
    A = dense(gd, Ud, 5e-12, fld.LEVERMORE)
    want = np.linalg.solve(A, Ud[-1].ravel()).reshape(gd.shape[1:])
    X, _, _ = fld.rad_diffuse(gd, Ud, 5e-12, ncycles=30)
    if not np.allclose(X[-1], want, rtol=1e-12):
        failed.append("dense solve")
    # textbook contraction of V(2,2) with a smooth coefficient (Eddington,
    # smooth rho): below 0.1 per cycle
    gc = grid((64, 64), (P, P, O, O))
    Uc = rstate(gc, 5)
    xc = (np.arange(64) + 0.5) / 64
    Uc[0] = 1.0 + 0.5 * np.sin(2 * np.pi * xc)[None, :] * np.cos(np.pi * xc)[:, None]
    X, _, res = fld.rad_diffuse(gc, Uc, 1e-10, ncycles=8, limiter=fld.EDDINGTON)
    if not (res[-1] / res[2]) ** (1 / 6) < 0.1:
        failed.append("contraction")
    return failed


MUTATIONS = {
    "face coefficient without the mean": ("const double Dface = 0.5 * (L.D[a] + L.D[b]);",
                                          "const double Dface = L.D[a] + L.D[b];"),
    "face coefficient over dx": ("P.dt * Dface / (L.dx[d] * L.dx[d])", "P.dt * Dface / L.dx[d]"),
    "operator sign": ("Ax += a * (x[c] - x[nb]);", "Ax -= a * (x[c] - x[nb]);"),
    "relaxation diagonal": ("den += a;", "den += 2.0 * a;"),
    "relaxation neighbour sign": ("num += a * L.x[nb];", "num -= a * L.x[nb];"),
    "limiter coefficient": ("6.0 + 3.0 * R + R * R", "6.0 + 2.0 * R + R * R"),
    "gradient without the half": ("(E[hi] - E[lo]) / (2.0 * L.dx[d])", "(E[hi] - E[lo]) / L.dx[d]"),
    "gradient not square-rooted": ("std::sqrt(g2) / (rho[c] * kappa * E[c])",
                                   "g2 / (rho[c] * kappa * E[c])"),
    "wall neighbour is the far cell": ("if (lo < 0) lo = c;", "if (lo < 0) lo = hi;"),
    "D without rho": ("C_LIGHT * lam / (kappa * rho[c])", "C_LIGHT * lam / kappa"),
    "restriction sums": ("C.b[c] = s * inv;", "C.b[c] = s;"),
    "residual sign": ("const double r = F.b[F.at(i, j, k)] - apply_row(F, P, F.x, i, j, k);",
                      "const double r = apply_row(F, P, F.x, i, j, k) - F.b[F.at(i, j, k)];"),
    "prolongation far weight": ("wf[d] = 0.25;", "wf[d] = 0.5;"),
    "prolongation far side": ("int64_t q = neighbour(I, C.n[d], side, P.bc[d]);",
                              "int64_t q = neighbour(I, C.n[d], 1 - side, P.bc[d]);"),
    "coarse spacing not doubled": ("C.dx[d] = h ? 2.0 * F.dx[d] : F.dx[d];", "C.dx[d] = F.dx[d];"),
    "correction subtracted": ("F.x[F.at(i, j, k)] += v;", "F.x[F.at(i, j, k)] -= v;"),
    "periodic wrap to the wrong end": ("if (periodic && n > 1) return n - 1;",
                                       "if (periodic && n > 1) return 0;"),
}


@pytest.fixture
def restore_fld():
    yield
    fld.use_library(obuild.FLD_LIB)


def test_unmodified_fld_oracle_passes_quick_pins(restore_fld):
    fld.use_library(obuild.FLD_LIB)
    assert quick_pins() == []


@pytest.mark.parametrize("name", list(MUTATIONS))
def test_planted_fld_mistake_is_caught(name, restore_fld, tmp_path):
    old, new = MUTATIONS[name]
    src = open(obuild.FLD_SRC[0]).read()
    assert src.count(old) == 1, f"mutation site missing or repeated: {old}"
    mutated = tmp_path / "fld_oracle_mutant.cpp"
    mutated.write_text(src.replace(old, new))
    lib = obuild.build_fld(src=str(mutated), out=str(tmp_path / "libfld_oracle_mutant.so"))
    fld.use_library(lib)
    try:
        with np.errstate(all="ignore"):
            failed = quick_pins()
    finally:
        fld.use_library(obuild.FLD_LIB)
    assert failed, f"no pin caught: {name}"
