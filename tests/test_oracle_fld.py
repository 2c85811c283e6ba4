"""Pins of the oracle's implicit flux-limited radiation diffusion step and its
geometric multigrid solver (paper section 2.2.1: the diffusion flux with the
Levermore limiter and its Eddington limit; section 2.2.2: the multigrid
solver of A u = f, the residual equation and the V-cycle).

What fixes the expected values, independently of the oracle's own code:
  * the limiter's closed-form values and both limits the paper states
    (lambda -> 1/3 for R -> 0, R lambda -> 1 for R -> infinity);
  * D on states built so that R is a chosen constant (linear E, rho scaled);
  * the operator: symmetric, A 1 = 1, sum(A x) = sum(x) (flux form), every
    eigenvalue >= 1, and the closed-form eigenvalues of Fourier and cosine
    modes when D is constant;
  * the solver: the V-cycle iterate converges to NumPy's dense solve of the
    assembled operator, to the closed-form mode decay, with a mesh-independent
    contraction per cycle; the converged step conserves the total and obeys
    the discrete maximum principle; dt = 0 leaves E unchanged.
"""
import numpy as np
import pytest

import oracle
from oracle import fld

P, O, R = oracle.PERIODIC, oracle.OUTFLOW, oracle.REFLECT
C_LIGHT = 2.99792458e10  # cm/s, written out here independently of the oracle
KAPPA = 0.4


def grid(n, bc, dx=None):
    return oracle.Grid(n, bc=bc, dx=dx, rad=(KAPPA, 0.6))


def state(g, rho, E):
    U = np.zeros(g.shape)
    U[0] = rho
    U[-1] = E
    return U


def random_state(g, seed):
    rng = np.random.default_rng(seed)
    shp = g.shape[1:]
    return state(g, 0.5 + rng.random(shp), 1.0 + rng.random(shp))


def centres(g):
    """Cell-centre coordinates, each of the grid's cell shape (x fastest)."""
    axes = [(np.arange(m) + 0.5) * h for m, h in zip(g.n, g.dx)]
    mesh = np.meshgrid(*reversed(axes), indexing="ij")
    return list(reversed(mesh))


def assemble(g, U, dt, limiter):
    """Dense matrix of the oracle's operator, column by column."""
    N = int(np.prod(g.n))
    A = np.empty((N, N))
    for j in range(N):
        e = np.zeros(N)
        e[j] = 1.0
        y, st = fld.fld_apply(g, U, dt, e.reshape(g.shape[1:]), limiter)
        assert st == 0
        A[:, j] = y.ravel()
    return A


# ---------------------------------------------------------------- limiter


def test_levermore_closed_form_values():
    assert fld.levermore(0.0) == 1.0 / 3.0
    assert fld.levermore(1.0) == pytest.approx(3.0 / 10.0, rel=1e-15)
    assert fld.levermore(2.0) == pytest.approx(1.0 / 4.0, rel=1e-15)
    assert fld.levermore(4.0) == pytest.approx(6.0 / 34.0, rel=1e-15)


def test_levermore_limits():
    # optically thick: lambda -> 1/3; free streaming: |F| = lambda c |grad E|/(kappa rho)
    # -> c E, i.e. R lambda -> 1
    assert abs(fld.levermore(1e-9) - 1.0 / 3.0) < 1e-9
    for R in (1e6, 1e9):
        assert abs(R * fld.levermore(R) - 1.0) < 2.0 / R
    # lambda decreases monotonically
    Rs = np.logspace(-3, 3, 61)
    lam = np.array([fld.levermore(r) for r in Rs])
    assert np.all(np.diff(lam) < 0)


# ---------------------------------------------------------------- D


@pytest.mark.parametrize("Rt, lam", [(1.0, 3.0 / 10.0), (2.0, 1.0 / 4.0), (4.0, 6.0 / 34.0)])
def test_coefficient_on_constant_R_states(Rt, lam):
    # E = 2 + 3x + 4y gives |grad E| = 5 at interior cells (central differences
    # are exact on linear data); rho = 5/(kappa E R) then makes R = Rt there
    g = grid((12, 10), (O, O, R, R), dx=(0.1, 0.1))
    x, y = centres(g)
    E = 2.0 + 3.0 * x + 4.0 * y
    rho = 5.0 / (KAPPA * E * Rt)
    D, st = fld.fld_coefficient(g, state(g, rho, E))
    assert st == 0
    want = C_LIGHT * lam / (KAPPA * rho)
    inner = (slice(1, -1), slice(1, -1))
    np.testing.assert_allclose(D[inner], want[inner], rtol=1e-13)


def test_coefficient_eddington_ignores_gradient():
    g = grid((8, 6, 4), (P, P, O, O, R, R))
    U = random_state(g, 1)
    D, st = fld.fld_coefficient(g, U, fld.EDDINGTON)
    assert st == 0
    np.testing.assert_allclose(D, C_LIGHT / (3.0 * KAPPA * U[0]), rtol=1e-15)


def test_coefficient_zero_gradient_at_walls():
    # a wall cell takes itself as the neighbour beyond the wall, so with E
    # linear in x the wall cells see half the interior gradient
    g = grid((8,), (O, O), dx=(1.0,))
    x = centres(g)[0]
    E = 10.0 + x
    rho = np.ones(8)
    D, _ = fld.fld_coefficient(g, state(g, rho, E))
    R_in = 1.0 / (KAPPA * E)
    R_wall = 0.5 / (KAPPA * E)
    lam = lambda R: (2 + R) / (6 + 3 * R + R * R)  # the paper's limiter, for the wall value
    assert D[3] == pytest.approx(C_LIGHT * lam(R_in[3]) / KAPPA, rel=1e-14)
    assert D[0] == pytest.approx(C_LIGHT * lam(R_wall[0]) / KAPPA, rel=1e-14)
    assert D[7] == pytest.approx(C_LIGHT * lam(R_wall[7]) / KAPPA, rel=1e-14)


def test_nonphysical_cells_are_flagged():
    g = grid((8,), (P, P))
    U = random_state(g, 2)
    U[-1, 3] = -1.0
    assert fld.fld_coefficient(g, U)[1] == 1
    U = random_state(g, 2)
    U[0, 5] = 0.0
    assert fld.fld_coefficient(g, U)[1] == 1


def test_odd_periodic_axis_is_rejected():
    g = grid((7, 4), (P, P, O, O))
    assert fld.fld_coefficient(g, random_state(g, 0))[1] == -1


# ---------------------------------------------------------------- operator


OPS = [((10,), (P, P)), ((9,), (O, R)), ((6, 4), (P, P, O, O)), ((4, 2, 3), (R, R, P, P, O, O))]
# multigrid hierarchies of two or more levels, small enough for a dense solve
SOLVES = [((16,), (P, P)), ((12,), (O, R)), ((8, 4), (P, P, O, O)),
          ((4, 2, 6), (R, R, P, P, O, O)), ((8, 8), (P, P, P, P))]


@pytest.mark.parametrize("n, bc", OPS)
@pytest.mark.parametrize("limiter", [fld.EDDINGTON, fld.LEVERMORE])
def test_operator_structure(n, bc, limiter):
    g = grid(n, bc)
    U = random_state(g, 3)
    dt = 2e-12
    A = assemble(g, U, dt, limiter)
    N = A.shape[0]
    # symmetric (the face coefficient is shared by both cells)
    np.testing.assert_allclose(A, A.T, rtol=0, atol=1e-15 * np.abs(A).max())
    # constants are not diffused: A 1 = 1
    np.testing.assert_allclose(A @ np.ones(N), np.ones(N), rtol=0, atol=1e-13 * np.abs(A).max())
    # flux form: the column sums are one, so sum(A x) = sum(x)
    np.testing.assert_allclose(A.sum(axis=0), np.ones(N), rtol=0, atol=1e-13 * np.abs(A).max())
    # off-diagonals are <= 0 and the spectrum starts at exactly 1
    off = A - np.diag(np.diag(A))
    assert np.all(off <= 0.0)
    assert (off < 0).sum() > 0
    ev = np.linalg.eigvalsh(0.5 * (A + A.T))
    assert ev.min() == pytest.approx(1.0, rel=1e-9)


def test_operator_fourier_eigenvalues_periodic():
    # D constant (Eddington, uniform rho): cos(2 pi k x) has eigenvalue
    # 1 + 4 dt D sin^2(pi k / n) / dx^2 per axis
    n, k = 32, 3
    g = grid((n, n), (P, P, P, P))
    x, y = centres(g)
    U = state(g, 2.0, 1.0 + x)
    D = C_LIGHT / (3.0 * KAPPA * 2.0)
    dt = 1e-12
    for kx, ky in ((k, 0), (k, 5)):
        v = np.cos(2 * np.pi * kx * x) * np.cos(2 * np.pi * ky * y)
        Av, st = fld.fld_apply(g, U, dt, v, fld.EDDINGTON)
        lam = 1.0 + 4.0 * dt * D * n * n * (np.sin(np.pi * kx / n) ** 2 + np.sin(np.pi * ky / n) ** 2)
        np.testing.assert_allclose(Av, lam * v, rtol=0, atol=1e-12 * lam)


@pytest.mark.parametrize("bc", [(O, O), (R, R), (O, R)])
def test_operator_cosine_eigenvalues_walls(bc):
    # zero-flux walls: cos(pi k (i + 1/2)/n) has eigenvalue 1 + 4 dt D sin^2(pi k/(2n))/dx^2
    n, k = 24, 5
    g = grid((n,), bc)
    i = np.arange(n)
    v = np.cos(np.pi * k * (i + 0.5) / n)
    U = state(g, 3.0, 1.0 + 0.1 * i)
    D = C_LIGHT / (3.0 * KAPPA * 3.0)
    dt = 3e-12
    Av, st = fld.fld_apply(g, U, dt, v, fld.EDDINGTON)
    lam = 1.0 + 4.0 * dt * D * n * n * np.sin(np.pi * k / (2 * n)) ** 2
    np.testing.assert_allclose(Av, lam * v, rtol=0, atol=1e-12 * lam)


# ---------------------------------------------------------------- hierarchy


def test_coarsening_rule():
    assert fld.gmg_levels(grid((32, 32), (P, P, O, O))) == [
        (32, 32, 1), (16, 16, 1), (8, 8, 1), (4, 4, 1), (2, 2, 1), (1, 1, 1)]
    # periodic axes are halved only to an even size or to one cell
    assert fld.gmg_levels(grid((48, 40, 24), (P, P, O, O, R, R))) == [
        (48, 40, 24), (24, 20, 12), (12, 10, 6), (6, 5, 3)]
    assert fld.gmg_levels(grid((6,), (P, P))) == [(6, 1, 1)]
    assert fld.gmg_levels(grid((6,), (O, O))) == [(6, 1, 1), (3, 1, 1)]
    # an axis that can no longer be halved stays while the others go on
    assert fld.gmg_levels(grid((12, 4), (O, O, O, O))) == [
        (12, 4, 1), (6, 2, 1), (3, 1, 1)]


# ---------------------------------------------------------------- solver


@pytest.mark.parametrize("n, bc", SOLVES)
@pytest.mark.parametrize("limiter", [fld.EDDINGTON, fld.LEVERMORE])
def test_vcycles_converge_to_the_dense_solve(n, bc, limiter):
    g = grid(n, bc)
    U = random_state(g, 4)
    dt = 5e-12
    A = assemble(g, U, dt, limiter)
    want = np.linalg.solve(A, U[-1].ravel()).reshape(g.shape[1:])
    X, st, res = fld.rad_diffuse(g, U, dt, ncycles=30, limiter=limiter)
    assert st == 0
    np.testing.assert_allclose(X[-1], want, rtol=1e-12)
    np.testing.assert_array_equal(X[:-1], U[:-1])  # only E_r changes


@pytest.mark.parametrize("n, bc", [((64,), (P, P)), ((32, 32), (O, O, P, P)),
                                   ((16, 16, 16), (R, R, P, P, O, O))])
def test_mode_decays_as_backward_euler(n, bc):
    # Eddington, uniform rho: one implicit step divides a mode by its eigenvalue
    g = grid(n, bc)
    cs = centres(g)
    shp = g.shape[1:]
    v = np.ones(shp)
    lam = 1.0
    dt = 4e-12
    D = C_LIGHT / (3.0 * KAPPA * 1.5)
    for d, (m, c) in enumerate(zip(g.n, cs)):
        k = d + 1
        if bc[2 * d] == P:
            v = v * np.cos(2 * np.pi * k * c)
            s = np.sin(np.pi * k / m)
        else:
            v = v * np.cos(np.pi * k * c)  # c = (i + 1/2)/m on the unit interval
            s = np.sin(np.pi * k / (2 * m))
        lam += 4.0 * dt * D * m * m * s * s
    E0 = 10.0 + v
    X, st, res = fld.rad_diffuse(g, state(g, 1.5, E0), dt, ncycles=24, limiter=fld.EDDINGTON)
    assert st == 0
    np.testing.assert_allclose(X[-1], 10.0 + v / lam, rtol=0, atol=1e-11)


@pytest.mark.parametrize("n", [16, 32, 64, 128])
def test_contraction_is_mesh_independent(n):
    # a smooth coefficient (Eddington limiter, smooth rho): V(2,2) cycles with
    # red-black relaxation and linear interpolation contract the residual by
    # about 0.06 per cycle whatever the grid (the textbook multigrid rate)
    g = grid((n, n), (P, P, O, O))
    U = random_state(g, 5)
    x, y = centres(g)
    U[0] = 1.0 + 0.5 * np.sin(2 * np.pi * x) * np.cos(np.pi * y)
    X, st, res = fld.rad_diffuse(g, U, 1e-10, ncycles=8, limiter=fld.EDDINGTON)
    rate = (res[-1] / res[2]) ** (1 / 6)
    assert rate < 0.1, rate


def test_rough_coefficients_still_converge():
    # Levermore on random E makes D jump from cell to cell; the cycles slow
    # down (rediscretised coarse operators) but keep converging
    g = grid((64, 64), (P, P, O, O))
    X, st, res = fld.rad_diffuse(g, random_state(g, 5), 1e-10, ncycles=8)
    assert np.all(res[1:] / res[:-1] < 0.35), res[1:] / res[:-1]


@pytest.mark.parametrize("bc", [(P, P, P, P), (O, O, R, R)])
def test_converged_step_conserves_and_is_bounded(bc):
    g = grid((32, 16), bc)
    U = random_state(g, 6)
    X, st, res = fld.rad_diffuse(g, U, 1e-9, ncycles=25)
    E0, E1 = U[-1], X[-1]
    assert abs(E1.sum() - E0.sum()) <= 1e-12 * E0.sum()
    assert E1.min() >= E0.min() - 1e-12 and E1.max() <= E0.max() + 1e-12
    assert E1.std() < E0.std()


def test_zero_dt_leaves_E_unchanged():
    g = grid((16, 8, 4), (P, P, O, O, R, R))
    U = random_state(g, 7)
    X, st, res = fld.rad_diffuse(g, U, 0.0, ncycles=3)
    np.testing.assert_array_equal(X, U)
    assert np.all(res == 0.0)


def test_one_cell_coarsest_level_is_solved_exactly():
    # a power-of-two hierarchy ends in one cell where A = [1]: one sweep solves
    # it, so more coarsest-level sweeps change nothing; a hierarchy that ends
    # on a larger grid does depend on them
    g = grid((16, 8), (P, P, O, O))
    U = random_state(g, 8)
    a = fld.rad_diffuse(g, U, 1e-10, ncycles=2, ncoarse=1)[0]
    b = fld.rad_diffuse(g, U, 1e-10, ncycles=2, ncoarse=9)[0]
    np.testing.assert_array_equal(a, b)
    g = grid((24, 20), (P, P, O, O))
    U = random_state(g, 8)
    a = fld.rad_diffuse(g, U, 1e-10, ncycles=2, ncoarse=1)[0]
    b = fld.rad_diffuse(g, U, 1e-10, ncycles=2, ncoarse=9)[0]
    assert np.abs(a - b).max() > 1e-6


def test_zero_cycles_return_the_old_field_and_its_residual():
    g = grid((8, 8), (P, P, P, P))
    U = random_state(g, 9)
    X, st, res = fld.rad_diffuse(g, U, 1e-10, ncycles=0)
    np.testing.assert_array_equal(X, U)
    y, _ = fld.fld_apply(g, U, 1e-10, U[-1])
    assert res[0] == pytest.approx(np.linalg.norm(U[-1] - y), rel=1e-12)


def test_gaussian_pulse_converges_at_first_order_in_dt():
    # Eddington limit, uniform rho: the diffusion step solves the heat
    # equation d_t E = D d_xx E, whose Gaussian pulse spreads with variance
    # s0^2 + 2 D t; backward Euler approaches it at first order in dt
    n = 512
    g = grid((n,), (P, P), dx=(1.0 / n,))
    x = (np.arange(n) + 0.5) / n - 0.5
    D = C_LIGHT / (3.0 * KAPPA * 1.0)
    s0 = 0.03
    t_final = 0.5 * s0 ** 2 / D

    def exact(t):
        s2 = s0 ** 2 + 2.0 * D * t
        return 1.0 + np.sqrt(s0 ** 2 / s2) * np.exp(-x ** 2 / (2.0 * s2))

    errs = []
    for k in (4, 8, 16, 32):
        U = state(g, 1.0, exact(0.0))
        for _ in range(k):
            U, st, _ = fld.rad_diffuse(g, U, t_final / k, ncycles=30, limiter=fld.EDDINGTON)
            assert st == 0
        errs.append(np.abs(U[-1] - exact(t_final)).max())
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all((orders > 0.85) & (orders < 1.15)), orders
    assert errs[-1] < 3e-3
