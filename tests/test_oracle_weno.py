"""Pins of the oracle's second scheme, the paper's own choice (section
2.2.2): WENO5-Z face states on primitive variables with the HLL flux.

Each test names what fixes the expected value.  The paper prints one
accuracy figure for this scheme: the Sod tube at t = 0.0669 with dx = 2^-10
and Courant number 0.3 has a density L1 error below 5e-4 (caption of the Sod
density figure, section 3.1); here that bound is a gate.
"""
import json
import os

import numpy as np
import pytest

import oracle
import workloads
from oracle.exact_riemann import RiemannSolution
from oracle.metrics import exact_sum, fitted_order, l1_error

GOLD = os.path.join(os.path.dirname(__file__), "golden")
P, O, R = oracle.PERIODIC, oracle.OUTFLOW, oracle.REFLECT
W5 = oracle.WENO5Z_HLL


def gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


def total_energy(W, g=1.4):
    r, un, *ut, p = W
    q = un * un
    for v in ut:
        q = q + v * v
    return p / (g - 1) + 0.5 * r * q


def physical_flux(W, g=1.4):
    r, un, *ut, p = W
    E = total_energy(W, g)
    return np.array([r * un, r * un * un + p] + [r * un * v for v in ut] + [(E + p) * un])


def conserved(W, g=1.4):
    r, un, *ut, p = W
    return np.array([r, r * un] + [r * v for v in ut] + [total_energy(W, g)])


# --------------------------------------------------------------------------
# the paper's printed figure
# --------------------------------------------------------------------------
def test_sod_paper_figure_bound():
    """Sod at the paper's settings: L1(rho) below the paper's 5e-4."""
    s = gold("sod_paper.json")
    n = int(round(1.0 / s["dx"]))
    g = oracle.Grid((n,), bc=(O, O), scheme=W5)
    U, t, _, st = oracle.run(g, workloads.sod(n), s["courant"], s["t_final"])
    ex = RiemannSolution(1.0, 0.0, 1.0, 0.125, 0.0, 0.1)
    r, _, _ = ex.cell_averages(n, t)
    err = l1_error(U[0], r, s["dx"])
    print(f"WENO5-Z + HLL Sod L1(rho) = {err:.3e} (paper: < {s['paper_L1_rho_bound']})")
    assert st == 0 and t == pytest.approx(s["t_final"], rel=1e-14)
    assert err < s["paper_L1_rho_bound"]


# --------------------------------------------------------------------------
# WENO5-Z reconstruction
# --------------------------------------------------------------------------
def cell_averages_of_poly(coef, h, x0=0.0, m=5):
    """Exact averages over [x0 + j h, x0 + (j+1) h] of sum_k coef[k] x^k."""
    out = []
    for j in range(m):
        a, b = x0 + j * h, x0 + (j + 1) * h
        out.append(sum(c * (b ** (k + 1) - a ** (k + 1)) / ((k + 1) * h) for k, c in enumerate(coef)))
    return np.array(out)


def test_weno5z_exact_for_quadratics():
    """Every candidate stencil reproduces a quadratic exactly, so any convex
    weights do: the face value equals the polynomial at the face."""
    rng = np.random.default_rng(7)
    for _ in range(50):
        coef = rng.uniform(-2, 2, 3)
        h = rng.uniform(0.01, 0.5)
        x0 = rng.uniform(-1, 1)
        v = cell_averages_of_poly(coef, h, x0)
        xf = x0 + 3 * h
        exact = coef[0] + coef[1] * xf + coef[2] * xf * xf
        assert oracle.weno5z(v) == pytest.approx(exact, rel=1e-12, abs=1e-12)
        # the left face of the middle cell from the mirrored cells
        xl = x0 + 2 * h
        assert oracle.weno5z(v[::-1]) == pytest.approx(
            coef[0] + coef[1] * xl + coef[2] * xl * xl, rel=1e-12, abs=1e-12)


def test_weno5z_fifth_order_on_smooth_data():
    """On a smooth profile the Z weights tend to the optimal ones fast enough
    for the fifth-order linear reconstruction: error order >= 4.5."""
    ms = [20, 40, 80, 160]
    errs = []
    for m in ms:
        h = 1.0 / m
        j = np.arange(5)
        v = (np.cos(2 * np.pi * j * h) - np.cos(2 * np.pi * (j + 1) * h)) / (2 * np.pi * h)
        errs.append(abs(oracle.weno5z(v) - np.sin(2 * np.pi * 3 * h)))
    assert fitted_order(ms, errs) >= 4.5, errs


def test_weno5z_step_is_non_oscillatory():
    """Across a jump the stencil that contains it gets vanishing weight: the
    face value is the smooth side's constant (to 1e-12)."""
    for lo, hi in ((0.0, 1.0), (2.0, -3.0), (0.125, 1.0)):
        # jump right of the face: cells i-2..i on the low side
        assert abs(oracle.weno5z([lo, lo, lo, hi, hi]) - lo) <= 1e-12 * max(abs(lo), abs(hi))
        # jump left of the cell: cells i-1..i+2 on the high side
        assert abs(oracle.weno5z([lo, hi, hi, hi, hi]) - hi) <= 1e-12 * max(abs(lo), abs(hi))


def test_weno5z_indicators_match_their_integral_definition():
    """Each smoothness indicator is, by its definition (Jiang and Shu 1996, the
    indicators WENO5-Z uses), the integral over the middle cell of
    dx (p_k')^2 + dx^3 (p_k'')^2 for the quadratic p_k whose averages over the
    stencil's three cells are the data.  Here p_k comes from solving that
    3 x 3 system and the integral from Gauss-Legendre quadrature (exact for
    these polynomials), with dx = 1 and the middle cell on [-1/2, 1/2]; this
    fixes both closed-form coefficients (13/12 and 1/4)."""
    rng = np.random.default_rng(17)
    xg, wg = np.polynomial.legendre.leggauss(4)
    xg, wg = 0.5 * xg, 0.5 * wg  # nodes and weights on [-1/2, 1/2]
    for _ in range(40):
        v = rng.uniform(-2, 2, 5)
        beta = oracle.weno5z_indicators(v)
        for k in range(3):
            centres = np.arange(k, k + 3) - 2.0
            # average of 1, x, x^2 over [c - 1/2, c + 1/2]
            A = np.stack([np.ones(3), centres, centres ** 2 + 1.0 / 12.0], axis=1)
            a, b, c = np.linalg.solve(A, v[k:k + 3])
            d1 = b + 2.0 * c * xg
            d2 = 2.0 * c
            expect = np.sum(wg * (d1 * d1 + d2 * d2))
            assert beta[k] == pytest.approx(expect, rel=1e-12, abs=1e-13)


def test_weno5z_tends_to_the_linear_scheme_at_eighth_order():
    """On smooth data with f' != 0, a Taylor expansion gives beta_k = f'^2 dx^2
    + O(dx^3) for every k and tau5 = |beta_0 - beta_2| = O(dx^5), so with the
    ratio tau5/(beta_k + eps) taken to the first power the face value differs
    from the fifth-order linear reconstruction (2, -13, 47, 27, -3)/60 (the
    limit of the optimal weights d = (1, 6, 3)/10) by O(dx^8); the square of
    the ratio would give O(dx^11).  Fitted order over dx = 1/4 .. 1/32."""
    # f = sin(2.1 x + 0.4) + exp(0.7 x) through its antiderivative
    F = lambda x: -np.cos(2.1 * x + 0.4) / 2.1 + np.exp(0.7 * x) / 0.7
    hs = [2.0 ** -k for k in range(2, 6)]
    diffs = []
    for h in hs:
        x = 0.3 + (np.arange(6) - 3) * h
        v = (F(x[1:]) - F(x[:-1])) / h
        lin = (2 * v[0] - 13 * v[1] + 47 * v[2] + 27 * v[3] - 3 * v[4]) / 60
        diffs.append(abs(oracle.weno5z(v) - lin))
    order = fitted_order([1 / h for h in hs], diffs)
    assert 7.0 <= order <= 9.0, (order, diffs)


def test_weno5z_affine_equivariance():
    """Shifting and scaling the data by a > 0 shifts and scales the face value
    (the smoothness ratios are scale-free; eps = 1e-40 is negligible here)."""
    rng = np.random.default_rng(9)
    for _ in range(50):
        v = rng.uniform(-1, 1, 5)
        a, b = rng.uniform(0.1, 10), rng.uniform(-5, 5)
        assert oracle.weno5z(a * v + b) == pytest.approx(a * oracle.weno5z(v) + b, rel=1e-12,
                                                         abs=1e-12)


# --------------------------------------------------------------------------
# HLL flux
# --------------------------------------------------------------------------
def random_face_state(rng, nt):
    return np.concatenate([[rng.uniform(0.2, 2)], rng.uniform(-1, 1, 1 + nt), [rng.uniform(0.2, 2)]])


@pytest.mark.parametrize("nt", [0, 1, 2])
def test_hll_consistency(nt):
    rng = np.random.default_rng(11 + nt)
    for _ in range(50):
        W = random_face_state(rng, nt)
        assert np.allclose(oracle.hll(W, W), physical_flux(W), rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("nt", [0, 2])
def test_hll_supersonic_upwinding(nt):
    """S_L >= 0 gives the left physical flux exactly, S_R <= 0 the right one."""
    rng = np.random.default_rng(21 + nt)
    for _ in range(20):
        WL = random_face_state(rng, nt)
        WR = random_face_state(rng, nt)
        WL[1] = WR[1] = 5.0  # faster than every sound speed here
        assert np.array_equal(oracle.hll(WL, WR), physical_flux(WL))
        WL[1] = WR[1] = -5.0
        assert np.array_equal(oracle.hll(WL, WR), physical_flux(WR))


@pytest.mark.parametrize("nt", [0, 2])
def test_hll_intermediate_state_jump_conditions(nt):
    """The HLL flux is the flux of the single intermediate state
    U* = (S_R U_R - S_L U_L - (F_R - F_L)) / (S_R - S_L) of the two-wave fan: it
    satisfies the jump conditions F* = F_L + S_L (U* - U_L) = F_R + S_R (U* - U_R)."""
    rng = np.random.default_rng(31 + nt)
    g = 1.4
    for _ in range(50):
        WL = random_face_state(rng, nt)
        WR = random_face_state(rng, nt)
        WL[1] *= 0.3
        WR[1] *= 0.3  # subsonic: both waves straddle the face
        cL = np.sqrt(g * WL[-1] / WL[0])
        cR = np.sqrt(g * WR[-1] / WR[0])
        SL = min(WL[1] - cL, WR[1] - cR)
        SR = max(WL[1] + cL, WR[1] + cR)
        assert SL < 0 < SR
        UL, UR = conserved(WL), conserved(WR)
        FL, FR = physical_flux(WL), physical_flux(WR)
        Us = (SR * UR - SL * UL - (FR - FL)) / (SR - SL)
        F = oracle.hll(WL, WR)
        scale = np.abs(FL).max() + np.abs(FR).max()
        assert np.abs(F - (FL + SL * (Us - UL))).max() <= 1e-13 * scale
        assert np.abs(F - (FR + SR * (Us - UR))).max() <= 1e-13 * scale


# --------------------------------------------------------------------------
# the whole step
# --------------------------------------------------------------------------
@pytest.mark.parametrize("ndim", [1, 2, 3])
@pytest.mark.parametrize("bc", [P, O, R])
def test_uniform_state_preserved_bitwise(ndim, bc):
    n = (12, 10, 6)[:ndim]
    shape = tuple(reversed(n))
    vel = [0.0] * ndim if bc == R else [0.3, -0.2, 0.1][:ndim]
    U0 = workloads.conserved_from_primitive(np.full(shape, 0.7), [np.full(shape, v) for v in vel],
                                            np.full(shape, 0.4))
    g = oracle.Grid(n, bc=(bc, bc), scheme=W5)
    dt, _ = oracle.cfl_dt(g, U0, 0.4)
    U, st = oracle.steps(g, U0, [dt] * 3)
    assert st == 0
    assert np.array_equal(U, U0)


@pytest.mark.parametrize("ndim", [2, 3])
def test_conservation_periodic(ndim):
    n = 32 if ndim == 2 else 12
    U0 = workloads.turbulent_box(n, ndim=ndim, seed=22)
    g = oracle.Grid((n,) * ndim, bc=(P, P), scheme=W5)
    dt, _ = oracle.cfl_dt(g, U0, 0.4)
    U, st = oracle.steps(g, U0, [dt] * 6)
    assert st == 0 and not np.array_equal(U, U0)
    for v in range(g.nvar):
        rel = abs(exact_sum(U[v]) - exact_sum(U0[v])) / exact_sum(np.abs(U0[v]))
        assert rel <= 1e-12, (v, rel)


def reflect(U, axis_arr, ndim):
    d = ndim - 1 - axis_arr
    V = np.flip(U, axis=1 + axis_arr).copy()
    V[1 + d] = -V[1 + d]
    return V


@pytest.mark.parametrize("ndim,bc", [(1, O), (2, P), (2, R), (3, R)])
def test_mirror_symmetry(ndim, bc):
    n = {1: 40, 2: 20, 3: 10}[ndim]
    rng = np.random.default_rng(32)
    shape = (n,) * ndim
    U0 = workloads.conserved_from_primitive(rng.uniform(0.5, 1.5, shape),
                                            [rng.uniform(-0.3, 0.3, shape) for _ in range(ndim)],
                                            rng.uniform(0.5, 1.5, shape))
    g = oracle.Grid(shape, bc=(bc, bc), scheme=W5)
    dt, _ = oracle.cfl_dt(g, U0, 0.4)
    A, _ = oracle.steps(g, U0, [dt] * 2)
    for ax in range(ndim):
        B, _ = oracle.steps(g, reflect(U0, ax, ndim), [dt] * 2)
        RA = reflect(A, ax, ndim)
        for v in range(g.nvar):
            assert np.abs(B[v] - RA[v]).max() <= 1e-13 * np.abs(RA[v]).max() + 1e-300


@pytest.mark.parametrize("bc", [P, O, R])
def test_3d_with_1d_data_equals_1d_bitwise(bc):
    n = 48
    rL, pL, rR, pR = workloads.random_two_state_params(4)
    U1 = workloads.two_state(n, (rL, 0.1, pL), (rR, -0.2, pR))
    dts = [2e-4] * 4
    A, _ = oracle.steps(oracle.Grid((n,), bc=(bc, bc), scheme=W5), U1, dts)
    U3 = np.zeros((5, 3, 4, n))
    U3[0], U3[1], U3[4] = U1[0], U1[1], U1[2]
    B, _ = oracle.steps(oracle.Grid((n, 4, 3), bc=(bc, bc, P, P, R, R), scheme=W5), U3, dts)
    for k in range(3):
        for j in range(4):
            assert np.array_equal(B[0, k, j], A[0])
            assert np.array_equal(B[1, k, j], A[1])
            assert np.array_equal(B[4, k, j], A[2])
            assert not B[2, k, j].any() and not B[3, k, j].any()


def test_acoustic_wave_converges():
    """The paper's acoustic wave (section 3.5 closed form): with dt tied to dx
    by the CFL condition, Heun's second-order time error dominates the
    fifth-order space error, so the order is at least 1.8; WENO5-Z must also
    be more accurate than MUSCL-minmod at every resolution."""
    a = gold("acoustic_paper.json")
    errs, errs_m = [], []
    for n in a["ns"]:
        U0 = workloads.acoustic_state(n, a["amplitude"], a["gamma"])
        r_ex = None
        for scheme, sink in ((W5, errs), (oracle.MUSCL_HLLC, errs_m)):
            g = oracle.Grid((n,), gamma=a["gamma"], bc=(P, P), scheme=scheme)
            U, t, _, st = oracle.run(g, U0, a["courant"], a["t_final"])
            r_ex, _, _ = workloads.acoustic_1d(n, a["amplitude"], a["gamma"], t=t)
            sink.append(l1_error(U[0], r_ex, 1.0 / n))
    assert fitted_order(a["ns"], errs) >= a["min_order_L1_rho"], errs
    assert all(e < m for e, m in zip(errs, errs_m)), (errs, errs_m)


@pytest.mark.parametrize("seed", [0, 2, 6])
def test_two_state_converges_to_exact_solution(seed):
    """Random two-state problems (c0 recipe) at t = 0.2: the density L1 error
    against the exact Riemann solution falls with every refinement."""
    rL, pL, rR, pR = workloads.random_two_state_params(seed)
    ex = RiemannSolution(rL, 0.0, pL, rR, 0.0, pR)
    errs = []
    for n in (128, 256, 512):
        g = oracle.Grid((n,), bc=(O, O), scheme=W5)
        U, t, _, st = oracle.run(g, workloads.random_two_state(n, seed), 0.4, 0.2)
        assert st == 0
        r, _, _ = ex.cell_averages(n, t)
        errs.append(l1_error(U[0], r, 1.0 / n))
    assert errs[0] > errs[1] > errs[2], errs
