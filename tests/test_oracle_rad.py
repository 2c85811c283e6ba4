"""Pins of the oracle's radiation energy field (the paper's fourth conserved
field, section 2.2.1): advection with the fluid velocity through the
Rusanov flux, and the heating/cooling exchange qdot = c kappa rho (E - a T^4)
integrated by backward Euler after each step.

What fixes the expected values: the paper's heating and cooling test
(section 3.2; its reference solution is the ODE of the heating rate,
integrated here by scipy's Radau method at tight tolerance), the closed-form
equilibrium C_v T + a T^4 = e + E, exact energy conservation of the
exchange, and, with kappa = 0, passive advection (hydro untouched bitwise,
conservation, the exact translated profile).
"""
import json
import os

import numpy as np
import pytest
from scipy.integrate import solve_ivp

import oracle
import workloads
from oracle.metrics import exact_sum, fitted_order, l1_error

GOLD = os.path.join(os.path.dirname(__file__), "golden")
P, O, R = oracle.PERIODIC, oracle.OUTFLOW, oracle.REFLECT
# CGS constants (CODATA 2018), written out here independently of the oracle
C_LIGHT = 2.99792458e10
A_RAD = 4.0 * 5.670374419e-5 / C_LIGHT
K_B = 1.380649e-16
M_U = 1.66053906660e-24


def gold():
    with open(os.path.join(GOLD, "heating_cooling_paper.json")) as f:
        return json.load(f)


def uniform_rad_state(n, rho, e, Er):
    U = np.zeros((4, n))
    U[0], U[2], U[3] = rho, e, Er
    return U


def run_exchange(s, T_fluid, t_end, dt, n=4):
    Cv = s["rho"] * K_B / (s["mu"] * M_U * (s["gamma"] - 1.0))
    e0, E0 = Cv * T_fluid, A_RAD * s["T_rad"] ** 4
    g = oracle.Grid((n,), gamma=s["gamma"], bc=(P, P), dx=(1.0,), rad=(s["kappa"], s["mu"]))
    U, st = oracle.steps(g, uniform_rad_state(n, s["rho"], e0, E0), [dt] * int(round(t_end / dt)))
    assert st == 0
    return U, Cv, e0, E0


def ode_reference(s, T_fluid, t_end):
    Cv = s["rho"] * K_B / (s["mu"] * M_U * (s["gamma"] - 1.0))
    q = C_LIGHT * s["kappa"] * s["rho"]

    def rhs(t, y):
        r = q * (y[1] - A_RAD * (y[0] / Cv) ** 4)
        return [r, -r]

    y0 = [Cv * T_fluid, A_RAD * s["T_rad"] ** 4]
    sol = solve_ivp(rhs, (0.0, t_end), y0, method="Radau", rtol=1e-12,
                    atol=[1e-9 * y0[1], 1e-9 * y0[1]])
    return sol.y[0, -1] / Cv


@pytest.mark.parametrize("case", ["heating", "cooling"])
def test_heating_cooling_converges_to_the_ode(case):
    """The paper's test: the fluid temperature at the end time converges to the
    ODE solution at first order in dt (backward Euler), and the fluid and
    radiation energies add up to their initial sum."""
    s = gold()
    T0 = s[f"T_fluid_{case}"]
    t_end = s[f"t_end_{case}"]
    ref = ode_reference(s, T0, t_end)
    errs = []
    dts = [4e-10, 2e-10, 1e-10]
    for dt in dts:
        U, Cv, e0, E0 = run_exchange(s, T0, t_end, dt)
        T = U[2, 0] / Cv
        errs.append(abs(T - ref) / ref)
        assert np.all(U == U[:, :1])  # the cells stay identical (uniform state, no flow)
        assert abs((U[2, 0] + U[3, 0]) - (e0 + E0)) <= 1e-15 * (e0 + E0)
    ratios = [errs[i] / errs[i + 1] for i in range(2)]
    assert all(1.8 <= r <= 2.2 for r in ratios), (errs, ratios)
    assert errs[-1] < 3e-3, errs


def test_equilibrium_is_the_closed_form_root():
    """Long enough, the exchange settles on C_v T + a T^4 = e0 + E0 with
    E = a T^4 (the fixed point of backward Euler is the equilibrium)."""
    s = gold()
    T0 = s["T_fluid_cooling"]
    U, Cv, e0, E0 = run_exchange(s, T0, 2e-6, 2e-8)
    W = e0 + E0
    roots = np.roots([A_RAD, 0.0, 0.0, Cv, -W])
    T_eq = max(r.real for r in roots if abs(r.imag) < 1e-6 * abs(r) and r.real > 0)
    T = U[2, 0] / Cv
    assert abs(T - T_eq) <= 1e-10 * T_eq, (T, T_eq)
    assert abs(U[3, 0] - A_RAD * T ** 4) <= 1e-9 * U[3, 0]


def test_kappa_zero_is_passive_advection():
    """kappa = 0: the radiation field does not touch the hydro fields (bitwise
    equal to the run without it), its total is conserved on a periodic grid,
    and a uniform E in any flow stays uniform."""
    n = 32
    U0 = workloads.turbulent_box(n, ndim=2, seed=23)
    g0 = oracle.Grid((n, n), bc=(P, P))
    g1 = oracle.Grid((n, n), bc=(P, P), rad=(0.0, 0.6))
    dt, _ = oracle.cfl_dt(g0, U0, 0.4)
    x = workloads.cell_centres(n)
    Er = 1.0 + 0.5 * np.sin(2 * np.pi * x)[None, :] * np.cos(2 * np.pi * x)[:, None]
    A, _ = oracle.steps(g0, U0, [dt] * 5)
    B, st = oracle.steps(g1, np.concatenate([U0, Er[None]]), [dt] * 5)
    assert st == 0
    assert np.array_equal(B[:4], A)
    assert abs(exact_sum(B[4]) - exact_sum(Er)) <= 1e-13 * exact_sum(np.abs(Er))
    # d_t E + div(E u) = 0 compresses a uniform E where div u != 0, so a
    # uniform E stays uniform only in a divergence-free flow; the discrete
    # turbulent field is not exactly one, a uniform flow is
    Uu = workloads.conserved_from_primitive(np.full((n, n), 1.0), [np.full((n, n), 0.3),
                                            np.full((n, n), -0.2)], np.full((n, n), 1.0))
    D, _ = oracle.steps(g1, np.concatenate([Uu, np.full((1, n, n), 0.7)]), [dt] * 5)
    assert np.array_equal(D[4], np.full((n, n), 0.7))


def test_advection_of_a_smooth_profile_converges():
    """E carried by a uniform flow u = 1 around a periodic box once: the L1
    error against the exact (unchanged) profile falls at order >= 1.5."""
    errs = []
    ns = [64, 128, 256]
    for n in ns:
        x = workloads.cell_centres(n)
        U = workloads.conserved_from_primitive(np.ones(n), [np.ones(n)], np.ones(n))
        Er = 1.0 + 0.3 * np.sin(2 * np.pi * x)
        g = oracle.Grid((n,), bc=(P, P), rad=(0.0, 0.6))
        dt = 0.4 / ((1.0 + np.sqrt(1.4)) * n)
        nst = int(np.ceil(1.0 / dt))
        out, st = oracle.steps(g, np.concatenate([U, Er[None]]), [1.0 / nst] * nst)
        assert st == 0
        errs.append(l1_error(out[3], Er, 1.0 / n))
    assert fitted_order(ns, errs) >= 1.5, errs


def test_rusanov_flux_of_equal_states_is_the_physical_flux():
    """With equal states on both sides the Rusanov flux is E u exactly: a
    uniform E in a uniform flow is preserved bitwise under every BC
    (reflecting walls need u = 0)."""
    for bc, u in ((P, 0.4), (O, -0.3), (R, 0.0)):
        n = 16
        U = workloads.conserved_from_primitive(np.full(n, 0.9), [np.full(n, u)], np.full(n, 1.2))
        g = oracle.Grid((n,), bc=(bc, bc), rad=(0.0, 0.6))
        X = np.concatenate([U, np.full((1, n), 2.5)])
        out, _ = oracle.steps(g, X, [1e-3] * 4)
        assert np.array_equal(out, X)


def jump_state(n, rho, u, p, Er, gamma=1.4):
    """1D state with rho, u, p and E_r each constant on the two halves
    (cells 0 .. n/2-1 and n/2 .. n-1), as (rho, m, E, E_r)."""
    half = lambda a, b: np.where(np.arange(n) < n // 2, a, b)
    r, vel, pr = half(*rho), half(*u), half(*p)
    U = workloads.conserved_from_primitive(r, [vel], pr, gamma)
    return np.concatenate([U, half(*Er)[None]])


def test_rusanov_jump_on_a_stationary_contact():
    """Fluid at rest at uniform pressure with a density jump (a stationary
    contact, so every hydro flux difference vanishes) and an E_r jump at the
    same face.  Every field is piecewise constant, so each minmod slope is 0
    and the face states are the cell values.  Only the jump face carries an
    E_r flux, pure dissipation: F = -s (E_R - E_L)/2 with the larger signal
    speed s = max(c_L, c_R), c = sqrt(gamma p/rho).  L(E_r) is -F/dx in the
    cell left of the face, +F/dx right of it, and 0 elsewhere."""
    n, g = 16, 1.4
    rho, p, Er = (1.0, 0.25), 0.7, (2.0, 0.5)
    X = jump_state(n, rho, (0.0, 0.0), (p, p), Er, g)
    grid = oracle.Grid((n,), gamma=g, bc=(O, O), rad=(0.0, 0.6))
    L, st = oracle.rhs(grid, X)
    assert st == 0
    assert np.all(L[:3] == 0.0)
    # pressure as the oracle recovers it from E (identical on both sides)
    pr = (g - 1.0) * X[2, 0]
    s = max(np.sqrt(g * pr / rho[0]), np.sqrt(g * pr / rho[1]))
    F = -0.5 * s * (Er[1] - Er[0])
    expect = np.zeros(n)
    expect[n // 2 - 1] = -F * n
    expect[n // 2] = F * n
    assert np.allclose(L[3], expect, rtol=1e-14, atol=0.0), (L[3], expect)


def test_rusanov_flux_at_a_velocity_jump():
    """Uniform rho and p, the velocity and E_r jumping at the same face (the
    right side moving left, faster): the slopes are 0, so the jump face sees
    the cell values and its E_r flux is the mean of the two advective fluxes,
    (E_L u_L + E_R u_R)/2, minus the dissipation s (E_R - E_L)/2 with
    s = max(|u_L| + c, |u_R| + c).  Every other face carries E u of its
    (equal) neighbours, so L(E_r) is -(F - E_L u_L)/dx and -(E_R u_R - F)/dx
    in the two cells at the jump and 0 elsewhere."""
    n, g = 16, 1.4
    rho, p, u, Er = 0.5, 0.625, (0.25, -0.75), (1.5, 0.4)
    X = jump_state(n, (rho, rho), u, (p, p), Er, g)
    grid = oracle.Grid((n,), gamma=g, bc=(O, O), rad=(0.0, 0.6))
    L, st = oracle.rhs(grid, X)
    assert st == 0
    vel = X[1] / X[0]
    pr = (g - 1.0) * (X[2] - 0.5 * X[1] * X[1] / X[0])
    c = np.sqrt(g * pr / X[0])
    uL, uR, cL, cR = vel[0], vel[-1], c[0], c[-1]
    s = max(abs(uL) + cL, abs(uR) + cR)
    F = 0.5 * (Er[0] * uL + Er[1] * uR) - 0.5 * s * (Er[1] - Er[0])
    expect = np.zeros(n)
    expect[n // 2 - 1] = -(F - Er[0] * uL) * n
    expect[n // 2] = -(Er[1] * uR - F) * n
    assert np.allclose(L[3], expect, rtol=1e-13, atol=1e-13 * np.abs(expect).max())


@pytest.mark.parametrize("bc", [P, R])
def test_mirror_symmetry_with_radiation(bc):
    n = 20
    rng = np.random.default_rng(33)
    shape = (n, n)
    U0 = workloads.conserved_from_primitive(rng.uniform(0.5, 1.5, shape),
                                            [rng.uniform(-0.3, 0.3, shape) for _ in range(2)],
                                            rng.uniform(0.5, 1.5, shape))
    X = np.concatenate([U0, rng.uniform(0.5, 1.5, (1,) + shape)])
    g = oracle.Grid(shape, bc=(bc, bc), rad=(1e-8, 0.6))
    dt, _ = oracle.cfl_dt(g, X, 0.4)
    A, _ = oracle.steps(g, X, [dt] * 2)
    M = np.flip(X, axis=2).copy()
    M[1] = -M[1]
    B, _ = oracle.steps(g, M, [dt] * 2)
    RA = np.flip(A, axis=2).copy()
    RA[1] = -RA[1]
    for v in range(5):
        assert np.abs(B[v] - RA[v]).max() <= 1e-13 * np.abs(RA[v]).max()
