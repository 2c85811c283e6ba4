"""The oracle's pins catch plausible mistakes.

Each case below plants one typical mistake in a copy of the oracle's source
(a wrong sign, a dropped factor, an off-by-one ghost, a wrong comparison,
the wrong stage combine, ...), builds that copy on the CPU, and checks that
at least one of a set of quick pins fails for it, while every pin passes
for the unmodified oracle.  The pins used here are the same kinds of facts
as in test_oracle_pins.py (closed forms, exact special cases, invariants,
the exact Riemann solution), evaluated on small grids.
"""
import os
import tempfile

import numpy as np
import pytest

import oracle
import workloads
from oracle import build as obuild
from oracle.exact_riemann import RiemannSolution
from oracle.metrics import exact_sum, fitted_order, l1_error

P, O, R = oracle.PERIODIC, oracle.OUTFLOW, oracle.REFLECT


def physical_flux(W, g=1.4):
    r, un, *ut, p = W
    E = p / (g - 1) + 0.5 * r * (un * un + sum(v * v for v in ut))
    return np.array([r * un, r * un * un + p] + [r * un * v for v in ut] + [(E + p) * un])


def quick_pins():
    """Names of the quick pins that fail for the currently loaded oracle."""
    failed = []
    rng = np.random.default_rng(5)
    # HLLC consistency (flux of equal states is the physical flux)
    ok = True
    for nt in (0, 2):
        for _ in range(20):
            W = np.concatenate([[rng.uniform(0.2, 2)], rng.uniform(-1, 1, 1 + nt),
                                [rng.uniform(0.2, 2)]])
            if not np.allclose(oracle.hllc(W, W), physical_flux(W), rtol=1e-12, atol=1e-12):
                ok = False
    if not ok:
        failed.append("hllc_consistency")
    # minmod truth table
    mm = oracle.minmod
    if not (mm(1.0, 2.0) == 1.0 and mm(-3.0, -2.0) == -2.0 and mm(1.0, -1.0) == 0.0
            and mm(0.0, 1.0) == 0.0):
        failed.append("minmod")
    # stationary contact is an exact solution of the flux
    F = oracle.hllc([1.0, 0.0, 0.3, 0.7], [0.2, 0.0, 0.3, 0.7])
    if not (F[0] == 0.0 and F[1] == 0.7 and F[2] == 0.0 and F[3] == 0.0):
        failed.append("stationary_contact")
    # uniform states are preserved
    for bc, vel in ((P, [0.3, -0.2]), (R, [0.0, 0.0]), (O, [0.2, 0.1])):
        shape = (10, 12)
        U0 = workloads.conserved_from_primitive(np.full(shape, 0.7),
                                                [np.full(shape, v) for v in vel],
                                                np.full(shape, 0.4))
        g = oracle.Grid((12, 10), bc=(bc, bc))
        U, _ = oracle.steps(g, U0, [2e-3] * 2)
        if not np.array_equal(U, U0):
            failed.append(f"uniform_{bc}")
    # periodic conservation
    n = 24
    U0 = workloads.turbulent_box(n, ndim=2, seed=21)
    g = oracle.Grid((n, n), bc=(P, P))
    U, _ = oracle.steps(g, U0, [2e-3] * 4)
    for v in range(4):
        if abs(exact_sum(U[v]) - exact_sum(U0[v])) > 1e-12 * exact_sum(np.abs(U0[v])):
            failed.append("conservation")
            break
    # reflecting walls conserve mass and energy (a moving state in a closed box)
    x = workloads.cell_centres(48)
    U0 = workloads.conserved_from_primitive(1.0 + 0.3 * np.sin(2 * np.pi * x),
                                            [0.3 + 0.1 * np.cos(2 * np.pi * x)],
                                            0.8 + 0.2 * x)
    U, _ = oracle.steps(oracle.Grid((48,), bc=(R, R)), U0, [2e-3] * 10)
    for v in (0, 2):
        if abs(exact_sum(U[v]) - exact_sum(U0[v])) > 1e-12 * exact_sum(np.abs(U0[v])):
            failed.append("wall_conservation")
            break
    # mirror symmetry with reflecting walls (x mirror: flip array axis 1, negate m_x)
    shape = (16, 16)
    U0 = workloads.conserved_from_primitive(rng.uniform(0.5, 1.5, shape),
                                            [rng.uniform(-0.3, 0.3, shape) for _ in range(2)],
                                            rng.uniform(0.5, 1.5, shape))
    g = oracle.Grid((16, 16), bc=(R, R))
    A, _ = oracle.steps(g, U0, [1e-3] * 2)
    M = np.flip(U0, axis=2).copy()
    M[1] = -M[1]
    B, _ = oracle.steps(g, M, [1e-3] * 2)
    RA = np.flip(A, axis=2).copy()
    RA[1] = -RA[1]
    if not np.allclose(B, RA, rtol=0, atol=1e-13 * np.abs(RA).max()):
        failed.append("mirror")
    # exact Riemann solution (seed 0, n = 256)
    rL, pL, rR, pR = workloads.random_two_state_params(0)
    ex = RiemannSolution(rL, 0.0, pL, rR, 0.0, pR)
    Ur, t, _, st = oracle.run(oracle.Grid((256,), bc=(O, O)), workloads.random_two_state(256, 0),
                              0.4, 0.2)
    r_ex, _, _ = ex.cell_averages(256, t)
    if not (np.isfinite(Ur).all() and l1_error(Ur[0], r_ex, 1 / 256) < 4e-3):
        failed.append("riemann")
    # acoustic wave: second order
    errs = []
    for nn in (64, 128, 256):
        Ua, t, _, _ = oracle.run(oracle.Grid((nn,), bc=(P, P)), workloads.acoustic_state(nn), 0.4,
                                 1.0)
        r_ex, _, _ = workloads.acoustic_1d(nn, t=t)
        errs.append(l1_error(Ua[0], r_ex, 1 / nn))
    if not (np.all(np.isfinite(errs)) and fitted_order([64, 128, 256], errs) >= 1.7):
        failed.append("acoustic_order")
    # CFL closed form on a uniform 3D state
    shape = (4, 6, 8)
    vel = [0.3, -0.2, 0.1]
    U0 = workloads.conserved_from_primitive(np.full(shape, 0.7), [np.full(shape, v) for v in vel],
                                            np.full(shape, 0.4))
    dt, _ = oracle.cfl_dt(oracle.Grid((8, 6, 4), bc=(P, P)), U0, 0.4)
    c = np.sqrt(1.4 * 0.4 / 0.7)
    if abs(dt - 0.4 / sum((abs(v) + c) * m for v, m in zip(vel, (8, 6, 4)))) > 1e-15 * dt:
        failed.append("cfl")
    return failed


MUTATIONS = {
    "minmod picks the larger slope": ("if (fabs(a) <= fabs(b)) return a;",
                                      "if (fabs(a) >= fabs(b)) return a;"),
    "left wave speed uses max": ("T SL = aL <= bL ? aL : bL;", "T SL = aL >= bL ? aL : bL;"),
    "contact speed sign": ("- R.rho * R.un * (SR - R.un);", "+ R.rho * R.un * (SR - R.un);"),
    "star energy sign": ("(Ss - W.un) * (W.rho * Ss", "(Ss + W.un) * (W.rho * Ss"),
    "kinetic energy factor dropped": ("T ke = T(0.5) * q / rho;", "T ke = q / rho;"),
    "wall does not flip momentum": ("if (flip && v == 1 + d) val = -val;",
                                    "if (flip && v == 1 + d) val = val;"),
    "periodic ghost off by one": ("if (bc_lo == BC_PERIODIC) return n - k;",
                                  "if (bc_lo == BC_PERIODIC) return n - 1;"),
    "Heun combine uses U1 twice": ("U[x] = T(0.5) * (U[x] + (U1[x] + dt * L[x]));",
                                   "U[x] = T(0.5) * (U1[x] + (U1[x] + dt * L[x]));"),
    "flux difference sign": ("- (Fp - Fm) / T(g.dx[d]);", "- (Fm - Fp) / T(g.dx[d]);"),
    "CFL takes the max over axes": ("s = s + (fabs(w[1 + d]) + cs) / T(g.dx[d]);",
                                    "s = std::max(s, (fabs(w[1 + d]) + cs) / T(g.dx[d]));"),
    "transverse momentum flux": ("FK[2 + t] = mn * W.ut[t];", "FK[2 + t] = W.rho * W.ut[t];"),
    "slope dropped (first order)": ("WL[v] = Wc[1][v] + T(0.5) * sl;",
                                    "WL[v] = Wc[1][v] + T(0.0) * sl;"),
}


@pytest.fixture(scope="module")
def restore_oracle():
    yield
    oracle.use_library(obuild.LIB)


def test_unmodified_oracle_passes_quick_pins(restore_oracle):
    oracle.use_library(obuild.LIB)
    assert quick_pins() == []


@pytest.mark.parametrize("name", list(MUTATIONS))
def test_planted_mistake_is_caught(name, restore_oracle, tmp_path):
    old, new = MUTATIONS[name]
    src = open(obuild.SRC[0]).read()
    # the first occurrence is the MUSCL-HLLC path the quick pins run (the
    # HLL flux of the second scheme repeats the wave-speed lines)
    assert src.count(old) >= 1, f"mutation site missing: {old}"
    mutated = tmp_path / "hydro_oracle_mutant.cpp"
    mutated.write_text(src.replace(old, new, 1))
    lib = obuild.build(src=str(mutated), out=str(tmp_path / "liboracle_mutant.so"))
    oracle.use_library(lib)
    try:
        with np.errstate(all="ignore"):
            failed = quick_pins()
    finally:
        oracle.use_library(obuild.LIB)
    assert failed, f"no pin caught: {name}"
