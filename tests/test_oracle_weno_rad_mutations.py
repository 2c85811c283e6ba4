"""The pins of the oracle's second scheme (WENO5-Z + HLL) and of its
radiation energy field catch plausible mistakes.

As in test_oracle_mutations.py, each case plants one typical mistake in a
copy of hydro_oracle.cpp (the exponent of the WENO-Z weight ratio, the order
of the optimal weights, a coefficient of the smoothness indicators or of a
candidate stencil, the global smoothness measure, the regulariser, the
mirrored right face state, the HLL dissipation, the Rusanov signal speed and
dissipation, the advective part of the Rusanov flux), builds that copy on the
CPU and checks that at least one of the pins in test_oracle_weno.py and
test_oracle_rad.py fails for it, while all of them pass for the unmodified
oracle.
"""
import numpy as np
import pytest

import oracle
from oracle import build as obuild

import test_oracle_rad as TR
import test_oracle_weno as TW

PINS = {
    "sod_bound": TW.test_sod_paper_figure_bound,
    "quadratics": TW.test_weno5z_exact_for_quadratics,
    "fifth_order": TW.test_weno5z_fifth_order_on_smooth_data,
    "indicators": TW.test_weno5z_indicators_match_their_integral_definition,
    "linear_limit_order": TW.test_weno5z_tends_to_the_linear_scheme_at_eighth_order,
    "non_oscillatory": TW.test_weno5z_step_is_non_oscillatory,
    "hll_jump_conditions": lambda: [TW.test_hll_intermediate_state_jump_conditions(nt)
                                    for nt in (0, 2)],
    "weno_mirror": lambda: TW.test_mirror_symmetry(2, oracle.REFLECT),
    "rusanov_contact": TR.test_rusanov_jump_on_a_stationary_contact,
    "rusanov_velocity_jump": TR.test_rusanov_flux_at_a_velocity_jump,
    "rusanov_equal_states": TR.test_rusanov_flux_of_equal_states_is_the_physical_flux,
}


def failing_pins():
    failed = []
    for name, fn in PINS.items():
        try:
            with np.errstate(all="ignore"):
                fn()
        except AssertionError:
            failed.append(name)
    return failed


MUTATIONS = {
    "WENO-Z weight ratio squared": [
        ("T(1.0) + tau / (b%d + eps))" % k,
         "T(1.0) + (tau / (b%d + eps)) * (tau / (b%d + eps)))" % (k, k)) for k in range(3)],
    "optimal weights in reverse order": [
        ("T a0 = T(0.1) * (", "T a0 = T(0.3) * ("), ("T a2 = T(0.3) * (", "T a2 = T(0.1) * (")],
    "indicator coefficient 13/12": [("c1(13.0 / 12.0)", "c1(1.0)")],
    "indicator coefficient 1/4": [("c2(0.25)", "c2(0.5)")],
    "candidate stencil coefficient": [("(-v[1] + T(5.0) * v[2] + T(2.0) * v[3])",
                                       "(-v[1] + T(4.0) * v[2] + T(3.0) * v[3])")],
    "global smoothness from beta_1": [("T tau = fabs(b0 - b2);", "T tau = fabs(b0 - b1);")],
    "regulariser 1e-6": [("eps(1e-40)", "eps(1e-6)")],
    "weights not normalised by their sum": [("/ (a0 + a1 + a2);", "/ (a0 + a1);")],
    "right face state not mirrored": [
        ("T b[5] = {Wst[5][v], Wst[4][v], Wst[3][v], Wst[2][v], Wst[1][v]};",
         "T b[5] = {Wst[1][v], Wst[2][v], Wst[3][v], Wst[4][v], Wst[5][v]};")],
    "HLL dissipation sign": [("SL * SR * (UR[v] - UL[v])", "SL * SR * (UL[v] - UR[v])")],
    "Rusanov speed is the smaller one": [("T s = sL >= sR ? sL : sR;", "T s = sL <= sR ? sL : sR;")],
    "Rusanov dissipation halved": [("- T(0.5) * s * (ER - EL);", "- T(0.25) * s * (ER - EL);")],
    "Rusanov speed without |u|": [("T sL = fabs(L.un) + cL, sR = fabs(R.un) + cR;",
                                   "T sL = L.un + cL, sR = R.un + cR;")],
    "Rusanov advection with one velocity": [("(EL * L.un + ER * R.un)", "(EL * L.un + ER * L.un)")],
}


@pytest.fixture(scope="module")
def restore_oracle():
    yield
    oracle.use_library(obuild.LIB)


def test_unmodified_oracle_passes_the_pins(restore_oracle):
    oracle.use_library(obuild.LIB)
    assert failing_pins() == []


@pytest.mark.parametrize("name", list(MUTATIONS))
def test_planted_mistake_is_caught(name, restore_oracle, tmp_path):
    src = open(obuild.SRC[0]).read()
    for old, new in MUTATIONS[name]:
        assert src.count(old) == 1, f"mutation site not unique: {old}"
        src = src.replace(old, new)
    mutated = tmp_path / "hydro_oracle_mutant.cpp"
    mutated.write_text(src)
    lib = obuild.build(src=str(mutated), out=str(tmp_path / "liboracle_mutant.so"))
    oracle.use_library(lib)
    try:
        failed = failing_pins()
    finally:
        oracle.use_library(obuild.LIB)
    assert failed, f"no pin caught: {name}"
    print(f"{name}: caught by {failed}")
