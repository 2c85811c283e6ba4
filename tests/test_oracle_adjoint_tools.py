"""The oracle's multi-direction dual numbers and branch signature (used by
the GPU adjoint tests), checked on the CPU.

* K directions at once give the same derivatives as K one-direction runs,
  bit for bit (the same operations per component).
* Away from kinks the dual derivative is the derivative: on single-entry
  samples whose branch signature does not change under +-h, the central
  difference of the oracle's own map converges to it at second order.
* The signature is a function of the branches only: the same input gives
  the same hash, a uniform state keeps its hash under a small uniform
  change of its values, and a change that flips a minmod choice changes it.
"""
import numpy as np
import pytest

import oracle
import workloads

P, O, R = 0, 1, 2


def smooth_2d(n, seed):
    rng = np.random.default_rng(seed)
    gf = lambda: workloads.gaussian_random_field((n, n), rng, spectral_index=-3.0)
    vel = [0.3 * gf() for _ in range(2)]
    return workloads.conserved_from_primitive(np.exp(0.2 * gf()), vel, 1.0 + 0.2 * gf())


def test_multi_direction_dual_equals_single_direction_runs():
    n = 24
    U0 = smooth_2d(n, 1)
    og = oracle.Grid((n, n), bc=(P, P, R, O))
    dt, _ = oracle.cfl_dt(og, U0, 0.4)
    rng = np.random.default_rng(2)
    for K in (2, 4, 8):
        V = [rng.standard_normal(U0.shape) for _ in range(K)]
        X, D, st = oracle.steps_tangent_multi(og, U0, V, [dt] * 5)
        assert st == 0
        for k in range(K):
            Xs, Ds, _ = oracle.steps_tangent(og, U0, V[k], [dt] * 5)
            assert np.array_equal(X, Xs) and np.array_equal(D[k], Ds)
    with pytest.raises(ValueError):
        oracle.steps_tangent_multi(og, U0, V[:3], [dt])


def test_dual_derivative_is_second_order_limit_of_central_differences():
    n, nsteps = 32, 10
    U0 = smooth_2d(n, 3)
    og = oracle.Grid((n, n), bc=(P, P, P, P))
    _, _, _, _, dts = oracle.run(og, U0, 0.4, 1e9, max_steps=nsteps, record_dts=True)
    s0 = oracle.branch_signature(og, U0, dts)
    rng = np.random.default_rng(5)
    h1, h2 = 1e-4, 2.5e-5
    second_order = 0
    for _ in range(40):
        f, i, j = int(rng.integers(0, 4)), int(rng.integers(0, n)), int(rng.integers(0, n))
        v = np.zeros_like(U0)
        v[f, i, j] = np.abs(U0[f]).mean()
        if any(oracle.branch_signature(og, U0 + sg * h * v, dts) != s0
               for h in (h1, h2) for sg in (1.0, -1.0)):
            continue
        _, D, _ = oracle.steps_tangent(og, U0, v, dts)
        nrm = np.abs(D).max()
        r = []
        for h in (h1, h2):
            Xp, _ = oracle.steps(og, U0 + h * v, dts)
            Xm, _ = oracle.steps(og, U0 - h * v, dts)
            r.append(np.abs((Xp - Xm) / (2.0 * h) - D).max() / nrm)
        # rounding of the state differences: a few ulp of the largest value
        floor = [8.0 * np.finfo(np.float64).eps * np.abs(U0).max() / (h * nrm) for h in (h1, h2)]
        assert r[1] <= r[0] / 8.0 + floor[1], (r, floor)
        second_order += r[0] > 10.0 * floor[0] and r[0] / r[1] > 12.0
    assert second_order >= 2


def test_branch_signature_tracks_branches_only():
    n = 16
    og = oracle.Grid((n, n), bc=(P, P, P, P))
    shape = (n, n)
    U = workloads.conserved_from_primitive(np.full(shape, 0.8), [np.full(shape, 0.1),
                                                                 np.full(shape, -0.2)],
                                           np.full(shape, 0.6))
    dts = [1e-3] * 3
    s = oracle.branch_signature(og, U, dts)
    assert s == oracle.branch_signature(og, U, dts)
    assert s == oracle.branch_signature(og, U * (1.0 + 1e-9), dts)
    # a density bump: its top is a minmod extremum; moving one neighbour
    # above the bump flips the choices around it
    B = U.copy()
    B[0, 8, 8] *= 1.1
    sb = oracle.branch_signature(og, B, dts)
    assert sb != s
    C = B.copy()
    C[0, 8, 9] = B[0, 8, 8] * 1.05
    assert oracle.branch_signature(og, C, dts) != sb
