"""The oracle's operation count (the algorithmic operations per zone-update
reported beside the byte roofline).

The counting scalar must see every operation of the step: the square roots
are an exact check, because the method takes exactly two per face (the sound
speeds of the two face states) in each of the two stages, plus one per cell
for the CFL step, whatever the data.  Counting must not change the values.
"""
import numpy as np

import oracle
import workloads

P = oracle.PERIODIC


def test_sqrt_count_is_exact_and_counting_is_pure():
    for ndim, n in ((1, 40), (2, 12), (3, 8)):
        U = workloads.turbulent_box(n, ndim=ndim, seed=3) if ndim > 1 else \
            workloads.acoustic_state(n)
        g = oracle.Grid((n,) * ndim, bc=(P, P))
        before = U.copy()
        c = oracle.count_ops(g, U, 1e-3)
        faces = ndim * (n + 1) * n ** (ndim - 1)
        assert c["sqrt"] == 2 * 2 * faces + n ** ndim
        assert np.array_equal(U, before)
        assert all(v > 0 for v in c.values())


def test_ops_per_zone_update_3d():
    r = oracle.ops_per_zone_update(3, lambda n: workloads.turbulent_box(n, ndim=3, seed=2), 16, 32)
    # two stages x three faces x two sound speeds + one for the CFL step
    assert r["sqrt"] == 13.0
    assert 900 < sum(r.values()) < 1500


def test_bench_reports_the_oracle_count():
    """bench.py quotes the count beside its VALU figures; it must be the oracle's."""
    import os
    import sys
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import bench
    r = oracle.ops_per_zone_update(3, lambda n: workloads.turbulent_box(n, ndim=3, seed=2), 16, 32)
    assert bench.OPS_PER_ZU_3D == round(sum(r.values()))
