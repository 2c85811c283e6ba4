"""Input generators: the stated recipe holds (these are inputs, not results)."""
import numpy as np

import workloads


def test_blast_hot_cells_and_energy():
    """32 cell centres lie within 2 dx of the corner point at the box centre,
    and the deposited energy sums to E0."""
    for n in (16, 64):
        hot = workloads.blast_hot_mask(n)
        assert hot.sum() == 32
        U = workloads.blast_3d(n)
        dx = 1.0 / n
        extra = (U[4] - 1e-5 / 0.4).sum() * dx ** 3
        assert abs(extra - 1.0) < 1e-12


def test_turbulent_box_statistics():
    U = workloads.turbulent_box(64, ndim=3, seed=2)
    rho = U[0]
    assert abs(rho.mean() - 1.0) < 0.03 and abs(rho.std() - 0.3) < 0.05
    vel = U[1:4] / rho
    assert abs(np.sqrt((vel ** 2).sum(axis=0).mean()) - 0.5 * np.sqrt(1.4)) < 1e-12


def test_solenoidal_projection():
    rng = np.random.default_rng(0)
    comps = workloads.solenoidal_velocity((32, 32, 32), rng)
    k = np.fft.fftfreq(32, 1.0 / 32)
    kk = np.meshgrid(k, k, k, indexing="ij")
    div = sum(kk[a] * np.fft.fftn(comps[a]) for a in range(3))
    assert np.abs(div).max() < 1e-9 * max(np.abs(np.fft.fftn(c)).max() for c in comps)


def test_batch_specs_ranges():
    specs = workloads.batch_problem_specs()
    assert len(specs) == 4096
    one = [s for s in specs if s[0] == 1]
    two = [s for s in specs if s[0] == 2]
    assert len(one) == 3072 and len(two) == 1024
    assert min(s[1] for s in one) >= 64 and max(s[1] for s in one) <= 4096
    assert min(s[1] for s in two) >= 32 and max(s[1] for s in two) <= 256
    for s in specs[:50]:
        assert all(0.1 <= v <= 1.0 for v in s[2])
