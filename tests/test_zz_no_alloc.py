"""hard_hydro_step_noalloc (the entry point for callers that cannot allocate)
against hard_hydro_step with a caller workspace, through the C ABI.

Both calls run the same kernels, so the states after each step and the fused
next dt must agree bit for bit (the 1e-12 FP64 bar would allow more).  Two
calls in a row share the library's static scratch; the second one takes a
smaller grid, so it must not be influenced by what the first left there.
"""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
H = pytest.importorskip("paper_2509_08971_amd")

P, O, R = 0, 1, 2
DEV = "cuda"


def log(*a):
    print(*a, flush=True)


def state(n, seed, dtype):
    full = workloads.turbulent_box(max(n), ndim=len(n), seed=seed)
    shape = tuple(reversed(n))
    sl = (slice(None),) + tuple(slice(0, s) for s in shape)
    return torch.from_numpy(np.ascontiguousarray(full[sl])).to(DEV, dtype)


def step_with_workspace(g, U0, dt0, steps):
    U = U0.clone()
    work = H.workspace(H.hard_workspace_bytes(g))
    dt = torch.full((1,), dt0, dtype=torch.float64, device=DEV)
    for _ in range(steps):
        H.hard_hydro_step(g, U, dt, work, cfl=0.4, next_dt_dev=dt)
    torch.cuda.synchronize()
    assert H.hard_status_read(work) == 0
    return U, dt.item()


def step_noalloc(g, U0, dt0, steps):
    U = U0.clone()
    dt = torch.full((1,), dt0, dtype=torch.float64, device=DEV)
    flags = torch.full((1,), 0xFFFF, dtype=torch.int32, device=DEV)
    for _ in range(steps):
        H.hard_hydro_step_noalloc(g, U, dt, cfl=0.4, next_dt_dev=dt, flags_dev=flags)
    torch.cuda.synchronize()
    assert flags.item() == 0
    return U, dt.item()


CASES = [
    # (n, bc, dtype, seed, steps): first a larger grid, then a smaller one
    ((48, 40, 36), (R, R, P, P, O, O), torch.float64, 3, 3),
    ((20, 12, 9), (P, P, R, O, O, R), torch.float64, 4, 2),
    ((96, 80), (P, P, P, P), torch.float32, 5, 3),
    ((33, 17), (R, O, P, P), torch.float32, 6, 2),
]


@pytest.mark.parametrize("first,second", [(0, 1), (2, 3), (0, 3)])
def test_noalloc_matches_workspace_step_twice(first, second):
    for k in (first, second):
        n, bc, dtype, seed, steps = CASES[k]
        log(f"noalloc case n={n} bc={bc} dtype={dtype} seed={seed} steps={steps}")
        g = H.make_grid(n, bc=bc, dtype=dtype)
        U0 = state(n, seed, dtype)
        dt0 = 0.1 / max(n) / 4.0
        ref, dt_ref = step_with_workspace(g, U0, dt0, steps)
        got, dt_got = step_noalloc(g, U0, dt0, steps)
        assert dt_got == dt_ref
        assert torch.equal(got, ref), (got - ref).abs().max().item()


def test_noalloc_rejects_grid_over_scratch():
    # 256^3 FP64: 671 MB of stage state, far beyond the static scratch
    g = H.make_grid((256, 256, 256), bc=(P, P, P, P, P, P))
    U = torch.zeros(1, dtype=torch.float64, device=DEV)
    dt = torch.zeros(1, dtype=torch.float64, device=DEV)
    with pytest.raises(H.HardError) as e:
        H.hard_hydro_step_noalloc(g, U, dt)
    assert e.value.code == H.ERR_WORKSPACE
