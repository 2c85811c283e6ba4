"""hard_run on small 1D grids (at most 2048 cells) runs its whole time loop in
one resident workgroup.  Its arithmetic is that of the tiled step,
expression for expression, so a run must equal, bit for bit, the same run
made one hard_hydro_step at a time with the fused next dt and the time
control done on the host in the same double arithmetic: same final state,
same step count, same t.  Cases span both cell counts per thread, the ragged
sizes around 1024, the smallest grids, every boundary kind, FP32, runs that
cross the 1024-step launch boundary, and a run cut short by max_steps."""
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


def stepwise(g, U, cfl, t_end, max_steps):
    """The time loop of hard_run one step at a time: dt from the CFL step of
    the current state, clamped so the run lands on t_end."""
    work = H.workspace(H.hard_workspace_bytes(g))
    dt = torch.zeros(1, dtype=torch.float64, device=DEV)
    H.hard_cfl_dt(g, U, cfl, dt, work)
    t, steps = 0.0, 0
    while t < t_end * (1.0 - 1e-14) and steps < max_steps:
        d = dt.item()
        if d > t_end - t:
            d = t_end - t
        dt.fill_(d)
        t = t + d
        steps += 1
        H.hard_hydro_step(g, U, dt, work, cfl=cfl, next_dt_dev=dt)
    torch.cuda.synchronize()
    return t, steps


CASES = [
    (1024, (O, O), torch.float64, 0.2, 10_000_000),
    (1000, (R, R), torch.float64, 0.1, 10_000_000),
    (1025, (P, P), torch.float64, 0.05, 10_000_000),
    (2048, (O, R), torch.float64, 0.2, 10_000_000),   # > 1024 steps: two launches
    (2, (P, P), torch.float64, 0.05, 10_000_000),
    (3, (R, O), torch.float64, 0.05, 10_000_000),
    (777, (O, O), torch.float32, 0.2, 10_000_000),
    (1536, (R, R), torch.float32, 0.1, 10_000_000),
    (512, (O, O), torch.float64, 0.2, 37),            # stopped by max_steps
]


@pytest.mark.parametrize("n,bc,dtype,t_end,max_steps", CASES)
def test_run1d_equals_stepwise_loop(n, bc, dtype, t_end, max_steps):
    log(f"run1d n={n} bc={bc} {dtype} t_end={t_end} max_steps={max_steps}")
    U0 = workloads.random_two_state(n, seed=n % 7)
    g = H.make_grid((n,), bc=bc, dtype=dtype)
    Ua = torch.from_numpy(U0).to(DEV, dtype)
    Ub = Ua.clone()
    work = H.workspace(H.hard_workspace_bytes(g))
    t_a, s_a = H.hard_run(g, Ua, 0.4, t_end, work, max_steps=max_steps)
    assert H.hard_status_read(work) == 0
    t_b, s_b = stepwise(g, Ub, 0.4, t_end, max_steps)
    assert s_a == s_b and t_a == t_b, (s_a, s_b, t_a, t_b)
    if max_steps >= 10_000_000:
        assert t_a == pytest.approx(t_end, rel=1e-13)
    else:
        assert s_a == max_steps
    assert torch.equal(Ua, Ub)
