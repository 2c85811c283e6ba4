"""Batched step (many independent problems in one launch per stage).

* Every problem of a mixed batch equals the single-grid GPU step bit for bit,
  state and fused dt (the tile body and the per-cell arithmetic are shared).
* Every work-item shape the autotuner may pick gives the same bits.
* A subset of the 4096-problem workload: 100 steps with per-problem dt
  against the FP64 oracle per problem (FP32: relative L1 <= 1e-5 per field),
  and runs to t = 0.2 against the exact Riemann solution.
* Graph capture: replays of captured batched steps equal eager steps.
"""
import os
import tempfile

import numpy as np
import pytest

import oracle
import workloads
from oracle.metrics import field_rel_l1

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
H = pytest.importorskip("paper_2509_08971_amd")

P, O, R = 0, 1, 2
DEV = "cuda"


def log(*a):
    print(*a, flush=True)


def mixed_batch():
    rng = np.random.default_rng(77)
    specs = [((64,), (O, O)), ((300,), (R, R)), ((1000,), (P, P)), ((4096,), (O, O)),
             ((255,), (O, R)), ((256,), (P, P)),
             ((32, 32), (O, O, O, O)), ((50, 37), (P, P, R, R)), ((100, 80), (R, R, O, O)),
             ((20, 18, 16), (P, P, P, P, P, P)), ((33, 20, 40), (O, O, R, R, P, P))]
    states = []
    for n, bc in specs:
        shape = tuple(reversed(n))
        rho = rng.uniform(0.4, 1.4, shape)
        vel = [rng.uniform(-0.4, 0.4, shape) for _ in n]
        p = rng.uniform(0.4, 1.4, shape)
        states.append(workloads.conserved_from_primitive(rho, vel, p))
    return specs, states


def single_runs(specs, states, dtype, steps):
    outs, dts = [], []
    for (n, bc), U0 in zip(specs, states):
        g = H.make_grid(n, bc=bc, dtype=dtype)
        U = torch.from_numpy(U0).to(DEV, dtype)
        work = H.workspace(H.hard_workspace_bytes(g))
        d = torch.zeros(1, dtype=torch.float64, device=DEV)
        H.hard_cfl_dt(g, U, 0.4, d, work)
        for _ in range(steps):
            H.hard_hydro_step(g, U, d, work, cfl=0.4, next_dt_dev=d)
        outs.append(U.cpu())
        dts.append(d.item())
    return outs, dts


def batched_run(specs, states, dtype, steps, tune=None):
    grids = [H.make_grid(n, bc=bc, dtype=dtype) for n, bc in specs]
    plan = H.hard_batch_plan_create(grids, tune)
    try:
        offs = H.hard_batch_offsets(plan, len(grids))
        U = H.batch_pack(states, offs, dtype)
        work = H.workspace(H.hard_batch_workspace_bytes(plan))
        dt = torch.zeros(len(grids), dtype=torch.float64, device=DEV)
        H.hard_cfl_dt_batched(plan, U, 0.4, dt, work)
        for _ in range(steps):
            H.hard_hydro_step_batched(plan, U, dt, work, cfl=0.4)
        torch.cuda.synchronize()
        assert H.hard_status_read(work) == 0
        outs = [t.cpu() for t in H.batch_unpack(U, offs, [s.shape for s in states])]
        return outs, dt.cpu().tolist()
    finally:
        H.hard_batch_plan_destroy(plan)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_batched_equals_single_bitwise(dtype):
    log("batched vs single", dtype)
    specs, states = mixed_batch()
    ref, ref_dt = single_runs(specs, states, dtype, 4)
    got, got_dt = batched_run(specs, states, dtype, 4)
    for p in range(len(specs)):
        assert torch.equal(got[p], ref[p]), (p, specs[p])
        assert got_dt[p] == ref_dt[p], (p, got_dt[p], ref_dt[p])


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_batched_tile_shapes_bitwise(dtype):
    """Every setting the autotuner may write gives the same bits."""
    specs, states = mixed_batch()
    base, base_dt = batched_run(specs, states, dtype, 3)
    k3 = "tile3d_f64" if dtype == torch.float64 else "tile3d_f32"
    settings = ["walk2d = 8", "walk2d = 64\ncz = 5", f"{k3} = 8x32\ncz = 3",
                f"{k3} = 32x8\nwalk2d = 1", f"{k3} = 16x16\ncz = 64"]
    for cand in settings:
        log("tune setting", repr(cand), dtype)
        fd, path = tempfile.mkstemp(suffix=".tune")
        with os.fdopen(fd, "w") as f:
            f.write(cand + "\n")
        try:
            got, got_dt = batched_run(specs, states, dtype, 3, tune=path)
        finally:
            os.unlink(path)
        for p in range(len(specs)):
            assert torch.equal(got[p], base[p]), (cand, p)
        assert got_dt == base_dt


def _subset():
    specs_all = workloads.batch_problem_specs()
    pick = list(range(0, 3072, 160)) + list(range(3072, 4096, 52))
    specs = [specs_all[i] for i in pick]
    states = [workloads.batch_problem_state(s).astype(np.float32).astype(np.float64)
              for s in specs]
    return pick, specs, states


def _run_subset(specs, states, t_end, max_steps):
    grids = [H.make_grid((s[1],) * s[0], bc=(O, O), dtype=torch.float32) for s in specs]
    plan = H.hard_batch_plan_create(grids)
    try:
        offs = H.hard_batch_offsets(plan, len(grids))
        U = H.batch_pack(states, offs, torch.float32)
        work = H.workspace(H.hard_batch_workspace_bytes(plan))
        dt = torch.zeros(len(grids), dtype=torch.float64, device=DEV)
        ts, steps = H.hard_run_batched(plan, len(grids), U, 0.4, t_end, dt, work,
                                       max_steps=max_steps)
        outs = [t.double().cpu().numpy() for t in
                H.batch_unpack(U, offs, [s.shape for s in states])]
    finally:
        H.hard_batch_plan_destroy(plan)
    return ts, steps, outs


def test_batched_100_steps_vs_oracle_fp32():
    """40 problems of the 4096-problem recipe (every 160th 1D, every 52nd 2D),
    100 steps each with its own CFL dt (the workload's step count), against
    the FP64 oracle run of the same float-rounded initial state with its own
    CFL steps: relative L1 <= 1e-5 per field."""
    pick, specs, states = _subset()
    ts, steps, outs = _run_subset(specs, states, 1e9, 100)
    worst = 0.0
    for k, (s, U0) in enumerate(zip(specs, states)):
        og = oracle.Grid((s[1],) * s[0], bc=(O, O))
        ref, t_ref, n_ref, st = oracle.run(og, U0, 0.4, 1e9, max_steps=100)
        assert st == 0 and steps[k] == 100 and n_ref == 100
        for v in range(s[0] + 2):
            e = field_rel_l1(outs[k][v], ref[v])
            worst = max(worst, e)
            assert e <= 1e-5, (pick[k], v, e)
    log("worst FP32 relative L1 over the subset (100 steps)", worst)


def test_batched_run_to_t_end_vs_exact_riemann():
    """The same 40 problems run to t = 0.2 with per-problem clipping: every
    problem lands on t = 0.2, and its density error against the exact Riemann
    solution matches the FP64 oracle's own error (FP32 rounding is far below
    the discretisation error)."""
    from oracle.exact_riemann import RiemannSolution
    from oracle.metrics import l1_error
    pick, specs, states = _subset()
    ts, steps, outs = _run_subset(specs, states, 0.2, 10_000_000)
    for k, (s, U0) in enumerate(zip(specs, states)):
        assert ts[k] == pytest.approx(0.2, rel=1e-14)
        ndim, n, (rL, pL, rR, pR) = s
        og = oracle.Grid((n,) * ndim, bc=(O, O))
        ref, t_ref, n_ref, st = oracle.run(og, U0, 0.4, 0.2)
        assert abs(steps[k] - n_ref) <= 1
        ex = RiemannSolution(rL, 0.0, pL, rR, 0.0, pR)
        r_ex, _, _ = ex.cell_averages(n, 0.2)
        rho_gpu = outs[k][0] if ndim == 1 else outs[k][0].mean(axis=0)
        rho_ref = ref[0] if ndim == 1 else ref[0].mean(axis=0)
        e_gpu = l1_error(rho_gpu, r_ex, 1.0 / n)
        e_ref = l1_error(rho_ref, r_ex, 1.0 / n)
        assert abs(e_gpu - e_ref) <= 0.02 * e_ref + 1e-6, (pick[k], e_gpu, e_ref)


def test_batched_graph_replay():
    """Captured batched steps replayed three times, eager work in between; each
    replay must equal the same steps run eagerly."""
    specs, states = mixed_batch()
    grids = [H.make_grid(n, bc=bc, dtype=torch.float32) for n, bc in specs]
    plan = H.hard_batch_plan_create(grids)
    try:
        offs = H.hard_batch_offsets(plan, len(grids))
        U = H.batch_pack(states, offs, torch.float32)
        work = H.workspace(H.hard_batch_workspace_bytes(plan))
        dt = torch.zeros(len(grids), dtype=torch.float64, device=DEV)
        H.hard_cfl_dt_batched(plan, U, 0.4, dt, work)
        torch.cuda.synchronize()
        U0, dt0 = U.clone(), dt.clone()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.stream(s):
            H.hard_hydro_step_batched(plan, U, dt, work, cfl=0.4)  # warm-up on the side stream
            s.synchronize()
            U.copy_(U0)
            dt.copy_(dt0)
            s.synchronize()
            with torch.cuda.graph(graph, stream=s):
                for _ in range(3):
                    H.hard_hydro_step_batched(plan, U, dt, work, cfl=0.4)
        torch.cuda.synchronize()
        # eager reference
        Ue, dte = U0.clone(), dt0.clone()
        for _ in range(3):
            H.hard_hydro_step_batched(plan, Ue, dte, work, cfl=0.4)
        torch.cuda.synchronize()
        for rep in range(3):
            U.copy_(U0)
            dt.copy_(dt0)
            torch.cuda.synchronize()
            graph.replay()
            torch.cuda.synchronize()
            assert torch.equal(U, Ue), rep
            assert torch.equal(dt, dte), rep
            _ = (Ue * 2).sum().item()  # unrelated eager work between replays
    finally:
        H.hard_batch_plan_destroy(plan)


def test_batched_full_workload_sampled():
    """The full 4096-problem batch (3072 1D + 1024 2D, FP32): three steps, then
    sampled problems equal single-grid GPU steps bit for bit."""
    specs_all = workloads.batch_problem_specs()
    states = [workloads.batch_problem_state(s) for s in specs_all]
    grids = [H.make_grid((s[1],) * s[0], bc=(O, O), dtype=torch.float32) for s in specs_all]
    plan = H.hard_batch_plan_create(grids)
    try:
        offs = H.hard_batch_offsets(plan, len(grids))
        U = H.batch_pack(states, offs, torch.float32)
        work = H.workspace(H.hard_batch_workspace_bytes(plan))
        dt = torch.zeros(len(grids), dtype=torch.float64, device=DEV)
        H.hard_cfl_dt_batched(plan, U, 0.4, dt, work)
        for _ in range(3):
            H.hard_hydro_step_batched(plan, U, dt, work, cfl=0.4)
        torch.cuda.synchronize()
        assert H.hard_status_read(work) == 0
        sample = [0, 1, 777, 3071, 3072, 3500, 4095]
        shapes = [states[i].shape for i in range(len(states))]
        outs = H.batch_unpack(U, offs, shapes)
        dts = dt.cpu().tolist()
    finally:
        H.hard_batch_plan_destroy(plan)
    for i in sample:
        s = specs_all[i]
        ref, ref_dt = single_runs([((s[1],) * s[0], (O, O))], [states[i]], torch.float32, 3)
        assert torch.equal(outs[i].cpu(), ref[0]), i
        assert dts[i] == ref_dt[0], i


def test_autotuner_writes_a_cache_the_plan_reads(tmp_path):
    """tune_batched times every candidate setting on the caller's grids and
    writes the winners; a plan built from that cache gives the same bits as
    the default plan."""
    from paper_2509_08971_amd import autotune

    specs, states = mixed_batch()
    grids = [H.make_grid(n, bc=bc, dtype=torch.float32) for n, bc in specs]
    cache = tmp_path / "batched.tune"
    best, times = autotune.tune_batched(grids, states, torch.float32, steps=2,
                                        cache_path=str(cache))
    text = cache.read_text()
    for k, v in best.items():
        assert f"{k} = {v}" in text
    assert len(times) == sum(len(v) for v in autotune.default_candidates(torch.float32).values())
    base, base_dt = batched_run(specs, states, torch.float32, 3)
    got, got_dt = batched_run(specs, states, torch.float32, 3, tune=str(cache))
    for p in range(len(specs)):
        assert torch.equal(got[p], base[p])
    assert got_dt == base_dt
