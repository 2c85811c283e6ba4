"""Throughput of the explicit hydro step on one MI355X.

Workload: the 256^3 FP64 point-energy blast (rho = 1, p = 1e-5, u = 0,
E0 = 1 over the 32 cells within 2 dx of the centre, gamma = 1.4, reflecting
walls), CFL 0.4.  One timed step is one full Heun step (stage-1 kernel +
stage-2 kernel with the next CFL dt folded in), the state resident in HBM.
After the warmup steps the state is reset to the initial blast, so the timed
steps are steps 1..K of the blast.

Prints one JSON line: zone-updates/s, the HBM roofline of the dominant kernel
(stage 2) from HIP events around each launch, and the CPU oracle timed on a
bounded sample of the same workload on the host cores.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402
import torch  # noqa: E402

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
# floating-point operations of one zone-update in 3D as the oracle evaluates
# them (oracle.ops_per_zone_update: 485 add, 378 mul, 87 div, 13 sqrt, 118
# compare, 64 abs); tests/test_oracle_opcount.py recomputes it
OPS_PER_ZU_3D = 1145


# Sources of the stage kernel; HBM byte counts taken with rocprofv3 are
# reported only while these files are unchanged since the counters were read.
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2509_08971_amd", "csrc", f)
                  for f in ("hydro_device.hpp", "stage_tile.hpp", "stage.hip", "launch.hpp")]
COUNTERS_FILE = os.path.join(ROOT, "profiles", "stage_kernel_blast256_fp64_hbm_counters.md")
def _csrc(*names):
    return [os.path.join(ROOT, "paper_2509_08971_amd", "csrc", f) for f in names]


FLD_SOURCES = _csrc("fld.hip", "hydro_device.hpp")
FLD_COUNTERS_FILE = os.path.join(ROOT, "profiles", "fld_relax_diffusion256_fp64_hbm_counters.md")
WENO_SOURCES = _csrc("weno.hip", "hydro_device.hpp", "launch.hpp")
WENO_COUNTERS_FILE = os.path.join(ROOT, "profiles", "weno_pipeline_blast256_fp64_hbm_counters.md")
RAD_SOURCES = _csrc("rad.hip", "stage.hip", "stage_tile.hpp", "hydro_device.hpp", "launch.hpp")
RAD_COUNTERS_FILE = os.path.join(ROOT, "profiles", "rad_step_radiation256_fp64_hbm_counters.md")


def code_hash(files):
    """sha256 of the code of the given C++/HIP sources: comments, trailing
    blanks and empty lines removed, so that an edit of a comment keeps the
    counters taken on the same code."""
    import hashlib
    import re

    h = hashlib.sha256()
    for f in files:
        with open(f) as fh:
            text = re.sub(r"/\*.*?\*/", "", fh.read(), flags=re.S)
        for line in text.splitlines():
            line = line.split("//", 1)[0].rstrip()
            if line:
                h.update(line.encode() + b"\n")
    return h.hexdigest()


def kernel_source_hash():
    return code_hash(KERNEL_SOURCES)


def fld_source_hash():
    return code_hash(FLD_SOURCES)


def measured_bytes(path, key, sources):
    """HBM bytes (FETCH_SIZE and WRITE_SIZE scaled by the copy-kernel factors)
    per unit of a bench leg from the committed counter summary `path`: its
    lines `<key>-source-sha256` and `<key>-bytes-measured`, or None if the code
    of `sources` changed since the counters were taken."""
    try:
        with open(path) as f:
            lines = dict(l.split(": ", 1) for l in f.read().splitlines()
                         if l.startswith(key + "-") and ": " in l)
    except OSError:
        return None
    if lines.get(f"{key}-source-sha256", "").strip() != code_hash(sources):
        return None
    try:
        return int(lines[f"{key}-bytes-measured"])
    except (KeyError, ValueError):
        return None


def fld_measured_cycle_bytes():
    """HBM bytes per V(2,2) cycle of the 256^3 diffusion."""
    return measured_bytes(FLD_COUNTERS_FILE, "fld", FLD_SOURCES)


def _counter_lines():
    """Machine-readable lines of the committed counter summary, or {} if the
    kernel sources changed since the counters were taken."""
    try:
        with open(COUNTERS_FILE) as f:
            kv = dict(l.split(":", 1) for l in f.read().splitlines() if ":" in l and
                      l.split(":", 1)[0].strip().startswith(("kernel-source-sha256", "stage1-",
                                                             "stage2-")))
    except OSError:
        return {}
    kv = {k.strip(): v.strip() for k, v in kv.items()}
    if kv.get("kernel-source-sha256") != kernel_source_hash():
        return {}
    return kv


def measured_traffic():
    """Stage-2 HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, each scaled by the
    copy-kernel factor), from the committed counter summary, or None if the
    kernel sources changed since it was taken."""
    kv = _counter_lines()
    try:
        return (int(kv["stage2-fetch-bytes-per-launch"]), int(kv["stage2-write-bytes-per-launch"]))
    except (KeyError, ValueError):
        return None


def measured_valu():
    """SQ_INSTS_VALU per 64 cells of stage 1 and stage 2 (same rule as above)."""
    kv = _counter_lines()
    try:
        return (float(kv["stage1-valu-per-64-cells"]), float(kv["stage2-valu-per-64-cells"]))
    except (KeyError, ValueError):
        return None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _time_steps(fn, steps, stream):
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record(stream)
    for _ in range(steps):
        fn()
    b.record(stream)
    torch.cuda.synchronize()
    return a.elapsed_time(b)


def bench_fp32_turbulent(args, n=512, steps=50):
    """512^3 periodic turbulent box, FP32 bulk, 50 steps with fused CFL dt."""
    import paper_2509_08971_amd as H
    import workloads

    log(f"bench: turbulent {n}^3 fp32, {steps} steps")
    U = workloads.turbulent_box_torch(n, ndim=3, seed=2, device="cuda", dtype=torch.float32)
    U0 = U.clone()
    g = H.make_grid((n, n, n), bc=(H.PERIODIC, H.PERIODIC), dtype=torch.float32)
    work = H.workspace(H.hard_workspace_bytes(g))
    dt = torch.zeros(1, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    H.hard_cfl_dt(g, U, 0.4, dt, work)
    for _ in range(3):
        H.hard_hydro_step(g, U, dt, work, cfl=0.4, next_dt_dev=dt)
    U.copy_(U0)
    H.hard_cfl_dt(g, U, 0.4, dt, work)
    ms = _time_steps(lambda: H.hard_hydro_step(g, U, dt, work, cfl=0.4, next_dt_dev=dt), steps,
                     stream)
    flags = H.hard_status_read(work)
    N = n ** 3
    zus = N * steps / (ms * 1e-3)
    bytes_step = 5 * 5 * 4 * N
    log(f"  {ms / steps:.3f} ms/step, {zus / 1e9:.2f} G zu/s")
    # accuracy against the plain FP64 step: the same initial state (the float
    # values widened) run in double with the fused CFL steps, then in float
    # with that dt sequence; per-field sum|f32 - f64| / sum|f64| at the end
    g64 = H.make_grid((n, n, n), bc=(H.PERIODIC, H.PERIODIC), dtype=torch.float64)
    work64 = H.workspace(H.hard_workspace_bytes(g64))
    U64 = U0.double()
    dts = torch.zeros(steps + 1, dtype=torch.float64, device="cuda")
    H.hard_cfl_dt(g64, U64, 0.4, dts[0:1], work64)
    for s in range(steps):
        H.hard_hydro_step(g64, U64, dts[s:s + 1], work64, cfl=0.4, next_dt_dev=dts[s + 1:s + 2])
    U32 = U0.clone()
    for s in range(steps):
        H.hard_hydro_step(g, U32, dts[s:s + 1], work)
    err = [((U32[v].double() - U64[v]).abs().sum() / U64[v].abs().sum()).item() for v in range(5)]
    flags |= H.hard_status_read(work) | H.hard_status_read(work64)
    del U64, work64, U32
    log(f"  per-field rel L1 vs the FP64 step after {steps} steps: "
        + ", ".join(f"{e:.2e}" for e in err))
    return {"value": zus, "unit": "zone-updates/s", "ms_per_step": ms / steps, "steps": steps,
            "dtype": "f32 (internal energy, dt in f64)",
            "workload": f"3D {n}^3 periodic log-normal rho, p = 1, solenoidal u (rms Mach 0.5)",
            "achieved_hbm_gbs": bytes_step / (ms / steps * 1e-3) / 1e9,
            "rel_l1_vs_fp64_step_per_field": dict(zip(["rho", "m_x", "m_y", "m_z", "E"], err)),
            "accuracy_bound": 1e-5, "status_flags": flags}


def bench_batched(args, steps=100):
    """4096 two-state problems (3072 1D nx in [64,4096], 1024 2D side in
    [32,256]), FP32, 100 steps each with per-problem CFL dt, the steps
    replayed from one captured graph."""
    import paper_2509_08971_amd as H
    import workloads

    log(f"bench: batched 4096 problems fp32, {steps} steps")
    specs = workloads.batch_problem_specs()
    grids = [H.make_grid((s[1],) * s[0], bc=(H.OUTFLOW, H.OUTFLOW), dtype=torch.float32)
             for s in specs]
    plan = H.hard_batch_plan_create(grids, None)
    try:
        offs = H.hard_batch_offsets(plan, len(grids))
        host = np.zeros(offs[-1], dtype=np.float32)
        cells = 0
        bytes_step = 0
        for p, s in enumerate(specs):
            a = workloads.batch_problem_state(s).astype(np.float32).ravel()
            host[offs[p]:offs[p] + a.size] = a
            nv = s[0] + 2
            cells += a.size // nv
            bytes_step += 5 * a.size * 4
        U = torch.from_numpy(host).to("cuda")
        U0 = U.clone()
        work = H.workspace(H.hard_batch_workspace_bytes(plan))
        dt = torch.zeros(len(grids), dtype=torch.float64, device="cuda")
        H.hard_cfl_dt_batched(plan, U, 0.4, dt, work)
        dt0 = dt.clone()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.stream(side):
            H.hard_hydro_step_batched(plan, U, dt, work, cfl=0.4)
            side.synchronize()
            with torch.cuda.graph(graph, stream=side):
                for _ in range(steps):
                    H.hard_hydro_step_batched(plan, U, dt, work, cfl=0.4)
        torch.cuda.synchronize()
        U.copy_(U0)
        dt.copy_(dt0)
        stream = torch.cuda.current_stream()
        ms = _time_steps(graph.replay, 1, stream)
        flags = H.hard_status_read(work)
    finally:
        H.hard_batch_plan_destroy(plan)
    zus = cells * steps / (ms * 1e-3)
    log(f"  {ms / steps:.3f} ms/step, {zus / 1e9:.2f} G zu/s ({cells} cells)")
    return {"value": zus, "unit": "zone-updates/s", "ms_per_step": ms / steps, "steps": steps,
            "cells": cells, "problems": len(specs), "dtype": "f32 (internal energy, dt in f64)",
            "launch": f"{steps} steps x (2 persistent stage launches + 1 per-problem dt "
                      f"launch) replayed from one captured graph",
            "achieved_hbm_gbs": bytes_step / (ms / steps * 1e-3) / 1e9, "status_flags": flags}


def bench_weno(args, n=256, steps=10):
    """The paper's own face scheme (WENO5-Z + HLL) on the 256^3 FP64 blast:
    the same step, as the per-axis pipeline (primitives, three face-flux
    kernels, update with the fused CFL step)."""
    import paper_2509_08971_amd as H
    import workloads

    log(f"bench: WENO5-Z + HLL blast {n}^3 fp64, {steps} steps")
    g = H.make_grid((n, n, n), bc=(H.REFLECT, H.REFLECT), scheme=H.WENO5Z_HLL)
    U = torch.from_numpy(workloads.blast_3d(n)).to("cuda")
    work = H.workspace(H.hard_workspace_bytes(g))
    dt = torch.zeros(1, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    H.hard_cfl_dt(g, U, 0.4, dt, work)
    for _ in range(2):
        H.hard_hydro_step(g, U, dt, work, cfl=0.4, next_dt_dev=dt)
    ms = _time_steps(lambda: H.hard_hydro_step(g, U, dt, work, cfl=0.4, next_dt_dev=dt), steps,
                     stream)
    flags = H.hard_status_read(work)
    N = n ** 3
    zus = N * steps / (ms * 1e-3)
    # pipeline words per cell and stage: prim (read U, write W), 3 x face
    # (read W, write F), update (read 3 F, read src, write dst; stage 2 also
    # reads U^n): 2 + 6 + 5 (+1) words of nvar; both stages
    words = (2 + 6 + 5) + (2 + 6 + 6)
    pipe_bytes = words * 5 * 8
    log(f"  {ms / steps:.3f} ms/step, {zus / 1e9:.2f} G zu/s")
    return {"value": zus, "unit": "zone-updates/s", "ms_per_step": ms / steps, "steps": steps,
            "dtype": "f64", "workload": f"3D {n}^3 FP64 point-energy blast, reflecting, CFL 0.4, "
                                         f"WENO5-Z + HLL (the paper's scheme) + SSP-RK2",
            "pipeline_bytes_per_zone_update": pipe_bytes,
            "roofline": {"bound": "hbm", "kernel": "whole WENO5-Z + HLL step (pipeline bytes)",
                         "achieved": pipe_bytes * zus / 1e9, "peak": 8000.0, "unit": "GB/s",
                         "frac": pipe_bytes * zus / 1e9 / 8000.0,
                         "traffic": measured_bytes(WENO_COUNTERS_FILE, "weno", WENO_SOURCES),
                         "algorithmic_bytes": pipe_bytes * N, "per": "step"},
            "status_flags": flags}


def bench_rad(args, n=256, steps=20):
    """The 256^3 FP64 blast carrying the radiation energy density (uniform
    E_r = 1, kappa = 1e-9 cm^2/g, mu = 0.6): the hydro stage kernels, the
    Rusanov advection of E_r in both stages and the heating/cooling exchange
    with the fused next dt."""
    import paper_2509_08971_amd as H
    import workloads

    log(f"bench: radiation blast {n}^3 fp64, {steps} steps")
    rad = (1e-9, 0.6)
    g = H.make_grid((n, n, n), bc=(H.REFLECT, H.REFLECT), rad=rad)
    U = torch.ones((6, n, n, n), dtype=torch.float64, device="cuda")
    U[:5] = torch.from_numpy(workloads.blast_3d(n)).to("cuda")
    work = H.workspace(H.hard_workspace_bytes(g))
    dt = torch.zeros(1, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    H.hard_cfl_dt(g, U, 0.4, dt, work)
    for _ in range(2):
        H.hard_hydro_step(g, U, dt, work, cfl=0.4, next_dt_dev=dt)
    ms = _time_steps(lambda: H.hard_hydro_step(g, U, dt, work, cfl=0.4, next_dt_dev=dt), steps,
                     stream)
    flags = H.hard_status_read(work)
    N = n ** 3
    zus = N * steps / (ms * 1e-3)
    # algorithmic bytes per zone-update: hydro stage 1 (read U^n, write U^1:
    # 2 x 5 words) and stage 2 (read U^1, U^n, write: 3 x 5); E_r advection
    # stage 1 (read 6 fields, write E_r) and stage 2 (also read E_r of U^n);
    # exchange + next dt (read 6 fields, write E and E_r)
    step_bytes = 8 * ((10 + 15) + (6 + 1) + (6 + 2) + (6 + 2))
    log(f"  {ms / steps:.3f} ms/step, {zus / 1e9:.2f} G zu/s")
    return {"value": zus, "unit": "zone-updates/s", "ms_per_step": ms / steps, "steps": steps,
            "dtype": "f64", "workload": f"3D {n}^3 FP64 point-energy blast with the radiation "
                                         f"energy density (E_r = 1, kappa = 1e-9, mu = 0.6)",
            "step_bytes_per_zone_update": step_bytes,
            "roofline": {"bound": "hbm", "kernel": "whole radiation step (stage kernels, E_r "
                                                  "advection, exchange)",
                         "achieved": step_bytes * zus / 1e9, "peak": 8000.0, "unit": "GB/s",
                         "frac": step_bytes * zus / 1e9 / 8000.0,
                         "traffic": measured_bytes(RAD_COUNTERS_FILE, "rad", RAD_SOURCES),
                         "algorithmic_bytes": step_bytes * N, "per": "step"},
            "status_flags": flags}


def fld_cycle_bytes(levels):
    """Algorithmic HBM bytes of one V(2,2) cycle over the given level sizes,
    per cell of a level: 8 red-black half-sweeps of 20 B (read the other
    colour's x, the own colour's b, both colours' D; write the own x); the
    restriction of the red residuals (the black ones are zero after the
    black half-sweep): read b, x and D of the red cells and x and D of the
    black ones, 20 B, and write the coarse b and x, 2 B; the prolongation into
    the black cells only (the red half-sweep that follows overwrites the red
    ones): read and write the black x, 8 B, and read the coarse x, 1 B.  The
    coarsest level has no transfers."""
    total = 0
    for l, (a, b, c) in enumerate(levels):
        cells = a * b * c
        total += 8 * 20 * cells
        if l + 1 < len(levels):
            total += (20 + 2 + 8 + 1) * cells
    return total


def bench_fld(args, n=256, ncycles=4, reps=10):
    """One implicit radiation diffusion step on the 256^3 grid: D from the
    Levermore limiter on a hot Gaussian radiation spot in a uniform gas
    (rho = 1 g/cm^3, kappa = 1 cm^2/g, reflecting walls), dt = 1e-12 s
    (dt D / dx^2 of about 650 in the cold gas), four V(2,2) cycles."""
    import paper_2509_08971_amd as H

    log(f"bench: radiation diffusion {n}^3 fp64, {ncycles} V(2,2) cycles")
    g = H.make_grid((n, n, n), bc=(H.REFLECT, H.REFLECT), rad=(1.0, 0.6))
    c = (torch.arange(n, dtype=torch.float64, device="cuda") + 0.5) / n - 0.5
    r2 = c[None, None, :] ** 2 + c[None, :, None] ** 2 + c[:, None, None] ** 2
    U = torch.zeros((6, n, n, n), dtype=torch.float64, device="cuda")
    U[0] = 1.0
    U[4] = 1.0
    a_rad = 4.0 * 5.670374419e-5 / 2.99792458e10
    T = 1e4 + 1e6 * torch.exp(-r2 / 0.01)
    U0 = U.clone()
    U0[5] = a_rad * T ** 4
    work = H.workspace(H.hard_rad_diffuse_workspace_bytes(g))
    dt = torch.full((1,), 1e-12, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    levels = H.hard_gmg_levels(g)
    res = torch.empty(ncycles + 1, dtype=torch.float64, device="cuda")
    U.copy_(U0)
    H.hard_rad_diffuse(g, U, dt, work, ncycles=ncycles, resid_dev=res)
    torch.cuda.synchronize()
    r = res.cpu().numpy()
    def timed(nc):
        times = []
        for _ in range(reps):
            U.copy_(U0)
            times.append(_time_steps(lambda: H.hard_rad_diffuse(g, U, dt, work, ncycles=nc), 1,
                                     stream))
        return sorted(times)[len(times) // 2]

    ms = timed(ncycles)
    ms2 = timed(2 * ncycles)  # the extra cycles alone give the time of one cycle
    flags = H.hard_status_read(work)
    N = n ** 3
    cyc = fld_cycle_bytes(levels)
    ms_cycle = (ms2 - ms) / ncycles
    log(f"  {ms:.3f} ms per diffusion step, {ms_cycle:.3f} ms per V-cycle, "
        f"{N / ms / 1e6:.2f} G cells/s, residual {r[0]:.3e} -> {r[-1]:.3e}")
    achieved = cyc / (ms_cycle * 1e-3) / 1e9
    return {"value": N / (ms * 1e-3), "unit": "zone-updates/s",
            "ms_per_step": ms, "ms_per_cycle": ms_cycle, "dtype": "f64",
            "workload": f"3D {n}^3 FP64 implicit flux-limited diffusion of E_r (Levermore), "
                        f"hot Gaussian spot, {ncycles} V(2,2) cycles, {len(levels)} levels",
            "residual_reduction": float(r[-1] / r[0]),
            "roofline": {"bound": "hbm", "kernel": "one V(2,2) cycle (all levels)",
                         "achieved": achieved, "peak": 8000.0, "unit": "GB/s",
                         "frac": achieved / 8000.0, "traffic": fld_measured_cycle_bytes(),
                         "algorithmic_bytes": cyc, "per": "V(2,2) cycle"},
            "timing": f"median of {reps} calls each of {ncycles} and {2 * ncycles} cycles, HIP "
                      f"events on the launch stream; a cycle is the difference / {ncycles}",
            "status_flags": flags}


def bench_adjoint(args, n=512, nsteps=200, every=20):
    """Config-4 gradient: 2D 512^2 FP64 periodic, 200 steps, checkpoints every
    20; gradient of J = dx^2/2 sum (rho_N - rho_T)^2 wrt the initial state."""
    import time as _t

    import paper_2509_08971_amd as H
    from paper_2509_08971_amd import autograd as AG
    import workloads

    log(f"bench: adjoint {n}^2 fp64, {nsteps} steps, checkpoint every {every}")
    g = H.make_grid((n, n), bc=(H.PERIODIC, H.PERIODIC))
    U0 = torch.from_numpy(workloads.turbulent_box(n, ndim=2, seed=4)).to("cuda")
    UT0 = torch.from_numpy(workloads.turbulent_box(n, ndim=2, seed=4,
                                                   rho_perturb=(0.01, 5))).to("cuda")
    dts, _ = AG.recorded_dts(U0, g, nsteps)
    rhoT = AG.run_fixed(UT0, g, dts)[0]
    torch.cuda.synchronize()
    t0 = _t.perf_counter()
    AG.recorded_dts(U0, g, nsteps)
    torch.cuda.synchronize()
    fwd = _t.perf_counter() - t0
    def gradient():
        X = U0.clone().requires_grad_(True)
        UN = AG.rollout(X, g, nsteps, 0.4, every)
        J = 0.5 * (1.0 / n) ** 2 * ((UN[0] - rhoT) ** 2).sum()
        J.backward()
        return X.grad

    gradient()  # untimed: the allocator's first requests for the checkpoints and buffers
    torch.cuda.synchronize()
    t0 = _t.perf_counter()
    gradient()
    torch.cuda.synchronize()
    full = _t.perf_counter() - t0
    N = n * n
    log(f"  forward {fwd * 1e3:.1f} ms, forward+gradient {full * 1e3:.1f} ms")
    return {"forward_ms": fwd * 1e3, "gradient_ms": full * 1e3,
            "gradient_over_forward": full / fwd,
            "forward_zone_updates_per_s": N * nsteps / fwd,
            "gradient_zone_updates_per_s": N * nsteps / full,
            "workload": f"2D {n}^2 FP64 periodic, {nsteps} steps, checkpoints every {every}, "
                        f"loss on final rho against a perturbed-start target",
            "timing": "host wall clock around the whole forward / forward+backward, after "
                      "one untimed forward+backward (allocator warm-up)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=2)
    ap.add_argument("--only-main", action="store_true",
                    help="time only the FP64 blast (skip the FP32 and batched lines)")
    ap.add_argument("--only-leg", choices=["fp32", "batched", "adjoint", "weno", "rad", "fld"],
                    help="only time one of the legs beside the FP64 step (prints its object)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy 5 times (the reference "
                         "kernel for scaling HBM byte counters)")
    args = ap.parse_args()
    if args.copy_probe:
        a = torch.ones(1 << 27, dtype=torch.float64, device="cuda")  # 1 GiB
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_each_way": a.numel() * 8, "launches": 5}), flush=True)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the kernels run on one GPU; --gpus must be 1"}), flush=True)
        sys.exit(2)
    if args.only_leg:
        legs = {"fp32": ("fp32_512_turbulent", bench_fp32_turbulent),
                "batched": ("batched_4096", bench_batched),
                "adjoint": ("adjoint_512", bench_adjoint),
                "weno": ("weno5z_hll_256", bench_weno),
                "rad": ("radiation_256", bench_rad),
                "fld": ("radiation_diffusion_256", bench_fld)}
        name, fn = legs[args.only_leg]
        print(json.dumps({name: fn(args)}), flush=True)
        return

    import paper_2509_08971_amd as H
    import workloads

    n = args.n
    N = n ** 3
    nvar, w = 5, 8
    dev = torch.device("cuda:0")
    g = H.make_grid((n, n, n), bc=(H.REFLECT, H.REFLECT))
    U0_host = workloads.blast_3d(n)
    U0 = torch.from_numpy(U0_host).to(dev)
    U = U0.clone()
    U1 = torch.empty_like(U)
    work = H.workspace(H.hard_workspace_bytes(g), dev)
    dt = torch.zeros(1, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()

    def step(ev=None):
        if ev is not None:
            ev[0].record(stream)
        H.hard_hydro_stage(g, 1, U, None, U1, dt, work)
        if ev is not None:
            ev[1].record(stream)
        H.hard_hydro_stage(g, 2, U1, U, U, dt, work, cfl=0.4, next_dt_dev=dt)
        if ev is not None:
            ev[2].record(stream)

    log(f"bench: blast {n}^3 fp64, warmup {args.warmup}, steps {args.steps}")
    H.hard_cfl_dt(g, U, 0.4, dt, work)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # reset to the initial state (untimed)
    U.copy_(U0)
    H.hard_cfl_dt(g, U, 0.4, dt, work)
    torch.cuda.synchronize()

    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record(stream)
    for k in range(args.steps):
        step(evs[k])
    stop.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_total = start.elapsed_time(stop)
    flags = H.hard_status_read(work)
    s1 = np.array([e[0].elapsed_time(e[1]) for e in evs])
    s2 = np.array([e[1].elapsed_time(e[2]) for e in evs])
    ms_per_step = ms_total / args.steps
    zus = N * args.steps / (ms_total * 1e-3)
    log(f"  {ms_per_step:.3f} ms/step (wall {wall * 1e3 / args.steps:.3f}), {zus / 1e9:.2f} G zu/s, "
        f"stage1 {s1.mean():.3f} ms, stage2 {s2.mean():.3f} ms, flags {flags}")

    b_stage2 = 3 * nvar * w * N  # read U1, read U^n, write U^{n+1}
    b_stage1 = 2 * nvar * w * N  # read U^n, write U1
    ach2 = b_stage2 / (s2.mean() * 1e-3) / 1e9
    ach1 = b_stage1 / (s1.mean() * 1e-3) / 1e9
    step_gbs = (b_stage1 + b_stage2) / (ms_per_step * 1e-3) / 1e9
    traffic = measured_traffic() if n == 256 else None
    valu = measured_valu() if n == 256 else None

    out = {
        "metric": "zone-updates/s",
        "value": zus,
        "unit": "zone-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"3D {n}^3 FP64 point-energy blast, reflecting, CFL 0.4, "
                               f"MUSCL-minmod + HLLC + SSP-RK2 with fused CFL dt",
                   "cells": N, "parallelism": "single GPU"},
        "achieved_hbm_gbs_step": step_gbs,
        "roofline": {"bound": "hbm", "kernel": "stage_kernel<3,double,2> (stage 2)",
                     "achieved": ach2, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": ach2 / HBM_PEAK_GBS,
                     "traffic": (sum(traffic) if traffic else None),
                     "traffic_fetch_write": traffic, "algorithmic_bytes": b_stage2,
                     "stage1_achieved": ach1, "stage1_ms": float(s1.mean()),
                     "stage2_ms": float(s2.mean())},
        "status_flags": flags,
    }
    # the VALU ceiling beside the byte roofline: one wave64 FP64 instruction
    # per 4 cycles on each of 1024 SIMDs at 2.4 GHz = 39.3 T lane-instr/s
    lane_peak = 256 * 4 * 16 * 2.4e9
    alu = {"bound": "alu", "unit": "lane-instr/s", "peak": lane_peak,
           "oracle_ops_per_zone_update": OPS_PER_ZU_3D}
    if valu:
        per_zu = valu[0] + valu[1]  # lane-instructions per zone-update, both stages
        alu.update({"valu_per_zone_update": per_zu, "achieved": zus * per_zu,
                    "frac": zus * per_zu / lane_peak, "ceiling_zone_updates_per_s": lane_peak / per_zu})
    out["alu_beside"] = alu

    if not args.only_main:
        extras = {}
        try:
            extras["fp32_512_turbulent"] = bench_fp32_turbulent(args)
        except Exception as e:  # reported, never hidden
            extras["fp32_512_turbulent"] = {"error": repr(e)}
        try:
            extras["batched_4096"] = bench_batched(args)
        except Exception as e:
            extras["batched_4096"] = {"error": repr(e)}
        try:
            extras["adjoint_512"] = bench_adjoint(args)
        except Exception as e:
            extras["adjoint_512"] = {"error": repr(e)}
        try:
            extras["weno5z_hll_256"] = bench_weno(args)
        except Exception as e:
            extras["weno5z_hll_256"] = {"error": repr(e)}
        try:
            extras["radiation_256"] = bench_rad(args)
        except Exception as e:
            extras["radiation_256"] = {"error": repr(e)}
        try:
            extras["radiation_diffusion_256"] = bench_fld(args)
        except Exception as e:
            extras["radiation_diffusion_256"] = {"error": repr(e)}
        out["beside_fp64_step"] = extras

    if not args.no_cpu_baseline:
        import oracle

        og = oracle.Grid((n, n, n), bc=(oracle.REFLECT, oracle.REFLECT))
        ksteps = args.cpu_steps
        log(f"cpu baseline: oracle, {ksteps} steps of the same blast on {oracle.threads()} threads")
        dt0, _ = oracle.cfl_dt(og, U0_host, 0.4)
        t0 = time.perf_counter()
        Uc = U0_host
        for _ in range(ksteps):
            d, _ = oracle.cfl_dt(og, Uc, 0.4)
            Uc, _ = oracle.step(og, Uc, d)
        el = time.perf_counter() - t0
        cpu = "unknown CPU"
        try:
            with open("/proc/cpuinfo") as f:
                cpu = next(l.split(":", 1)[1].strip() for l in f if l.startswith("model name"))
        except (OSError, StopIteration):
            pass
        out["cpu_baseline"] = {"value": N * ksteps / el, "unit": "zone-updates/s",
                               "cores": oracle.threads(), "kind": "oracle",
                               "sample": f"{ksteps} steps (CFL dt + step) of the {n}^3 blast from "
                                         f"its initial state, {el:.1f} s, on {cpu}"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
