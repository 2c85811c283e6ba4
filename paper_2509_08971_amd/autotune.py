"""Autotuner for the batched step's tile shape.

Times hard_hydro_step_batched on the caller's own set of grids for each
candidate x-y tile shape of the 2D/3D batched kernels and writes the fastest
to a tune-cache text file that hard_batch_plan_create reads
(lines "tile2d_f32 = 32x8" / "tile2d_f64 = 16x16").  Every candidate gives
bitwise identical results (the face arithmetic does not depend on the tile),
so the choice only affects speed.
"""
import os
import tempfile

import torch

from . import (batch_pack, hard_batch_offsets, hard_batch_plan_create, hard_batch_plan_destroy,
               hard_batch_workspace_bytes, hard_cfl_dt_batched, hard_hydro_step_batched, workspace)

CANDIDATES = ("16x16", "32x8", "8x32")


def _key(dtype):
    return "tile2d_f64" if dtype == torch.float64 else "tile2d_f32"


def tune_batched(grids, states, dtype=torch.float32, steps=5, cache_path=None, cfl=0.4,
                 candidates=CANDIDATES, device="cuda"):
    """Returns (best, {shape: ms_per_step}) and writes `cache_path` if given."""
    times = {}
    key = _key(dtype)
    for cand in candidates:
        fd, path = tempfile.mkstemp(suffix=".tune")
        with os.fdopen(fd, "w") as f:
            f.write(f"{key} = {cand}\n")
        plan = hard_batch_plan_create(grids, path)
        os.unlink(path)
        try:
            offs = hard_batch_offsets(plan, len(grids))
            U = batch_pack(states, offs, dtype, device)
            work = workspace(hard_batch_workspace_bytes(plan), device)
            dt = torch.zeros(len(grids), dtype=torch.float64, device=device)
            hard_cfl_dt_batched(plan, U, cfl, dt, work)
            hard_hydro_step_batched(plan, U, dt, work, cfl=cfl)  # warm-up
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            a.record()
            for _ in range(steps):
                hard_hydro_step_batched(plan, U, dt, work, cfl=cfl)
            b.record()
            torch.cuda.synchronize()
            times[cand] = a.elapsed_time(b) / steps
        finally:
            hard_batch_plan_destroy(plan)
    best = min(times, key=times.get)
    if cache_path:
        lines = []
        if os.path.exists(cache_path):
            with open(cache_path) as f:
                lines = [l for l in f if not l.startswith(key)]
        lines.append(f"{key} = {best}\n")
        with open(cache_path, "w") as f:
            f.writelines(lines)
    return best, times
