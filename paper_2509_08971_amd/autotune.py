"""Autotuner for the batched step's work-item shapes.

Times hard_hydro_step_batched on the caller's own set of grids for each
candidate setting and writes the fastest to a tune-cache text file that
hard_batch_plan_create reads, one "key = value" per line:

  walk2d = 64          rows per 2D work item
  tile3d_f64 = 16x16   x-y tile of 3D problems (tile3d_f32 for float)
  cz = 32              planes per 3D work item

The keys are tuned one after the other (coordinate search), each with the
best values found so far for the others.  Every setting gives bitwise
identical results (the face arithmetic does not depend on the work split),
so the choice only affects speed.
"""
import os
import tempfile

import torch

from . import (batch_pack, hard_batch_offsets, hard_batch_plan_create, hard_batch_plan_destroy,
               hard_batch_workspace_bytes, hard_cfl_dt_batched, hard_hydro_step_batched, workspace)

TILES_3D = ("16x16", "32x8", "8x32")


def default_candidates(dtype):
    k3 = "tile3d_f64" if dtype == torch.float64 else "tile3d_f32"
    return {"walk2d": ("32", "64", "128"), k3: TILES_3D, "cz": ("16", "32", "64")}


def _time_setting(grids, states, dtype, setting, steps, cfl, device):
    fd, path = tempfile.mkstemp(suffix=".tune")
    with os.fdopen(fd, "w") as f:
        f.writelines(f"{k} = {v}\n" for k, v in setting.items())
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
        return a.elapsed_time(b) / steps
    finally:
        hard_batch_plan_destroy(plan)


def tune_batched(grids, states, dtype=torch.float32, steps=5, cache_path=None, cfl=0.4,
                 candidates=None, device="cuda"):
    """Returns (best setting dict, {(key, value): ms_per_step}); writes `cache_path` if given."""
    candidates = candidates or default_candidates(dtype)
    best = {k: v[0] for k, v in candidates.items()}
    times = {}
    for key, values in candidates.items():
        for val in values:
            setting = dict(best, **{key: val})
            times[(key, val)] = _time_setting(grids, states, dtype, setting, steps, cfl, device)
        best[key] = min(values, key=lambda v: times[(key, v)])
    if cache_path:
        lines = []
        if os.path.exists(cache_path):
            with open(cache_path) as f:
                lines = [l for l in f if l.split("=")[0].strip() not in best]
        lines += [f"{k} = {v}\n" for k, v in best.items()]
        with open(cache_path, "w") as f:
            f.writelines(lines)
    return best, times
