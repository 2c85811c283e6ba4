"""Gradient of a final-time loss with respect to the initial state.

HydroRollout.apply(U0, grid, nsteps, cfl, every) runs `nsteps` Heun steps
with the CFL step of each state (the step sizes are recorded and then held
fixed: the time-step selection is not differentiated), keeping the state
every `every` steps.  Its backward pass walks the segments in reverse:
it recomputes the states of one segment from its checkpoint with the
recorded step sizes (keeping each step's stage-1 state), then applies the
adjoint of each step, last step first, with that stage-1 state
(hard_hydro_step_adjoint_given_u1; the segment's last step, whose stage 1
was not recomputed, through hard_hydro_step_adjoint).  Every state update
and every vector-Jacobian product runs in libhard's kernels; this module
only sequences the calls and keeps the checkpoints.
"""
import torch

from . import (hard_adjoint_workspace_bytes, hard_cfl_dt, hard_hydro_stage, hard_hydro_step,
               hard_hydro_step_adjoint, hard_hydro_step_adjoint_given_u1, hard_workspace_bytes,
               workspace)


class HydroRollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U0, grid, nsteps, cfl=0.4, every=20):
        U = U0.detach().clone().contiguous()
        dev = U.device
        work = workspace(hard_workspace_bytes(grid), dev)
        # dts[n] is the step buffer of step n; the fused CFL of step n writes
        # dts[n + 1] directly (the last one goes to a spare slot)
        dts_buf = torch.zeros(nsteps + 1, dtype=torch.float64, device=dev)
        hard_cfl_dt(grid, U, cfl, dts_buf[0:1], work)
        ckpts = []
        for n in range(nsteps):
            if n % every == 0:
                ckpts.append(U.clone())
            hard_hydro_step(grid, U, dts_buf[n:n + 1], work, cfl=cfl,
                            next_dt_dev=dts_buf[n + 1:n + 2])
        dts = dts_buf[:nsteps]
        ctx.grid = grid
        ctx.nsteps = nsteps
        ctx.every = every
        ctx.save_for_backward(dts, *ckpts)
        return U

    @staticmethod
    def backward(ctx, lam_out):
        dts, *ckpts = ctx.saved_tensors
        grid, nsteps, every = ctx.grid, ctx.nsteps, ctx.every
        lam = lam_out.detach().clone().contiguous()
        dev = lam.device
        work = workspace(hard_workspace_bytes(grid), dev)
        awork = workspace(hard_adjoint_workspace_bytes(grid), dev)
        for seg in reversed(range(len(ckpts))):
            start = seg * every
            end = min(start + every, nsteps)
            states = [ckpts[seg]]
            stage1 = []
            for n in range(start, end - 1):
                # recompute the segment's states, keeping each step's stage-1
                # state for its adjoint (stage 2 writes the new state directly)
                U1 = torch.empty_like(lam)
                U = torch.empty_like(lam)
                hard_hydro_stage(grid, 1, states[-1], None, U1, dts[n:n + 1], work)
                hard_hydro_stage(grid, 2, U1, states[-1], U, dts[n:n + 1], work)
                stage1.append(U1)
                states.append(U)
            for n in reversed(range(start, end)):
                k = n - start
                if k < len(stage1):
                    hard_hydro_step_adjoint_given_u1(grid, states[k], stage1[k], dts[n:n + 1], lam,
                                                     awork)
                else:  # the segment's last step: its stage 1 was not recomputed
                    hard_hydro_step_adjoint(grid, states[k], dts[n:n + 1], lam, awork)
            del states, stage1
        return lam, None, None, None, None


def rollout(U0, grid, nsteps, cfl=0.4, every=20):
    """Differentiable nsteps-step run (see HydroRollout)."""
    return HydroRollout.apply(U0, grid, nsteps, cfl, every)


def recorded_dts(U0, grid, nsteps, cfl=0.4):
    """The step sizes a rollout from U0 uses (device tensor of nsteps)."""
    U = U0.detach().clone().contiguous()
    work = workspace(hard_workspace_bytes(grid), U.device)
    dts = torch.zeros(nsteps + 1, dtype=torch.float64, device=U.device)
    hard_cfl_dt(grid, U, cfl, dts[0:1], work)
    for n in range(nsteps):
        hard_hydro_step(grid, U, dts[n:n + 1], work, cfl=cfl, next_dt_dev=dts[n + 1:n + 2])
    return dts[:nsteps], U


def run_fixed(U0, grid, dts):
    """Steps of the given (device) dt list from U0; returns the final state."""
    U = U0.detach().clone().contiguous()
    work = workspace(hard_workspace_bytes(grid), U.device)
    for n in range(dts.numel()):
        hard_hydro_step(grid, U, dts[n:n + 1], work)
    return U
