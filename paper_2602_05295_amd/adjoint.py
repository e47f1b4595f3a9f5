"""Differentiable HOME-LBM rollouts: a torch.autograd.Function over the HIP
library's forward step (lbm_step) and its hand-written adjoint
(lbm_adjoint_step), with checkpointing.

forward:  m(0) = equilibrium(rho0, u0); a raw-state checkpoint every k steps;
          T steps; returns the final moment field (10, nz, ny, nx).
backward: for each checkpointed segment, last first: recompute the
          segment's states from its checkpoint (lbm_step_into, each written
          to its own tensor), run the adjoint steps backwards through them;
          finally map lam(0) through the equilibrium initialisation to d/du0
          and d/drho0.
Memory: T/k checkpoints plus k states, each 40 B per cell.
All arithmetic runs in the library; torch provides device memory and the stream.
"""
from __future__ import annotations

import torch

from .homelbm import FP32, HomeLBM


class _Rollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u0, rho0, sim, nsteps, every):
        if sim.fmt != FP32:
            raise ValueError("gradients need an FP32 context")
        u0 = u0.detach().contiguous()
        rho0 = rho0.detach().contiguous()
        sim.set_stream(torch.cuda.current_stream().cuda_stream)
        sim.set_equilibrium(rho0, u0)
        shape = (10,) + sim.dims[::-1]
        t0 = sim.step_count
        cps = []
        done = 0
        while done < nsteps:
            cp = torch.empty(shape, device=u0.device, dtype=torch.float32)
            sim.get_raw(cp)
            cps.append(cp)
            k = min(every, nsteps - done)
            sim.step(k)
            done += k
        out = torch.empty(shape, device=u0.device, dtype=torch.float32)
        sim.get_moments(out)
        ctx.sim, ctx.nsteps, ctx.every, ctx.t0 = sim, nsteps, every, t0
        ctx.cps = cps
        ctx.save_for_backward(u0, rho0)
        return out

    @staticmethod
    def backward(ctx, g_out):
        u0, rho0 = ctx.saved_tensors
        sim, nsteps, every = ctx.sim, ctx.nsteps, ctx.every
        lam = g_out.detach().contiguous().clone()
        spare = torch.empty_like(lam)
        nseg = len(ctx.cps)
        for s in range(nseg - 1, -1, -1):
            k = min(every, nsteps - s * every)
            # recompute the segment's states straight into their own tensors
            sim.step_count = ctx.t0 + s * every
            states = [ctx.cps[s]]
            for _ in range(k - 1):
                st = torch.empty_like(lam)
                sim.step_into(states[-1], st)
                states.append(st)
            for st in reversed(states):
                sim.adjoint_step(st, lam, spare)
                lam, spare = spare, lam
        g_u = torch.empty_like(u0)
        g_rho = torch.empty_like(rho0)
        sim.equilibrium_vjp(rho0, u0, lam, g_u, g_rho)
        sim.step_count = ctx.t0 + nsteps
        return g_u, g_rho, None, None, None


def rollout(sim: HomeLBM, u0: torch.Tensor, nsteps: int, every: int = 20, rho0: torch.Tensor | None = None):
    """Differentiable T-step rollout from the equilibrium of (rho0, u0).

    u0: (3, nz, ny, nx) float32 CUDA tensor; rho0 defaults to ones.  Returns
    the final moments (10, nz, ny, nx) (rho, j, P); gradients flow to u0 and
    rho0 through the library's adjoint step.
    """
    if rho0 is None:
        rho0 = torch.ones(u0.shape[1:], device=u0.device, dtype=torch.float32)
    return _Rollout.apply(u0, rho0, sim, int(nsteps), int(every))
