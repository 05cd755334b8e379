"""torch.autograd wrapper of RK4 time stepping with a checkpointed adjoint.

Forward: nsteps classical RK4 steps (the library's captured step graph),
keeping the state every `ckpt` steps.  Backward: segments from last to
first; each segment is replayed forward from its checkpoint (states kept in
device memory), then the hand-written RK4 step adjoint of the library is
applied step by step in reverse.  Torch holds the tensors; all arithmetic
runs in the HIP library.
"""
from __future__ import annotations

import torch


class FRSteps(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u0, solver, dt, nsteps, ckpt):
        work = u0.detach().clone()
        ckpts = []
        for n in range(nsteps):
            if n % ckpt == 0:
                ckpts.append(work.clone())
            solver.step(work, dt, 1)
        ctx.solver, ctx.dt, ctx.nsteps, ctx.ckpt, ctx.ckpts = solver, dt, nsteps, ckpt, ckpts
        return work

    @staticmethod
    def backward(ctx, lam_out):
        s, dt, ckpt = ctx.solver, ctx.dt, ctx.ckpt
        lam = lam_out.detach().contiguous().clone()
        work = torch.empty_like(lam)
        for seg in reversed(range(len(ctx.ckpts))):
            n0 = seg * ckpt
            n1 = min(ctx.nsteps, n0 + ckpt)
            states = [ctx.ckpts[seg]]
            work.copy_(ctx.ckpts[seg])
            for _ in range(n0, n1 - 1):
                s.step(work, dt, 1)
                states.append(work.clone())
            for u_n in reversed(states):
                s.rk_step_adjoint(u_n, dt, lam, out=lam)
        return lam, None, None, None, None


def integrate_steps(solver, u0, dt, nsteps, ckpt=20):
    """u(nsteps) as a differentiable function of u0."""
    return FRSteps.apply(u0, solver, dt, nsteps, ckpt)


class KineticEnergy(torch.autograd.Function):
    """Sum over problems of the kinetic-energy integral of the state."""

    @staticmethod
    def forward(ctx, u, solver):
        ctx.solver = solver
        ctx.save_for_backward(u)
        return solver.integrate(u)[:, -1].sum()

    @staticmethod
    def backward(ctx, g):
        (u,) = ctx.saved_tensors
        return ctx.solver.kinetic_energy_grad(u) * g, None
