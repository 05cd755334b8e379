"""torch.autograd wrapper of RK4 time stepping with a checkpointed adjoint.

Forward: nsteps classical RK4 steps (the library's captured step graph),
keeping the state every `ckpt` steps; the steps of the last segment use the
library's stashing step instead, which leaves their stage states and primal
intermediates in device memory (~40 states per step for Navier-Stokes), so
that segment is never replayed.  Backward: segments from last to first;
each earlier segment is replayed forward from its checkpoint with the
stashing step, then the hand-written RK4 step adjoint consumes the stash step
by step in reverse with no recomputation.  Torch holds the tensors; all
arithmetic runs in the HIP library.
"""
from __future__ import annotations

import torch


class FRSteps(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u0, solver, dt, nsteps, ckpt):
        work = u0.detach().clone()
        ckpts = []
        L = solver.stash_len()
        # one segment's stash: stage states and primal intermediates of every
        # step, written by the stashing steps and read by the step adjoints
        stash = torch.empty(ckpt * L, dtype=torch.float64, device=work.device)
        last0 = ((nsteps - 1) // ckpt) * ckpt if nsteps > 0 else 0
        for n in range(nsteps):
            if n % ckpt == 0:
                ckpts.append(work.clone())
            if n >= last0:
                solver.step_stash(work, dt, stash[(n - last0) * L:(n - last0 + 1) * L])
            else:
                solver.step(work, dt, 1)
        ctx.solver, ctx.dt, ctx.nsteps, ctx.ckpt, ctx.ckpts = solver, dt, nsteps, ckpt, ckpts
        ctx.stash = stash
        return work

    @staticmethod
    def backward(ctx, lam_out):
        s, dt, ckpt = ctx.solver, ctx.dt, ctx.ckpt
        lam = lam_out.detach().contiguous().clone()
        work = torch.empty_like(lam)
        L = s.stash_len()
        stash = ctx.stash
        for seg in reversed(range(len(ctx.ckpts))):
            n0 = seg * ckpt
            n1 = min(ctx.nsteps, n0 + ckpt)
            if seg < len(ctx.ckpts) - 1:       # the last segment was stashed by forward
                work.copy_(ctx.ckpts[seg])
                for i in range(n1 - n0):
                    s.step_stash(work, dt, stash[i * L:(i + 1) * L])
            for i in reversed(range(n1 - n0)):
                s.rk_step_adjoint_stash(stash[i * L:(i + 1) * L], dt, lam, out=lam)
        ctx.stash = None
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
