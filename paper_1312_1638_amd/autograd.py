"""torch.autograd wrapper of RK4 time stepping with a checkpointed adjoint.

Forward: nsteps classical RK4 steps in segments of `ckpt` steps.  The last
segments, as many as fit in a device-memory budget (at least one), run with
the library's stashing step, which leaves every step's stage states and
primal intermediates in device memory (~40 states per step for
Navier-Stokes); the earlier segments run the captured step graph and keep
only their starting state (a checkpoint every `ckpt` steps).  Backward:
segments from last to first; a segment without a stash is replayed from its
checkpoint with the stashing step (into a reused buffer) and its adjoint run
at once, both as one captured graph in the library (fr_rk_segment_adjoint);
a resident stash is consumed by the hand-written RK4 step adjoint step by
step in reverse.  Neither recomputes anything inside a step.  The budget
defaults to the free device memory less a reserve, so on a 288 GB device
most segments are never replayed; budget 0 replays every segment but the
last.  Torch holds the tensors; all arithmetic
runs in the HIP library.
"""
from __future__ import annotations

import torch


class FRSteps(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u0, solver, dt, nsteps, ckpt, budget):
        # the solver's own state buffer: the step graph captured for it on
        # an earlier call is reused (a new address would be captured again)
        work = solver.graph_state()
        work.copy_(u0.detach())
        L = solver.stash_len()
        nseg = -(-nsteps // ckpt) if nsteps > 0 else 0
        resident = min(nseg, max(1, int(stash_segments(L, ckpt, budget, work.device))))
        first = nseg - resident            # segments first.. keep their stash
        ckpts, stashes = {}, {}
        for seg in range(nseg):
            steps = min(ckpt, nsteps - seg * ckpt)
            if seg < first:
                # checkpoint, then the whole segment through the step graph
                ckpts[seg] = work.clone()
                solver.step(work, dt, steps)
                continue
            # a stash of stage states and primal intermediates per step,
            # written here and read by the step adjoints
            stashes[seg] = torch.empty(steps * L, dtype=torch.float64, device=work.device)
            for i in range(steps):
                solver.step_stash(work, dt, stashes[seg][i * L:(i + 1) * L])
        ctx.solver, ctx.dt, ctx.nsteps, ctx.ckpt = solver, dt, nsteps, ckpt
        ctx.ckpts, ctx.stashes, ctx.nseg = ckpts, stashes, nseg
        return work.clone()

    @staticmethod
    def backward(ctx, lam_out):
        s, dt, ckpt = ctx.solver, ctx.dt, ctx.ckpt
        # the cotangent and the replay start live in solver-owned buffers, so
        # that the library's captured segment graphs see the same addresses
        # on every segment and every call
        lam = s.adjoint_state()
        lam.copy_(lam_out.detach())
        start = s.graph_state()
        L = s.stash_len()
        spare = None                         # replay buffer: a consumed full-length stash
        for seg in reversed(range(ctx.nseg)):
            n0 = seg * ckpt
            n1 = min(ctx.nsteps, n0 + ckpt)
            if seg in ctx.stashes:
                stash = ctx.stashes.pop(seg)
                for i in reversed(range(n1 - n0)):
                    s.rk_step_adjoint_stash(stash[i * L:(i + 1) * L], dt, lam, out=lam)
            else:
                # replay from the checkpoint and run the segment's adjoint,
                # one graph in the library
                if spare is None:
                    spare = torch.empty(ckpt * L, dtype=torch.float64, device=lam.device)
                stash = spare
                start.copy_(ctx.ckpts.pop(seg))
                s.segment_adjoint(start, dt, n1 - n0, lam, stash, out=lam)
            if spare is None and stash.numel() == ckpt * L:
                spare = stash
        ctx.stashes, ctx.ckpts = None, None
        return lam.clone(), None, None, None, None, None


# Device memory left free when the stash budget is taken from what is free.
RESERVE_FRACTION, RESERVE_MIN = 0.1, 8 << 30


def stash_segments(L, ckpt, budget, device):
    """Segments of `ckpt` steps whose stash (L float64 per step) fits in
    `budget` bytes; budget None: the free device memory, counting what
    torch's allocator holds unused, less a reserve (the larger of 10% of
    the device and 8 GiB)."""
    if budget is None:
        free, total = torch.cuda.mem_get_info(device)
        cached = torch.cuda.memory_reserved(device) - torch.cuda.memory_allocated(device)
        budget = max(0, free + cached - max(RESERVE_FRACTION * total, RESERVE_MIN))
    return budget // (ckpt * L * 8)


def integrate_steps(solver, u0, dt, nsteps, ckpt=20, stash_budget=None):
    """u(nsteps) as a differentiable function of u0.  stash_budget: bytes of
    device memory the forward pass may keep for stashed segments (None: the
    free memory less a reserve; 0: only the last segment)."""
    return FRSteps.apply(u0, solver, dt, nsteps, ckpt, stash_budget)


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
