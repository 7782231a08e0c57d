"""Differentiable HGKS steps: torch.autograd.Function wrappers around hgks_step
and its hand-written adjoint hgks_step_vjp, with checkpoint-and-recompute.

Time steps are frozen: the forward pass takes a given dt per step (record the
CFL sequence of an undifferentiated run first), because the CFL maximum is not
differentiable.  Every step, forward and reverse, runs in the library's HIP
kernels; torch only holds the states and the autograd graph.
"""
from __future__ import annotations

import torch

from . import hgks


class Stepper:
    """A solver bound to a private work state, so that any state tensor can be
    stepped or differentiated without touching the caller's tensors."""

    def __init__(self, params: dict, like: torch.Tensor):
        # the library takes its reference state (for the deviation-form flux
        # arithmetic) from cell 0 of the state bound at init: bind a copy of a
        # representative state
        self.work = like.detach().clone().contiguous()
        self.solver = hgks.Solver(params, self.work)

    def step(self, q: torch.Tensor, dt: float) -> torch.Tensor:
        self.work.copy_(q)
        self.solver.step(1, dt=float(dt))
        return self.work.clone()

    def vjp(self, q: torch.Tensor, dt: float, lam: torch.Tensor) -> torch.Tensor:
        return self.solver.step_vjp(q.contiguous(), float(dt), lam.contiguous())


class HGKSStep(torch.autograd.Function):
    """q_next = step(q) with frozen dt; backward via hgks_step_vjp."""

    @staticmethod
    def forward(ctx, q: torch.Tensor, dt: float, stepper: Stepper):
        ctx.save_for_backward(q)
        ctx.dt = float(dt)
        ctx.stepper = stepper
        return stepper.step(q.detach(), dt)

    @staticmethod
    def backward(ctx, grad):
        (q,) = ctx.saved_tensors
        return ctx.stepper.vjp(q, ctx.dt, grad), None, None


class HGKSSegment(torch.autograd.Function):
    """Several frozen-dt steps as one autograd node that stores only its input
    state (a checkpoint); backward recomputes the intermediate states and runs
    the step adjoints in reverse."""

    @staticmethod
    def forward(ctx, q: torch.Tensor, dts, stepper: Stepper):
        ctx.save_for_backward(q)
        ctx.dts = [float(d) for d in dts]
        ctx.stepper = stepper
        x = q.detach()
        for dt in ctx.dts:
            x = stepper.step(x, dt)
        return x

    @staticmethod
    def backward(ctx, grad):
        (q,) = ctx.saved_tensors
        st = ctx.stepper
        states = [q.detach()]
        for dt in ctx.dts[:-1]:
            states.append(st.step(states[-1], dt))
        lam = grad.contiguous()
        for x, dt in zip(reversed(states), reversed(ctx.dts)):
            lam = st.vjp(x, dt, lam)
        return lam, None, None


def run_checkpointed(stepper: Stepper, q0: torch.Tensor, dts, every: int = 10) -> torch.Tensor:
    """Differentiable run over the given time steps with a checkpoint every
    `every` steps (memory: one state per segment plus one segment's states)."""
    q = q0
    dts = [float(d) for d in dts]
    for i in range(0, len(dts), every):
        q = HGKSSegment.apply(q, dts[i:i + every], stepper)
    return q


def cfl_time_steps(params: dict, q0: torch.Tensor, nsteps: int) -> list:
    """CFL time steps of an undifferentiated run from q0 (used to freeze dt)."""
    work = q0.detach().clone()
    s = hgks.Solver(params, work)
    dts = s.step(nsteps, return_dt=True)
    s.close()
    return dts
