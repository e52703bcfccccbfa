"""Reverse-mode differentiation through the solver (Sec. 3.4) with checkpointed unrolls.

``step(solver, u, dt)`` is a ``torch.autograd.Function`` whose backward is the
library's hand-written RK4-step pullback (``ins_step_rk4_vjp``); torch only
chains the steps. ``rollout_loss`` unrolls many steps and keeps only every
``checkpoint_every``-th state: the backward recomputes each segment from its
first state, so memory grows with (steps / k + k) fields instead of with the
number of steps (the paper's outlook, Sec. 8.2, names checkpointing as the
remedy for storing every state).
"""
from __future__ import annotations

import torch
import torch.utils.checkpoint as _ckpt


def _forward_step(ctx, u0, solver, dt, scheme, keep_stages):
    ctx.solver = solver
    ctx.dt = float(dt)
    ctx.scheme = scheme
    ctx.keep = bool(keep_stages)
    u0 = u0.contiguous()
    if ctx.keep:
        # keep the stage inputs (the paper's store-the-sub-steps strategy) instead of recomputing them
        stages, pstages = solver.stage_buffers(scheme)
        u1 = solver.step(u0, dt, scheme=scheme, keep=(stages, pstages))
        ctx.save_for_backward(u0, stages, pstages)
    else:
        u1 = solver.step(u0, dt, scheme=scheme)
        ctx.save_for_backward(u0)
    return u1


def _backward_step(ctx, u1bar):
    if ctx.keep:
        u0, stages, pstages = ctx.saved_tensors
        kept = (stages, pstages)
    else:
        (u0,) = ctx.saved_tensors
        kept = None
    return ctx.solver.step_vjp(u0, u1bar.contiguous(), ctx.dt, scheme=ctx.scheme, kept=kept)


class _Step(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u0, solver, dt, scheme, keep_stages):
        return _forward_step(ctx, u0, solver, dt, scheme, keep_stages)

    @staticmethod
    def backward(ctx, u1bar):
        return _backward_step(ctx, u1bar), None, None, None, None


class _Rhs(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u, solver):
        ctx.solver = solver
        ctx.save_for_backward(u)
        return solver.rhs(u.contiguous())

    @staticmethod
    def backward(ctx, fbar):
        (u,) = ctx.saved_tensors
        return ctx.solver.rhs_vjp(u.contiguous(), fbar.contiguous()), None


class _Project(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u, solver):
        ctx.solver = solver
        return solver.project(u.contiguous())

    @staticmethod
    def backward(ctx, ubar):
        return ctx.solver.project_vjp(ubar.contiguous()), None


class _StepClosure(torch.autograd.Function):
    """RK4 step with the closure; theta (the parameters the solver's closure was
    set from) is an input so that autograd routes its gradient."""

    @staticmethod
    def forward(ctx, u0, theta, solver, dt, scheme, keep_stages):
        return _forward_step(ctx, u0, solver, dt, scheme, keep_stages)

    @staticmethod
    def backward(ctx, u1bar):
        ctx.solver.closure_grad()  # start from an empty accumulator
        g = _backward_step(ctx, u1bar)
        return g, ctx.solver.closure_grad(), None, None, None, None


def step(solver, u, dt, theta=None, scheme="rk4", keep_stages=False):
    """One differentiable time step (RK4, or "wray3"; with the closure when theta is given).
    keep_stages stores the stage inputs for the backward pass instead of recomputing them
    (scheme-dependent 2-3 velocity and pressure fields per step, about a fifth less work)."""
    if theta is not None:
        return _StepClosure.apply(u, theta, solver, dt, scheme, keep_stages)
    return _Step.apply(u, solver, dt, scheme, keep_stages)


def rhs(solver, u):
    """Differentiable right-hand side F(u)."""
    return _Rhs.apply(u, solver)


def project(solver, u):
    """Differentiable projection P u."""
    return _Project.apply(u, solver)


def rollout(solver, u0, dt, nsteps, scheme="rk4"):
    """States u_1..u_n (every state kept by autograd; use rollout_loss for long unrolls)."""
    out = []
    u = u0
    for _ in range(nsteps):
        u = step(solver, u, dt, scheme=scheme)
        out.append(u)
    return out


def rollout_loss(solver, u0, dt, refs, checkpoint_every=10, per_step_loss=None, theta=None, scheme="rk4",
                 keep_stages=False):
    """Sum over s = 1..len(refs) of per_step_loss(u_s, refs[s-1]), differentiable in u0.

    Default per-step loss: mean over cells and components of (u_s - ref_s)^2,
    divided by the number of steps (so the total is the trajectory MSE).
    Only the state at the start of every segment of ``checkpoint_every`` steps
    is kept; each segment is recomputed in the backward pass. With ``theta``
    (the closure parameters the solver was set with) the loss is also
    differentiable in theta.
    """
    nsteps = len(refs)
    if per_step_loss is None:

        def per_step_loss(u, r):
            return ((u - r) ** 2).mean() / nsteps

    def segment(u, s0, s1):
        total = u.new_zeros(())
        for s in range(s0, s1):
            u = step(solver, u, dt, theta, scheme, keep_stages)
            total = total + per_step_loss(u, refs[s])
        return u, total

    k = max(1, int(checkpoint_every))
    u = u0
    loss = u0.new_zeros(())
    for s0 in range(0, nsteps, k):
        s1 = min(s0 + k, nsteps)
        u, seg = _ckpt.checkpoint(segment, u, s0, s1, use_reentrant=False)
        loss = loss + seg
    return loss
