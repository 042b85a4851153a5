"""Differentiable fixed-step TVD-RK3 rollouts (the paper's fixed-dt,
differentiable `feed_forward` rollout, §4.5) backed by the hand-written
discrete adjoint of libcfd.

RK3Rollout.apply(U0, solver, dt, n_steps, ckpt_every, keep_stages) returns
U_N; its backward pass walks the rollout in reverse segment by segment: the
segment's states are recomputed from its checkpoint (kept every `ckpt_every`
steps in the forward pass), then the step adjoint maps the adjoint back one
step at a time. With keep_stages (the default) the recompute keeps the
primitives of each step's three stage inputs (cfd_rk3_step_prims) and
cfd_rk3_step_adjoint_prims uses them; otherwise cfd_rk3_step_adjoint
recomputes the stages in every step adjoint. Memory: the checkpoints plus one
segment of states (with keep_stages, 18 components per padded cell and step
instead of 5). Gradients flow to the interior cells of U0; halo entries of the
returned gradient are zero.
"""
from __future__ import annotations

import torch

from .solver import Solver, interior


class RK3Rollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U0, solver: Solver, dt: float, n_steps: int, ckpt_every: int = 20,
                keep_stages: bool = True):
        if n_steps < 0 or ckpt_every < 1:
            raise ValueError("need n_steps >= 0 and ckpt_every >= 1")
        U = U0.detach().clone().contiguous()
        solver.fill_halo(U)
        ckpts = []
        done = 0
        while done < n_steps:
            ckpts.append((done, U.clone()))
            k = min(ckpt_every, n_steps - done)
            solver.advance_fixed(U, k, dt)
            done += k
        ctx.solver = solver
        ctx.dt = float(dt)
        ctx.n_steps = int(n_steps)
        ctx.ckpt_every = int(ckpt_every)
        ctx.ckpts = ckpts
        ctx.keep_stages = bool(keep_stages)
        return U

    @staticmethod
    def backward(ctx, Ubar):
        solver, dt = ctx.solver, ctx.dt
        Ub = torch.zeros_like(Ubar)
        interior(solver.case, Ub).copy_(interior(solver.case, Ubar))
        scratch = torch.empty_like(Ub)
        for start, ck in reversed(ctx.ckpts):
            k = min(ctx.ckpt_every, ctx.n_steps - start)
            U = ck.clone()
            if ctx.keep_stages:
                prims = []
                for i in range(k):
                    P = solver.empty_stage_prims()
                    solver.step_prims(U, dt, P)
                    prims.append(P)
                for s in reversed(range(k)):
                    solver.step_adjoint_prims(prims[s], dt, Ub, scratch)
                    Ub, scratch = scratch, Ub
                del prims
            else:
                states = [ck]
                for i in range(k - 1):
                    solver.advance_fixed(U, 1, dt)
                    states.append(U.clone())
                for s in reversed(range(k)):
                    solver.step_adjoint(states[s], dt, Ub, scratch)
                    Ub, scratch = scratch, Ub
                del states
        ctx.ckpts = None
        return Ub, None, None, None, None, None


def rollout(U0, solver: Solver, dt: float, n_steps: int, ckpt_every: int = 20, keep_stages: bool = True):
    return RK3Rollout.apply(U0, solver, dt, n_steps, ckpt_every, keep_stages)


class StateInit(torch.autograd.Function):
    """U = S(W): the padded conservative state (halos filled) of interior
    primitive point values W (5, nz, ny, nx), by cfd_state_init; the backward
    pass is cfd_state_init_adjoint (the transposed halo fill and primitive map)."""

    @staticmethod
    def forward(ctx, W, solver: Solver):
        W = W.detach().contiguous()
        U = solver.empty_state()
        solver.state_init(W, U)
        ctx.solver = solver
        ctx.save_for_backward(W)
        return U

    @staticmethod
    def backward(ctx, Ubar):
        (W,) = ctx.saved_tensors
        Wbar = torch.zeros_like(W)
        ctx.solver.state_init_adjoint(W, Ubar.contiguous(), Wbar)
        return Wbar, None


def state_init(solver: Solver, W):
    """Differentiable cfd_state_init: interior primitives W (5, nz, ny, nx) on
    the solver's device to the padded conservative state."""
    return StateInit.apply(W, solver)
