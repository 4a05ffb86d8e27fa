"""``torch.autograd.Function`` around the fused forward rollout (with
checkpoints) and the hand-written adjoint of libpotato.so.

Inputs that carry gradients: the initial state x0 [30, N] and per-agent
gains [9, N].  The forward keeps the rounding carries of its integrator in
a buffer of its own (zeros at the start: x0 is taken as exact), because the
reverse sweep replays that compensated integrator from the checkpoints.
The loss is any torch expression of the returned final state [30, N].
"""
from __future__ import annotations

import torch

from .sim import N_CARRY, N_CKPT, Simulator


class Rollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x0, gains, sim: Simulator, wp, dt: float, n_steps: int, ckpt_every: int,
                resample_every: int = 0, step0: int = 0, type_idx=None, perm=None):
        if sim.mode != 1:
            raise ValueError("Rollout needs a closed-loop Simulator")
        n = x0.shape[1]
        x = x0.detach().clone().contiguous()
        carry = torch.zeros((N_CARRY, n), dtype=torch.float32, device=x0.device)
        slots = max(1, -(-int(n_steps) // int(ckpt_every)))
        ckpt = torch.empty((slots, N_CKPT, n), dtype=torch.float32, device=x0.device)
        g = None if gains is None else gains.detach().contiguous()
        sim.step(x, n_steps, dt, gains=g, wp=wp, resample_every=resample_every, step0=step0,
                 type_idx=type_idx, perm=perm, ckpt=ckpt, ckpt_every=ckpt_every, carry=carry)
        ctx.save_for_backward(ckpt, g if g is not None else torch.empty(0, device=x0.device), wp)
        ctx.has_gains = g is not None
        ctx.sim, ctx.dt, ctx.n_steps, ctx.K = sim, dt, n_steps, ckpt_every
        ctx.resample_every, ctx.step0 = resample_every, step0
        ctx.type_idx, ctx.perm = type_idx, perm
        return x

    @staticmethod
    def backward(ctx, grad_out):
        ckpt, g, wp = ctx.saved_tensors
        g = g if ctx.has_gains else None
        gfin = grad_out.contiguous()
        gx0, gg = ctx.sim.step_backward(ckpt, ctx.K, ctx.n_steps, ctx.dt, gfin, gains=g, wp=wp,
                                        resample_every=ctx.resample_every, step0=ctx.step0,
                                        type_idx=ctx.type_idx, perm=ctx.perm,
                                        want_gains=ctx.needs_input_grad[1])
        return (gx0, gg if ctx.needs_input_grad[1] else None, None, None, None, None, None, None,
                None, None, None)


def rollout(x0, gains, sim, wp, dt, n_steps, ckpt_every, resample_every=0, step0=0,
            type_idx=None, perm=None):
    """Differentiable closed-loop rollout: returns the final state [30, N]."""
    return Rollout.apply(x0, gains, sim, wp, dt, n_steps, ckpt_every, resample_every, step0,
                         type_idx, perm)
