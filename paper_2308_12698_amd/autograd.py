"""``torch.autograd.Function`` around the fused forward rollout (with
checkpoints) and the hand-written adjoint of libpotato.so.

Inputs that carry gradients: the initial state x0 [40, N] (rows 30-39 are
rounding carries; a carry row receives the cotangent of its row because the
represented value is row + carry) and per-agent gains [9, N].  The loss is
any torch expression of the returned final state; only the cotangent of the
30 physical rows enters the reverse sweep.
"""
from __future__ import annotations

import torch

from .sim import N_ROWS, Simulator


class Rollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x0, gains, sim: Simulator, wp, dt: float, n_steps: int, ckpt_every: int,
                resample_every: int = 0, step0: int = 0, type_idx=None, perm=None):
        if sim.mode != 1:
            raise ValueError("Rollout needs a closed-loop Simulator")
        n = x0.shape[1]
        x = x0.detach().clone().contiguous()
        slots = max(1, -(-int(n_steps) // int(ckpt_every)))
        ckpt = torch.empty((slots, N_ROWS, n), dtype=torch.float32, device=x0.device)
        g = None if gains is None else gains.detach().contiguous()
        sim.step(x, n_steps, dt, gains=g, wp=wp, resample_every=resample_every, step0=step0,
                 type_idx=type_idx, perm=perm, ckpt=ckpt, ckpt_every=ckpt_every)
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
        gfin = grad_out[:30].contiguous()
        gx0, gg = ctx.sim.step_backward(ckpt, ctx.K, ctx.n_steps, ctx.dt, gfin, gains=g, wp=wp,
                                        resample_every=ctx.resample_every, step0=ctx.step0,
                                        type_idx=ctx.type_idx, perm=ctx.perm,
                                        want_gains=ctx.needs_input_grad[1])
        full = torch.empty((N_ROWS, gx0.shape[1]), dtype=gx0.dtype, device=gx0.device)
        full[:30] = gx0
        full[30:33] = gx0[0:3]
        full[33:36] = gx0[3:6]
        full[36] = gx0[29]
        full[37:40] = gx0[17:20]
        return (full, gg if ctx.needs_input_grad[1] else None, None, None, None, None, None, None,
                None, None, None)


def rollout(x0, gains, sim, wp, dt, n_steps, ckpt_every, resample_every=0, step0=0,
            type_idx=None, perm=None):
    """Differentiable closed-loop rollout: returns the final state [40, N]."""
    return Rollout.apply(x0, gains, sim, wp, dt, n_steps, ckpt_every, resample_every, step0,
                         type_idx, perm)
