"""torch.autograd.Function around the differentiable lattice rollout.

LBRollout.apply(n0, g, params, nsteps, checkpoint_every) runs `nsteps`
fluctuating LB steps on the GPU from the pre-collision populations n0
([19, nz, ny, nx], float64 or float32) with uniform body force g (tensor of
3) and returns n(T).  Its backward calls lb_backward: reverse streaming and
the transposed moment-space collision with the noise replayed from its
Philox counters, segment by segment from checkpoints taken every
`checkpoint_every` steps.  Gradients flow to n0 and g.
"""
from __future__ import annotations

import dataclasses

import torch

from .lattice import FluidParams, Lattice


class LBRollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, n0: torch.Tensor, g: torch.Tensor, params: FluidParams, nsteps: int, checkpoint_every: int):
        gv = tuple(float(v) for v in g.detach().cpu().reshape(3))
        p = dataclasses.replace(params, body_force=gv, track_totals=False)
        lat = Lattice(p)
        lat.set_populations(n0.detach())
        lat.tape_begin(checkpoint_every)
        lat.step(nsteps)
        nT = lat.get_populations(dtype=n0.dtype)
        ctx.lat = lat
        ctx.g_dtype = g.dtype
        ctx.g_device = g.device
        return nT

    @staticmethod
    def backward(ctx, dnT: torch.Tensor):
        lat = ctx.lat
        dn0, dg = lat.backward(dnT.contiguous())
        lat.close()
        ctx.lat = None
        return dn0, torch.tensor(dg, dtype=ctx.g_dtype, device=ctx.g_device), None, None, None


def rollout(n0: torch.Tensor, g: torch.Tensor, params: FluidParams, nsteps: int, checkpoint_every: int = 50):
    return LBRollout.apply(n0, g, params, nsteps, checkpoint_every)
