"""torch.autograd.Function around the differentiable lattice rollout.

LBRollout.apply(n0, g, params, nsteps, checkpoint_every) runs `nsteps`
fluctuating LB steps on the GPU from the pre-collision populations n0
([19, nz, ny, nx], float64 or float32) with uniform body force g (tensor of
3) and returns n(T).  Its backward calls lb_backward: reverse streaming and
the transposed moment-space collision with the noise replayed from its
Philox counters, segment by segment from checkpoints taken every
`checkpoint_every` steps (0: a moments tape, every step's density and
momentum kept and nothing recomputed).  Gradients flow to n0 and g.

LBCoupledRollout.apply(n0, g, pos0, mom0, beads, params, nsteps,
checkpoint_every) runs `nsteps` coupled steps (particle half, then the LB
step with the spread bead force) and returns (n(T), R(T), P(T)); its backward
calls lb_backward_coupled, so gradients flow to n0, g and the initial bead
positions and momenta.  `beads` supplies mass, friction and bonds (its
positions and momenta are not used).
"""
from __future__ import annotations

import dataclasses

import torch

from .lattice import DeviceBeads, FluidParams, Lattice


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


class LBCoupledRollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, n0: torch.Tensor, g: torch.Tensor, pos0: torch.Tensor, mom0: torch.Tensor, beads: DeviceBeads,
                params: FluidParams, nsteps: int, checkpoint_every: int):
        gv = tuple(float(v) for v in g.detach().cpu().reshape(3))
        p = dataclasses.replace(params, body_force=gv, track_totals=False)
        lat = Lattice(p)
        lat.set_populations(n0.detach())
        b = DeviceBeads(pos0.detach(), mom0.detach(), beads.mass, beads.zeta, beads.bonds, beads.k_bond, beads.r0,
                        device=n0.device, stencil=beads.stencil, fext=beads.fext, bond=beads.bond,
                        wca_epsilon=beads.wca_epsilon, wca_sigma=beads.wca_sigma, noise=beads.noise)
        lat.tape_begin(checkpoint_every)
        for _ in range(nsteps):
            lat.coupled_step(b)
        nT = lat.get_populations(dtype=n0.dtype)
        ctx.lat, ctx.beads = lat, b
        ctx.g_dtype, ctx.g_device = g.dtype, g.device
        ctx.pos_dtype, ctx.mom_dtype = pos0.dtype, mom0.dtype
        return nT, b.pos.clone().to(pos0.dtype), b.mom.clone().to(mom0.dtype)

    @staticmethod
    def backward(ctx, dnT: torch.Tensor, dRT: torch.Tensor, dPT: torch.Tensor):
        lat = ctx.lat
        dn0, dg, dR0, dP0 = lat.backward_coupled(dnT.contiguous(), dRT, dPT)
        lat.close()
        ctx.lat = ctx.beads = None
        return (dn0, torch.tensor(dg, dtype=ctx.g_dtype, device=ctx.g_device), dR0.to(ctx.pos_dtype),
                dP0.to(ctx.mom_dtype), None, None, None, None)


def coupled_rollout(n0: torch.Tensor, g: torch.Tensor, pos0: torch.Tensor, mom0: torch.Tensor, beads: DeviceBeads,
                    params: FluidParams, nsteps: int, checkpoint_every: int = 50):
    return LBCoupledRollout.apply(n0, g, pos0, mom0, beads, params, nsteps, checkpoint_every)


_C = [[0, 0, 0], [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1], [1, 1, 0], [-1, -1, 0],
      [1, -1, 0], [-1, 1, 0], [1, 0, 1], [-1, 0, -1], [1, 0, -1], [-1, 0, 1], [0, 1, 1], [0, -1, -1], [0, 1, -1],
      [0, -1, 1]]


def velocity_field(nT: torch.Tensor, g: torch.Tensor):
    """(rho, u) of full populations [19, nz, ny, nx]: u = (sum n c + g/2)/rho
    (eq. special_choice_momentum_density)."""
    c = torch.tensor(_C, dtype=nT.dtype, device=nT.device)
    rho = nT.sum(0)
    J = (c.t() @ nT.reshape(19, -1)).reshape((3,) + nT.shape[1:]) + 0.5 * g.to(nT.dtype).reshape(3, 1, 1, 1)
    return rho, J / rho


def interpolate(u: torch.Tensor, pos: torch.Tensor):
    """Trilinear (two-point kernel per axis, eq. Delta) interpolation of a
    periodic vector field u [3, nz, ny, nx] at positions pos [n, 3] (x, y, z);
    differentiable in u and pos."""
    nz, ny, nx = u.shape[1:]
    base = torch.floor(pos)
    frac = pos - base
    b = base.long()
    out = torch.zeros((pos.shape[0], 3), dtype=u.dtype, device=u.device)
    for dz in (0, 1):
        for dy in (0, 1):
            for dx in (0, 1):
                w = ((frac[:, 0] if dx else 1 - frac[:, 0]) * (frac[:, 1] if dy else 1 - frac[:, 1]) *
                     (frac[:, 2] if dz else 1 - frac[:, 2]))
                x = (b[:, 0] + dx) % nx
                y = (b[:, 1] + dy) % ny
                z = (b[:, 2] + dz) % nz
                out = out + w[:, None] * u[:, z, y, x].t()
    return out


def probe_drag_loss(nT: torch.Tensor, g: torch.Tensor, posT: torch.Tensor, momT: torch.Tensor, mass: torch.Tensor,
                    zeta: torch.Tensor, lo: int, hi: int):
    """Loss of the differentiation workload: mean abs(u)^2 over the probe
    cube [lo, hi)^3 plus the mean squared bead drag abs(zeta (V - u(R)))^2,
    V = P/m, all at the final step."""
    rho, u = velocity_field(nT, g)
    probe = (u[:, lo:hi, lo:hi, lo:hi] ** 2).sum(0).mean()
    ub = interpolate(u, posT)
    drag = zeta.to(u.dtype)[:, None] * (momT / mass.to(u.dtype)[:, None] - ub)
    return probe + (drag ** 2).sum(1).mean()

