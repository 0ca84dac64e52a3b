"""Python face of liblbmi: a periodic fluctuating D3Q19 box with point beads.

PyTorch supplies device memory (CUDA/HIP tensors) and the stream; every
numerical step is a HIP kernel behind the C ABI of include/lb.h.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

from . import _lib
from ._lib import LB_BF16, LB_F16, LB_F32, LB_F64, check

Q = 19
_STORAGE = {"f32": LB_F32, "bf16": LB_BF16, "f16": LB_F16, LB_F32: LB_F32, LB_BF16: LB_BF16, LB_F16: LB_F16}


def two_rate(gamma_e: float, magic: float = 3.0 / 16.0) -> dict:
    """Two-rate relaxation (Sec. "D3Q19 model II"): keyword arguments for
    FluidParams from lb_params_two_rate, which sets the even rate gamma_e on
    the bulk, shear and even kinetic modes and the odd rate on the odd
    kinetic modes so that the product of the two relaxation times equals
    `magic` (3/16: a stationary bounce-back wall exactly half way along the
    link for plane Poiseuille flow)."""
    p = _lib.lb_params()
    rc = _lib.load().lb_params_two_rate(float(gamma_e), float(magic), ctypes.byref(p))
    if rc != 0:
        raise ValueError(_lib.load().lb_last_error(None).decode())
    return dict(gamma_shear=p.gamma_shear, gamma_bulk=p.gamma_bulk, gamma_4a=p.gamma_4a, gamma_4b=p.gamma_4b,
                gamma_3a=p.gamma_3a, gamma_3b=p.gamma_3b)


@dataclass
class FluidParams:
    """Fluid parameters (lattice units).  nu = (1/6)(1+gamma_shear)/(1-gamma_shear)."""
    nx: int
    ny: int
    nz: int
    storage: str = "f32"
    rho0: float = 1.0
    gamma_shear: float = 0.0
    gamma_bulk: float = 0.0
    gamma_3a: float = 0.0
    gamma_3b: float = 0.0
    gamma_4a: float = 0.0
    gamma_4b: float = 0.0
    kT: float = 0.0
    body_force: tuple = (0.0, 0.0, 0.0)
    seed: int = 0
    noise_rho0: bool = False
    block: int = 0
    track_totals: bool = True
    box_id: int = 0
    vacf_lags: int = 0
    graph_steps: int = 0
    rounding: str = "nearest"   # "nearest" or "stochastic" (16-bit storage)
    walls: bool = False         # stationary walls at z = -1/2 and z = nz - 1/2

    @property
    def N(self) -> int:
        return self.nx * self.ny * self.nz

    def to_c(self) -> _lib.lb_params:
        p = _lib.lb_params()
        p.nx, p.ny, p.nz = self.nx, self.ny, self.nz
        p.storage = _STORAGE[self.storage]
        p.rho0 = self.rho0
        p.gamma_shear, p.gamma_bulk = self.gamma_shear, self.gamma_bulk
        p.gamma_3a, p.gamma_3b, p.gamma_4a, p.gamma_4b = self.gamma_3a, self.gamma_3b, self.gamma_4a, self.gamma_4b
        p.kT = self.kT
        for a in range(3):
            p.body_force[a] = float(self.body_force[a])
        p.seed = int(self.seed) & 0xFFFFFFFFFFFFFFFF
        p.noise_rho0 = 1 if self.noise_rho0 else 0
        p.block = int(self.block)
        p.track_totals = 1 if self.track_totals else 0
        p.box_id = int(self.box_id)
        p.vacf_lags = int(self.vacf_lags)
        p.graph_steps = int(self.graph_steps)
        p.rounding = {"nearest": _lib.LB_ROUND_NEAREST, "stochastic": _lib.LB_ROUND_STOCHASTIC}[self.rounding]
        p.walls = 1 if self.walls else 0
        return p


class DeviceBeads:
    """Bead state on the device (float64 tensors, positions unwrapped)."""

    def __init__(self, pos, mom, mass, zeta, bonds=None, k_bond=0.0, r0=1.0, device="cuda", stencil: int = 2,
                 fext=None, bond: str = "harmonic", wca_epsilon: float = 0.0, wca_sigma: float = 1.0,
                 noise: str = "gaussian"):
        """stencil: points per axis of the interpolation kernel (2, 3, 4 for
        phi_2, phi_3, phi_4); fext: optional [n, 3] external force per bead;
        bond: "harmonic" ((k/2)(r - r0)^2) or "fene" (-(k/2) r0^2 ln(1 - r^2/r0^2),
        r0 the maximum extension); wca_epsilon > 0 adds the purely repulsive
        Lennard-Jones pair force (cut at 2^(1/6) wca_sigma) between all beads;
        noise: "gaussian" or "three_point" (the finite-range variate 0, +-sqrt(3)
        with probabilities 2/3, 1/6, 1/6) for the bead momentum update."""
        dev = torch.device(device)
        noises = {"gaussian": _lib.LB_NOISE_GAUSSIAN, "three_point": _lib.LB_NOISE_THREE_POINT}
        if noise not in noises:
            raise ValueError(f"noise must be one of {sorted(noises)}")
        self.noise = noise
        self._noise_code = noises[noise]
        self.stencil = int(stencil)
        kinds = {"harmonic": _lib.LB_BOND_HARMONIC, "fene": _lib.LB_BOND_FENE}
        if bond not in kinds:
            raise ValueError(f"bond must be one of {sorted(kinds)}")
        self.bond = bond
        self._bond_code = kinds[bond]
        self.wca_epsilon = float(wca_epsilon)
        self.wca_sigma = float(wca_sigma)
        self.fext = None if fext is None else torch.as_tensor(fext, dtype=torch.float64, device=dev).reshape(-1, 3)
        if self.fext is not None:
            self.fext = self.fext.contiguous()
        self.pos = torch.as_tensor(pos, dtype=torch.float64, device=dev).reshape(-1, 3).contiguous()
        self.mom = torch.as_tensor(mom, dtype=torch.float64, device=dev).reshape(-1, 3).contiguous()
        self.mass = torch.as_tensor(mass, dtype=torch.float64, device=dev).reshape(-1).contiguous()
        self.zeta = torch.as_tensor(zeta, dtype=torch.float64, device=dev).reshape(-1).contiguous()
        if bonds is None:
            bonds = torch.zeros((0, 2), dtype=torch.int32)
        self.bonds = torch.as_tensor(bonds, dtype=torch.int32, device=dev).reshape(-1, 2).contiguous()
        self.k_bond = float(k_bond)
        self.r0 = float(r0)
        n = self.pos.shape[0]
        if self.mom.shape[0] != n or self.mass.shape[0] != n or self.zeta.shape[0] != n:
            raise ValueError("bead arrays must have matching lengths")

    @property
    def n(self) -> int:
        return self.pos.shape[0]

    def to_c(self) -> _lib.lb_beads:
        b = _lib.lb_beads()
        b.n = self.n
        b.nbonds = self.bonds.shape[0]
        b.pos = self.pos.data_ptr()
        b.mom = self.mom.data_ptr()
        b.mass = self.mass.data_ptr()
        b.zeta = self.zeta.data_ptr()
        b.bonds = self.bonds.data_ptr() if self.bonds.numel() else None
        b.k_bond = self.k_bond
        b.r0 = self.r0
        b.fext = self.fext.data_ptr() if self.fext is not None else None
        b.stencil = self.stencil
        b.bond = self._bond_code
        b.wca_epsilon = self.wca_epsilon
        b.wca_sigma = self.wca_sigma
        b.noise = self._noise_code
        return b


class Lattice:
    """One periodic box on the current GPU, enqueued on torch's current stream."""

    def __init__(self, params: FluidParams, stream: torch.cuda.Stream | None = None):
        self.L = _lib.load()
        if not torch.cuda.is_available():
            raise RuntimeError("liblbmi needs a GPU (torch.cuda.is_available() is False)")
        self.params = params
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self._p = params.to_c()
        ctx = ctypes.c_void_p()
        rc = self.L.lb_create(ctypes.byref(self._p), ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(ctx))
        if rc != 0:
            raise _lib.LBError(rc, self.L.lb_last_error(None).decode())
        self.ctx = ctx

    # -- lifetime
    def close(self) -> None:
        if getattr(self, "ctx", None):
            self.L.lb_destroy(self.ctx)
            self.ctx = None
        self._tape_refs = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc: int) -> None:
        check(rc, self.ctx)

    @property
    def N(self) -> int:
        return self.params.N

    def _dev(self, t: torch.Tensor, dtype) -> torch.Tensor:
        t = torch.as_tensor(t, dtype=dtype, device=self.device).contiguous()
        return t

    # -- state
    def init_equilibrium(self, rho=None, u=None) -> None:
        r = self._dev(rho, torch.float64).reshape(-1) if rho is not None else None
        uu = self._dev(u, torch.float64).reshape(-1) if u is not None else None
        if r is not None and r.numel() != self.N:
            raise ValueError("rho must have N elements")
        if uu is not None and uu.numel() != 3 * self.N:
            raise ValueError("u must have 3N elements")
        self._check(self.L.lb_init_equilibrium(self.ctx, r.data_ptr() if r is not None else None,
                                               uu.data_ptr() if uu is not None else None))
        self._keep = (r, uu)
        self._tape_ended()

    def set_populations(self, n, shifted: bool = False) -> None:
        t = torch.as_tensor(n, device=self.device)
        if t.dtype not in (torch.float64, torch.float32):
            t = t.to(torch.float64)
        t = t.contiguous()
        if t.numel() != Q * self.N:
            raise ValueError("populations must have 19*N elements")
        dt = LB_F64 if t.dtype == torch.float64 else LB_F32
        self._check(self.L.lb_set_populations(self.ctx, t.data_ptr(), dt, 1 if shifted else 0))
        self._keep = t
        self._tape_ended()

    def _tape_ended(self) -> None:
        # the library ends a tape when the state or the step counter is replaced
        self._taped_beads = None
        self._tape_refs = []

    def get_populations(self, dtype=torch.float64, shifted: bool = False) -> torch.Tensor:
        out = torch.empty((Q, self.params.nz, self.params.ny, self.params.nx), dtype=dtype, device=self.device)
        dt = LB_F64 if dtype == torch.float64 else LB_F32
        self._check(self.L.lb_get_populations(self.ctx, out.data_ptr(), dt, 1 if shifted else 0))
        return out

    # -- dynamics
    def step(self, nsteps: int = 1) -> None:
        self._check(self.L.lb_step(self.ctx, int(nsteps)))

    def couple(self, beads: DeviceBeads) -> None:
        b = beads.to_c()
        self._check(self.L.lb_couple(self.ctx, ctypes.byref(b)))
        if getattr(self, "_taped_beads", None) is not None:
            self._taped_beads = beads.n
            # the tape keeps this call's lb_beads descriptor (mass, zeta,
            # bonds, fext pointers) until backward: keep the tensors alive
            if not any(x is beads for x in self._tape_refs):
                self._tape_refs.append(beads)

    def coupled_step(self, beads: DeviceBeads) -> None:
        """Particle update + spreading, then one LB step (the paper's schedule)."""
        self.couple(beads)
        self.step(1)

    def coupled_steps(self, beads: DeviceBeads, nsteps: int) -> None:
        """nsteps coupled steps (lb_coupled_steps: one launch per step where
        the run allows it; the same bits as nsteps coupled_step calls)."""
        b = beads.to_c()
        self._check(self.L.lb_coupled_steps(self.ctx, ctypes.byref(b), int(nsteps)))
        if getattr(self, "_taped_beads", None) is not None and nsteps > 0:
            self._taped_beads = beads.n
            if not any(x is beads for x in self._tape_refs):
                self._tape_refs.append(beads)

    # -- observables
    def moments(self):
        rho = torch.empty((self.params.nz, self.params.ny, self.params.nx), dtype=torch.float64, device=self.device)
        u = torch.empty((3, self.params.nz, self.params.ny, self.params.nx), dtype=torch.float64,
                        device=self.device)
        self._check(self.L.lb_moments(self.ctx, rho.data_ptr(), u.data_ptr()))
        return rho, u

    def totals(self, exact: bool = False):
        out = (ctypes.c_double * 4)()
        fn = self.L.lb_totals_exact if exact else self.L.lb_totals
        self._check(fn(self.ctx, out))
        return [out[i] for i in range(4)]

    def mode_stats(self):
        out = (ctypes.c_double * 19)()
        self._check(self.L.lb_mode_stats(self.ctx, out))
        return [out[i] for i in range(19)]

    def noise_sample(self, site0: int, count: int, step: int) -> torch.Tensor:
        out = torch.empty((count, 15), dtype=torch.float32, device=self.device)
        self._check(self.L.lb_noise_sample(self.ctx, int(site0), int(count), int(step), out.data_ptr()))
        return out

    def negative_count(self):
        """(sites with a negative population, smallest population) of the
        current state (lb_negative_count)."""
        n = ctypes.c_uint64(0)
        m = ctypes.c_double(0.0)
        self._check(self.L.lb_negative_count(self.ctx, ctypes.byref(n), ctypes.byref(m)))
        return int(n.value), float(m.value)

    def sync(self) -> None:
        self._check(self.L.lb_sync(self.ctx))

    def tape_begin(self, checkpoint_every: int) -> None:
        self._check(self.L.lb_tape_begin(self.ctx, int(checkpoint_every)))
        self._taped_beads = 0
        self._tape_refs = []

    def tape_reserve(self, nsteps: int, beads: DeviceBeads | None = None) -> None:
        """Allocate now the checkpoints (and, with beads, the bead tape) that
        the next nsteps taped steps will take (lb_tape_reserve)."""
        b = beads.to_c() if beads is not None else None
        self._check(self.L.lb_tape_reserve(self.ctx, int(nsteps), ctypes.byref(b) if b is not None else None))

    def backward(self, dL_dnT: torch.Tensor):
        """dL/dn(t0) and dL/dg for the steps taken since tape_begin."""
        t = torch.as_tensor(dL_dnT, device=self.device)
        if t.dtype not in (torch.float64, torch.float32):
            t = t.to(torch.float64)
        t = t.contiguous()
        if t.numel() != Q * self.N:
            raise ValueError("dL_dnT must have 19*N elements")
        out = torch.empty_like(t)
        gbar = (ctypes.c_double * 3)()
        dt = LB_F64 if t.dtype == torch.float64 else LB_F32
        self._check(self.L.lb_backward(self.ctx, t.data_ptr(), dt, out.data_ptr(), gbar))
        return out.reshape(t.shape), [gbar[i] for i in range(3)]

    def backward_coupled(self, dL_dnT: torch.Tensor, dL_dRT: torch.Tensor | None = None,
                         dL_dPT: torch.Tensor | None = None):
        """(dL/dn(t0), dL/dg, dL/dR(t0), dL/dP(t0)) for the steps taken since
        tape_begin, coupled steps included; the bead adjoints are float64
        [n, 3] device tensors (None if no coupled step was taped)."""
        t = torch.as_tensor(dL_dnT, device=self.device)
        if t.dtype not in (torch.float64, torch.float32):
            t = t.to(torch.float64)
        t = t.contiguous()
        if t.numel() != Q * self.N:
            raise ValueError("dL_dnT must have 19*N elements")
        nb = getattr(self, "_taped_beads", 0)
        out = torch.empty_like(t)
        gbar = (ctypes.c_double * 3)()
        dt = LB_F64 if t.dtype == torch.float64 else LB_F32

        def bead_in(x):
            if x is None or nb == 0:
                return None
            x = torch.as_tensor(x, dtype=torch.float64, device=self.device).contiguous()
            if x.numel() != 3 * nb:
                raise ValueError("bead gradients must have n*3 elements")
            return x
        rt, pt = bead_in(dL_dRT), bead_in(dL_dPT)
        r0 = torch.empty((nb, 3), dtype=torch.float64, device=self.device) if nb else None
        p0 = torch.empty((nb, 3), dtype=torch.float64, device=self.device) if nb else None
        ptr = lambda x: x.data_ptr() if x is not None else None
        self._check(self.L.lb_backward_coupled(self.ctx, t.data_ptr(), dt, ptr(rt), ptr(pt), out.data_ptr(), gbar,
                                               ptr(r0), ptr(p0)))
        return out.reshape(t.shape), [gbar[i] for i in range(3)], r0, p0

    def save(self, path: str) -> None:
        """Write the state and step counter to a checkpoint file (lb_save)."""
        self._check(self.L.lb_save(self.ctx, os.fsencode(path)))

    def load(self, path: str) -> None:
        """Resume from a checkpoint file of the same layout (lb_load)."""
        self._check(self.L.lb_load(self.ctx, os.fsencode(path)))
        self._tape_ended()

    def launch_config(self, force: bool = False):
        """(threads per block, blocks per step, tiles per block, XCD mapping) of
        the step kernel; `force`: the variant that runs after couple()."""
        out = (ctypes.c_int32 * 4)()
        self._check(self.L.lb_launch_config(self.ctx, 1 if force else 0, out))
        return tuple(out)

    @property
    def step_count(self) -> int:
        return int(self.L.lb_step_count(self.ctx))

    @step_count.setter
    def step_count(self, v: int) -> None:
        self._check(self.L.lb_set_step_count(self.ctx, int(v)))
        self._tape_ended()


class BatchLattice(Lattice):
    """Many independent periodic replica boxes advanced together (one
    persistent launch per step, optionally replayed from a HIP graph).

    dims: sequence of (nx, ny, nz).  Box b uses Philox box id params.box_id + b.
    Population / field arrays are concatenated box after box, each in the
    single-box layout ([19][N_b] resp. [3][N_b])."""

    def __init__(self, params: FluidParams, dims, stream: torch.cuda.Stream | None = None):
        self.L = _lib.load()
        if not torch.cuda.is_available():
            raise RuntimeError("liblbmi needs a GPU (torch.cuda.is_available() is False)")
        self.params = params
        self.dims = [tuple(int(v) for v in d) for d in dims]
        self.sizes = [d[0] * d[1] * d[2] for d in self.dims]
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self._p = params.to_c()
        flat = (ctypes.c_int32 * (3 * len(self.dims)))(*[v for d in self.dims for v in d])
        ctx = ctypes.c_void_p()
        rc = self.L.lb_create_batch(ctypes.byref(self._p), len(self.dims), flat,
                                    ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(ctx))
        if rc != 0:
            raise _lib.LBError(rc, self.L.lb_last_error(None).decode())
        self.ctx = ctx

    @property
    def N(self) -> int:
        return sum(self.sizes)

    def get_populations(self, dtype=torch.float64, shifted: bool = False) -> torch.Tensor:
        out = torch.empty(Q * self.N, dtype=dtype, device=self.device)
        dt = LB_F64 if dtype == torch.float64 else LB_F32
        self._check(self.L.lb_get_populations(self.ctx, out.data_ptr(), dt, 1 if shifted else 0))
        return out

    def split(self, flat: torch.Tensor, comps: int = Q):
        """Split a concatenated per-box array into [comps, nz, ny, nx] views."""
        outs, o = [], 0
        for (nx, ny, nz), n in zip(self.dims, self.sizes):
            outs.append(flat[o:o + comps * n].reshape(comps, nz, ny, nx))
            o += comps * n
        return outs

    def moments(self):
        rho = torch.empty(self.N, dtype=torch.float64, device=self.device)
        u = torch.empty(3 * self.N, dtype=torch.float64, device=self.device)
        self._check(self.L.lb_moments(self.ctx, rho.data_ptr(), u.data_ptr()))
        return rho, u

    def vacf(self):
        R = self.params.vacf_lags
        out = (ctypes.c_double * (len(self.dims) * R))()
        ns = ctypes.c_int64()
        self._check(self.L.lb_vacf(self.ctx, out, ctypes.byref(ns)))
        import numpy as np
        return np.frombuffer(out, dtype=np.float64).reshape(len(self.dims), R).copy(), int(ns.value)
