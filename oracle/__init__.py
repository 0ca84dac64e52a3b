"""FP64 CPU oracle for the fluctuating D3Q19 lattice-Boltzmann hot path.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  It is the plain,
slow, obviously-correct reference the GPU library is checked against, and it
shares no code, header, table or generator with that library.

The arithmetic lives in ``lb_oracle.c`` (plain C, IEEE double, no
contraction); this module only builds it with gcc and marshals numpy arrays
through ctypes.  Each wrapped function names the passage of the paper it
follows in the C source.

Array layouts (all float64, C-contiguous):
  populations  n[19, nz, ny, nx]   (index i*N + x + nx*(y + ny*z))
  vector field  u[3, nz, ny, nx]
  bead arrays   pos, mom [nb, 3];  mass, zeta [nb];  bonds int32 [nbonds, 2]
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lb_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liblb_oracle.so")

Q = 19


def build(force: bool = False) -> str:
    """Compile lb_oracle.c into liblb_oracle.so with gcc (FP64, no contraction)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
               "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class OrcParams(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("noise_rho0", ctypes.c_int32),
        ("rho0", ctypes.c_double),
        ("gamma_shear", ctypes.c_double), ("gamma_bulk", ctypes.c_double),
        ("gamma_3a", ctypes.c_double), ("gamma_3b", ctypes.c_double),
        ("gamma_4a", ctypes.c_double), ("gamma_4b", ctypes.c_double),
        ("kT", ctypes.c_double),
        ("g", ctypes.c_double * 3),
        ("seed", ctypes.c_uint64),
        ("box", ctypes.c_uint32),
        ("walls", ctypes.c_uint32),
    ]



class OrcBeadset(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32), ("nbonds", ctypes.c_int32),
        ("mass", ctypes.POINTER(ctypes.c_double)), ("zeta", ctypes.POINTER(ctypes.c_double)),
        ("bonds", ctypes.POINTER(ctypes.c_int32)),
        ("kbond", ctypes.c_double), ("r0", ctypes.c_double),
        ("stencil", ctypes.c_int32), ("fene", ctypes.c_int32),
        ("fext", ctypes.POINTER(ctypes.c_double)),
        ("wca_eps", ctypes.c_double), ("wca_sigma", ctypes.c_double),
        ("three_point", ctypes.c_int32),
    ]

@dataclass
class Params:
    """Fluid parameters in lattice units (b = h = 1)."""
    nx: int
    ny: int
    nz: int
    rho0: float = 1.0
    gamma_shear: float = 0.0
    gamma_bulk: float = 0.0
    gamma_3a: float = 0.0
    gamma_3b: float = 0.0
    gamma_4a: float = 0.0
    gamma_4b: float = 0.0
    kT: float = 0.0
    g: tuple = (0.0, 0.0, 0.0)
    seed: int = 0
    noise_rho0: bool = False
    box: int = 0
    walls: bool = False   # stationary walls at z = -1/2 and z = nz - 1/2

    @property
    def N(self) -> int:
        return self.nx * self.ny * self.nz

    def c(self) -> OrcParams:
        p = OrcParams()
        p.nx, p.ny, p.nz = self.nx, self.ny, self.nz
        p.noise_rho0 = 1 if self.noise_rho0 else 0
        p.rho0 = self.rho0
        p.gamma_shear, p.gamma_bulk = self.gamma_shear, self.gamma_bulk
        p.gamma_3a, p.gamma_3b = self.gamma_3a, self.gamma_3b
        p.gamma_4a, p.gamma_4b = self.gamma_4a, self.gamma_4b
        p.kT = self.kT
        for a in range(3):
            p.g[a] = float(self.g[a])
        p.seed = int(self.seed) & 0xFFFFFFFFFFFFFFFF
        p.box = int(self.box)
        p.walls = 1 if self.walls else 0
        return p


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = build()
        L = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int32)
        up = ctypes.POINTER(ctypes.c_uint32)
        lp = ctypes.POINTER(ctypes.c_int64)
        pp = ctypes.POINTER(OrcParams)
        L.orc_tables.argtypes = [ip, dp, dp, dp]
        L.orc_philox4x32_10.argtypes = [up, up, up]
        L.orc_fluid_normals.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, dp]
        L.orc_bead_normals.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, dp]
        L.orc_bead_three_point.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, dp]
        L.orc_equilibrium.argtypes = [ctypes.c_double, dp, dp]
        L.orc_moments_site.argtypes = [dp, dp]
        L.orc_back_site.argtypes = [dp, dp]
        L.orc_collide_site.argtypes = [pp, dp, dp, dp, dp]
        L.orc_init_equilibrium.argtypes = [pp, dp, dp, dp]
        L.orc_step.argtypes = [pp, dp, dp, dp, ctypes.c_uint32]
        L.orc_run.argtypes = [pp, dp, ctypes.c_int32, ctypes.c_uint32]
        L.orc_fields.argtypes = [pp, dp, dp, dp]
        L.orc_totals.argtypes = [pp, dp, dp]
        L.orc_mode_field.argtypes = [pp, dp, dp]
        L.orc_transverse_modes.argtypes = [pp, dp, dp]
        L.orc_stencil.argtypes = [pp, dp, lp, dp]
        L.orc_couple.argtypes = [pp, dp, ctypes.c_uint32, ctypes.POINTER(OrcBeadset), dp, dp, dp]
        L.orc_coupled_step.argtypes = [pp, dp, dp, dp, ctypes.c_uint32, ctypes.POINTER(OrcBeadset), dp, dp]
        L.orc_stencil_w.argtypes = [pp, dp, ctypes.c_int32, lp, dp, dp]
        L.orc_stencil_w.restype = ctypes.c_int
        L.orc_phi.argtypes = [ctypes.c_int32, ctypes.c_double, dp]
        L.orc_bead_forces.argtypes = [pp, ctypes.POINTER(OrcBeadset), dp, dp]
        L.orc_collide_site_adjoint.argtypes = [pp, dp, dp, dp, dp, dp, dp]
        L.orc_step_adjoint.argtypes = [pp, dp, dp, dp, dp, dp, ctypes.c_uint32, dp]
        L.orc_backward.argtypes = [pp, dp, ctypes.c_int32, ctypes.c_uint32, dp, dp]
        L.orc_couple_adjoint.argtypes = [pp, dp, ctypes.c_uint32, ctypes.POINTER(OrcBeadset), dp, dp, dp, dp, dp, dp,
                                         dp]
        L.orc_backward_coupled.argtypes = [pp, dp, ctypes.c_int32, ctypes.c_uint32, ctypes.POINTER(OrcBeadset), dp, dp,
                                           dp, dp, dp, dp]
        L.orc_num_threads.argtypes = []
        L.orc_num_threads.restype = ctypes.c_int
        for name in ("orc_tables", "orc_philox4x32_10", "orc_fluid_normals", "orc_bead_normals", "orc_bead_three_point",
                     "orc_equilibrium", "orc_moments_site", "orc_back_site", "orc_collide_site",
                     "orc_init_equilibrium", "orc_step", "orc_run", "orc_fields", "orc_totals",
                     "orc_mode_field", "orc_transverse_modes", "orc_stencil", "orc_couple", "orc_coupled_step",
                     "orc_collide_site_adjoint", "orc_step_adjoint", "orc_backward", "orc_couple_adjoint",
                     "orc_backward_coupled", "orc_phi", "orc_bead_forces"):
            getattr(L, name).restype = None
        _lib = L
    return _lib


def num_threads() -> int:
    return int(lib().orc_num_threads())


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


# --------------------------------------------------------------------------
# tables, RNG
# --------------------------------------------------------------------------

def tables():
    """Return (c [19,3] int, a [19], e [19,19], w [19]) as written in the oracle."""
    c = np.zeros((Q, 3), np.int32)
    a = np.zeros(Q)
    e = np.zeros((Q, Q))
    w = np.zeros(Q)
    lib().orc_tables(c.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _dp(a), _dp(e), _dp(w))
    return c, a, e, w


def philox4x32_10(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(np.asarray(ctr, dtype=np.uint32))
    k = np.ascontiguousarray(np.asarray(key, dtype=np.uint32))
    out = np.zeros(4, np.uint32)
    up = ctypes.POINTER(ctypes.c_uint32)
    lib().orc_philox4x32_10(c.ctypes.data_as(up), k.ctypes.data_as(up), out.ctypes.data_as(up))
    return out


def fluid_normals(seed: int, site: int, step: int, box: int = 0) -> np.ndarray:
    g = np.zeros(16)
    lib().orc_fluid_normals(seed, site, step, box, _dp(g))
    return g


def bead_normals(seed: int, bead: int, step: int, box: int = 0) -> np.ndarray:
    g = np.zeros(3)
    lib().orc_bead_normals(seed, bead, step, box, _dp(g))
    return g


def bead_three_point(seed: int, bead: int, step: int, box: int = 0) -> np.ndarray:
    g = np.zeros(3)
    lib().orc_bead_three_point(seed, bead, step, box, _dp(g))
    return g


# --------------------------------------------------------------------------
# single site
# --------------------------------------------------------------------------

def equilibrium(rho: float, u) -> np.ndarray:
    uu = _f64(u)
    out = np.zeros(Q)
    lib().orc_equilibrium(float(rho), _dp(uu), _dp(out))
    return out


def moments_site(n) -> np.ndarray:
    nn = _f64(n)
    out = np.zeros(Q)
    lib().orc_moments_site(_dp(nn), _dp(out))
    return out


def back_site(m) -> np.ndarray:
    mm = _f64(m)
    out = np.zeros(Q)
    lib().orc_back_site(_dp(mm), _dp(out))
    return out


def collide_site(p: Params, n, F=(0.0, 0.0, 0.0), gnoise=None) -> np.ndarray:
    nn = _f64(n)
    FF = _f64(F)
    g = _f64(gnoise if gnoise is not None else np.zeros(16))
    out = np.zeros(Q)
    pc = p.c()
    lib().orc_collide_site(ctypes.byref(pc), _dp(nn), _dp(FF), _dp(g), _dp(out))
    return out


# --------------------------------------------------------------------------
# lattice
# --------------------------------------------------------------------------

def init_equilibrium(p: Params, rho=None, u=None) -> np.ndarray:
    n = np.zeros((Q, p.nz, p.ny, p.nx))
    r = _f64(rho).reshape(-1) if rho is not None else None
    uu = _f64(u).reshape(-1) if u is not None else None
    pc = p.c()
    lib().orc_init_equilibrium(ctypes.byref(pc), _dp(r) if r is not None else None,
                               _dp(uu) if uu is not None else None, _dp(n))
    return n


def step(p: Params, n: np.ndarray, step_index: int, extra_force=None) -> None:
    """One collide+stream step in place (extra_force: [3,nz,ny,nx] or None)."""
    work = np.empty_like(n)
    pc = p.c()
    ef = _f64(extra_force) if extra_force is not None else None
    lib().orc_step(ctypes.byref(pc), _dp(n), _dp(work), _dp(ef) if ef is not None else None, step_index)


def run(p: Params, n: np.ndarray, nsteps: int, step0: int = 0) -> None:
    pc = p.c()
    lib().orc_run(ctypes.byref(pc), _dp(n), int(nsteps), int(step0))


def fields(p: Params, n: np.ndarray):
    rho = np.zeros((p.nz, p.ny, p.nx))
    u = np.zeros((3, p.nz, p.ny, p.nx))
    pc = p.c()
    lib().orc_fields(ctypes.byref(pc), _dp(n), _dp(rho), _dp(u))
    return rho, u


def totals(p: Params, n: np.ndarray) -> np.ndarray:
    out = np.zeros(4)
    pc = p.c()
    lib().orc_totals(ctypes.byref(pc), _dp(n), _dp(out))
    return out


def mode_field(p: Params, n: np.ndarray) -> np.ndarray:
    m = np.zeros((Q, p.nz, p.ny, p.nx))
    pc = p.c()
    lib().orc_mode_field(ctypes.byref(pc), _dp(n), _dp(m))
    return m


def transverse_modes(p: Params, n: np.ndarray) -> np.ndarray:
    """The six lowest transverse Fourier amplitudes (complex) of the
    momentum density of n: k along z (j_x, j_y), along y (j_x, j_z), along x
    (j_y, j_z)."""
    out = np.zeros(12)
    pc = p.c()
    lib().orc_transverse_modes(ctypes.byref(pc), _dp(n), _dp(out))
    return out[0::2] + 1j * out[1::2]


def stencil(p: Params, R):
    RR = _f64(R)
    node = np.zeros(8, np.int64)
    w = np.zeros(8)
    pc = p.c()
    lib().orc_stencil(ctypes.byref(pc), _dp(RR), node.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _dp(w))
    return node, w


@dataclass
class Beads:
    """Bead state for the oracle (float64, positions unwrapped)."""
    pos: np.ndarray
    mom: np.ndarray
    mass: np.ndarray
    zeta: np.ndarray
    bonds: np.ndarray = field(default_factory=lambda: np.zeros((0, 2), np.int32))
    k_bond: float = 0.0
    r0: float = 1.0
    stencil: int = 2                 # points per axis of the interpolation kernel: 2, 3 or 4
    fext: np.ndarray | None = None   # [nb, 3] external force per bead
    fene: bool = False               # FENE bonds (k_bond = k, r0 = R0) instead of harmonic
    wca_eps: float = 0.0             # WCA interaction strength (0: off)
    wca_sigma: float = 1.0
    three_point: bool = False        # bead noise from the three-point distribution instead of Gaussians

    def copy(self) -> "Beads":
        return Beads(self.pos.copy(), self.mom.copy(), self.mass.copy(), self.zeta.copy(),
                     self.bonds.copy(), self.k_bond, self.r0, self.stencil,
                     None if self.fext is None else self.fext.copy(), self.fene, self.wca_eps, self.wca_sigma,
                     self.three_point)

    def c(self):
        """ctypes bead-set descriptor (and the arrays it points to)."""
        keep = [np.ascontiguousarray(self.mass, dtype=np.float64), np.ascontiguousarray(self.zeta, dtype=np.float64),
                np.ascontiguousarray(self.bonds, dtype=np.int32).reshape(-1),
                None if self.fext is None else np.ascontiguousarray(self.fext, dtype=np.float64)]
        b = OrcBeadset()
        b.n = self.pos.shape[0]
        b.nbonds = self.bonds.shape[0]
        b.mass = _dp(keep[0])
        b.zeta = _dp(keep[1])
        b.bonds = keep[2].ctypes.data_as(ctypes.POINTER(ctypes.c_int32)) if keep[2].size else None
        b.kbond = float(self.k_bond)
        b.r0 = float(self.r0)
        b.stencil = int(self.stencil)
        b.fene = 1 if self.fene else 0
        b.fext = _dp(keep[3]) if keep[3] is not None else None
        b.wca_eps = float(self.wca_eps)
        b.wca_sigma = float(self.wca_sigma)
        b.three_point = 1 if self.three_point else 0
        return b, keep


def couple(p: Params, n: np.ndarray, step_index: int, beads: Beads, force: np.ndarray) -> None:
    """Particle half-step; updates beads in place and accumulates into force [3,nz,ny,nx]."""
    bs, keep = beads.c()
    pc = p.c()
    lib().orc_couple(ctypes.byref(pc), _dp(n), int(step_index), ctypes.byref(bs), _dp(beads.pos), _dp(beads.mom),
                     _dp(force))


def coupled_step(p: Params, n: np.ndarray, step_index: int, beads: Beads) -> np.ndarray:
    """Particle update, spreading, then one LB step.  Returns the force field used."""
    force = np.zeros((3, p.nz, p.ny, p.nx))
    couple(p, n, step_index, beads, force)
    step(p, n, step_index, extra_force=force)
    return force


def stencil_w(p: Params, R, W: int):
    """(nodes, weights, d weights / dR) of the W-point interpolation stencil at R."""
    node = np.zeros(64, np.int64)
    w = np.zeros(64)
    dw = np.zeros(192)
    pc = p.c()
    q = lib().orc_stencil_w(ctypes.byref(pc), _dp(_f64(R)), int(W), node.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                            _dp(w), _dp(dw))
    return node[:q], w[:q], dw[:3 * q].reshape(q, 3)


def bead_forces(p: Params, beads: Beads, R: np.ndarray) -> np.ndarray:
    """Conservative forces [nb, 3] (bonds, WCA, external) at positions R."""
    bs, keep = beads.c()
    out = np.zeros((beads.pos.shape[0], 3))
    pc = p.c()
    lib().orc_bead_forces(ctypes.byref(pc), ctypes.byref(bs), _dp(_f64(R)), _dp(out))
    return out


def phi(W: int, r: float):
    """(phi_W(r), phi_W'(r))."""
    out = np.zeros(2)
    lib().orc_phi(int(W), float(r), _dp(out))
    return out[0], out[1]


# --------------------------------------------------------------------------
# adjoint
# --------------------------------------------------------------------------

def collide_site_adjoint(p: Params, n, F, gnoise, nbar_star):
    """Returns (dL/dn, dL/dF) given dL/dn* for one collision."""
    nn, FF = _f64(n), _f64(F)
    g = _f64(gnoise if gnoise is not None else np.zeros(16))
    nbs = _f64(nbar_star)
    nb = np.zeros(Q)
    Fb = np.zeros(3)
    pc = p.c()
    lib().orc_collide_site_adjoint(ctypes.byref(pc), _dp(nn), _dp(FF), _dp(g), _dp(nbs), _dp(nb), _dp(Fb))
    return nb, Fb


def step_adjoint(p: Params, n: np.ndarray, lam: np.ndarray, step_index: int, gbar: np.ndarray, extra_force=None,
                 extra_bar=None) -> None:
    """Adjoint of step(): lam (in: dL/dn after the step, out: before it) and
    gbar in place; with extra_force, its adjoint accumulates into extra_bar."""
    work = np.empty_like(lam)
    pc = p.c()
    ef = _f64(extra_force) if extra_force is not None else None
    lib().orc_step_adjoint(ctypes.byref(pc), _dp(_f64(n)), _dp(lam), _dp(work), _dp(ef) if ef is not None else None,
                           _dp(extra_bar) if extra_bar is not None else None, int(step_index), _dp(gbar))


def couple_adjoint(p: Params, n: np.ndarray, step_index: int, beads: "Beads", force_bar: np.ndarray,
                   pos_bar: np.ndarray, mom_bar: np.ndarray, lam: np.ndarray, gbar: np.ndarray) -> None:
    """Adjoint of couple() for the bead state `beads` the step started from:
    pos_bar / mom_bar (in: after the step, out: before it), lam and gbar
    accumulate; force_bar [3,nz,ny,nx] is the adjoint of the spread force."""
    bs, keep = beads.c()
    pc = p.c()
    lib().orc_couple_adjoint(ctypes.byref(pc), _dp(_f64(n)), int(step_index), ctypes.byref(bs), _dp(_f64(beads.pos)),
                             _dp(_f64(beads.mom)), _dp(_f64(force_bar)), _dp(pos_bar), _dp(mom_bar), _dp(lam),
                             _dp(gbar))


def backward_coupled(p: Params, n0: np.ndarray, nsteps: int, beads: "Beads", lam_T: np.ndarray,
                     pos_bar_T=None, mom_bar_T=None, step0: int = 0):
    """dL/dn(0), dL/dg, dL/dR(0), dL/dP(0) through nsteps coupled steps from
    (n0, beads) given dL/dn(T), dL/dR(T), dL/dP(T)."""
    nb = beads.pos.shape[0]
    lam = np.ascontiguousarray(lam_T, dtype=np.float64).copy()
    pb = np.zeros((nb, 3)) if pos_bar_T is None else np.ascontiguousarray(pos_bar_T, dtype=np.float64).copy()
    mb = np.zeros((nb, 3)) if mom_bar_T is None else np.ascontiguousarray(mom_bar_T, dtype=np.float64).copy()
    gbar = np.zeros(3)
    bs, keep = beads.c()
    pc = p.c()
    lib().orc_backward_coupled(ctypes.byref(pc), _dp(_f64(n0)), int(nsteps), int(step0), ctypes.byref(bs),
                               _dp(_f64(beads.pos)), _dp(_f64(beads.mom)), _dp(lam), _dp(gbar), _dp(pb), _dp(mb))
    return lam, gbar, pb, mb


def backward(p: Params, n0: np.ndarray, nsteps: int, lam_T: np.ndarray, step0: int = 0):
    """dL/dn(0) and dL/dg (through the dynamics) from dL/dn(T), no particles."""
    lam = np.ascontiguousarray(lam_T, dtype=np.float64).copy()
    gbar = np.zeros(3)
    pc = p.c()
    lib().orc_backward(ctypes.byref(pc), _dp(_f64(n0)), int(nsteps), int(step0), _dp(lam), _dp(gbar))
    return lam, gbar
