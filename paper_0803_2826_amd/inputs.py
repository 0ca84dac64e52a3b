"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke
check.  Holds none of the method's arithmetic: only initial fields and bead
configurations, drawn with numpy's PCG64 generator from a fixed seed.

Recipes (lattice units):
  shear_wave      rho = rho0, u_flow(coord) = A sin(2 pi coord / L)
  random_walk_chains
                  n_chains chains of `length` beads; each chain starts at a
                  uniform random point of the box and takes unit-length steps
                  in uniformly random directions (isotropic unit vectors);
                  positions are unwrapped; momenta zero; bonds join
                  consecutive beads of a chain.
  kremer_grest_chains
                  self-avoiding random walks for the bead-spring model:
                  uniform starts, steps of `bond` (0.97 sigma) in isotropic
                  random directions, every new bead at least `min_dist`
                  (0.95 sigma, minimum image) from all beads placed before.
"""
from __future__ import annotations

import numpy as np


def shear_wave(nx: int, ny: int, nz: int, amp: float = 0.01, flow_axis: int = 0, var_axis: int = 2):
    """Velocity field [3, nz, ny, nx] of a sinusoidal shear wave."""
    dims = (nx, ny, nz)
    L = dims[var_axis]
    prof = amp * np.sin(2.0 * np.pi * np.arange(L) / L)
    shape = [1, 1, 1]
    shape[2 - var_axis] = L
    u = np.zeros((3, nz, ny, nx))
    u[flow_axis] = np.broadcast_to(prof.reshape(shape), (nz, ny, nx))
    return u


def random_velocity(nx: int, ny: int, nz: int, scale: float, seed: int):
    rng = np.random.default_rng(seed)
    return rng.normal(scale=scale, size=(3, nz, ny, nx))


def random_walk_chains(n_chains: int, length: int, box, seed: int):
    """Returns pos [n,3], mom [n,3], bonds [n_chains*(length-1), 2] (int32)."""
    rng = np.random.default_rng(seed)
    L = np.asarray(box, dtype=float)
    pos = np.zeros((n_chains * length, 3))
    bonds = []
    for c in range(n_chains):
        start = rng.uniform(0.0, 1.0, size=3) * L
        steps = rng.normal(size=(length - 1, 3))
        steps /= np.linalg.norm(steps, axis=1, keepdims=True)
        chain = np.vstack([start, start + np.cumsum(steps, axis=0)])
        pos[c * length:(c + 1) * length] = chain
        for k in range(length - 1):
            bonds.append((c * length + k, c * length + k + 1))
    bonds = np.asarray(bonds, dtype=np.int32).reshape(-1, 2)
    return pos, np.zeros_like(pos), bonds


def uniform_beads(n: int, box, seed: int):
    rng = np.random.default_rng(seed)
    return rng.uniform(0.0, 1.0, size=(n, 3)) * np.asarray(box, dtype=float)


def kremer_grest_chains(n_chains: int, length: int, box, seed: int, bond: float = 0.97, min_dist: float = 0.95,
                        max_tries: int = 200):
    """Self-avoiding random-walk chains for the bead-spring (Kremer-Grest)
    model: starts uniform in the box, consecutive beads `bond` apart in
    isotropic random directions, every new bead at least `min_dist` (minimum
    image) from all beads placed so far.  Returns pos [n, 3] (unwrapped),
    mom (zeros), bonds [n_chains*(length-1), 2] (int32)."""
    rng = np.random.default_rng(seed)
    L = np.asarray(box, dtype=float)
    pos = np.zeros((n_chains * length, 3))
    count = 0

    def free(x):
        if count == 0:
            return True
        d = pos[:count] - x
        d -= L * np.round(d / L)
        return (d * d).sum(1).min() >= min_dist * min_dist

    for c in range(n_chains):
        for _ in range(max_tries):
            start = rng.uniform(0.0, 1.0, size=3) * L
            if free(start):
                break
        else:
            raise RuntimeError("no room for a new chain")
        pos[count] = start
        count += 1
        for k in range(1, length):
            for _ in range(max_tries):
                step = rng.normal(size=3)
                x = pos[count - 1] + bond * step / np.linalg.norm(step)
                if free(x):
                    break
            else:
                raise RuntimeError("chain growth is stuck")
            pos[count] = x
            count += 1
    bonds = np.array([(c * length + k, c * length + k + 1) for c in range(n_chains) for k in range(length - 1)],
                     dtype=np.int32).reshape(-1, 2)
    return pos, np.zeros_like(pos), bonds


# The differentiation workload (lattice units): a 128^3 box at rest, kT 1e-4,
# Philox seed 0, uniform body force g, 16 random-walk chains of 32 beads
# (harmonic bonds k = 10 kT, r0 = 1, zeta = 20, m = 1), 500 coupled steps with
# a checkpoint every 50; loss = mean abs(u)^2 over the probe cube [56, 72)^3
# plus the mean squared bead drag abs(zeta (P/m - u(R)))^2 at the final step.
DIFF_WORKLOAD = dict(L=128, steps=500, checkpoint_every=50, chains=16, length=32, chain_seed=0, zeta=20.0,
                     k_bond=1e-3, r0=1.0, mass=1.0, kT=1e-4, seed=0, g=(1e-5, 0.0, 0.0), probe=(56, 72))


def direction(n_pops: int, n_beads: int, seed: int, scale_n: float = 1e-3, scale_g: float = 1e-6,
              scale_R: float = 1e-5, scale_P: float = 1e-3):
    """A seeded random direction (v_n [n_pops], v_g [3], v_R [n_beads, 3],
    v_P [n_beads, 3]) in (n(0), g, R(0), P(0)) for directional derivatives."""
    rng = np.random.default_rng(seed)
    return (rng.normal(size=n_pops) * scale_n, rng.normal(size=3) * scale_g, rng.normal(size=(n_beads, 3)) * scale_R,
            rng.normal(size=(n_beads, 3)) * scale_P)
