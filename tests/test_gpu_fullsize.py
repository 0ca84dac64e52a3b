"""Parity at full workload sizes, in the launch configuration bench.py times,
on sampled outputs that the oracle computes one by one.

After a few steps on the GPU, the device state n(t) is read back and one more
step is taken on the device; for sampled sites r the oracle recomputes
n_i(r, t+1) = C(n(r - c_i, t), F(r - c_i))_i with the same Philox counters
(site, step, box) and compares.  With beads, the oracle's coupling routine
is run on the device state (FP64 copy) and bead state, and its bead update and
spread force field are compared with the device's (the force enters the
sampled collisions).  Tolerances as in the small-size parity tests.
"""
import numpy as np
import pytest

from conftest import gpu_available

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

C = np.array([[0, 0, 0], [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1], [1, 1, 0], [-1, -1, 0],
              [1, -1, 0], [-1, 1, 0], [1, 0, 1], [-1, 0, -1], [1, 0, -1], [-1, 0, 1], [0, 1, 1], [0, -1, -1],
              [0, 1, -1], [0, -1, 1]])


@pytest.fixture(scope="module")
def lat():
    if not gpu_available():
        pytest.skip("no GPU")
    from paper_0803_2826_amd import lattice
    return lattice


def sampled_step_reference(orc, p, n_flat, dims, sites, step, force=None):
    """Oracle n_i(r, t+1) for sampled sites r (n_flat: [19, N] FP64 state at t)."""
    nx, ny, nz = dims
    N = nx * ny * nz
    out = np.zeros((len(sites), 19))
    for k, s in enumerate(sites):
        x, y, z = s % nx, (s // nx) % ny, s // (nx * ny)
        for i in range(19):
            src = ((x - C[i, 0]) % nx) + nx * (((y - C[i, 1]) % ny) + ny * ((z - C[i, 2]) % nz))
            F = np.array(p.g, dtype=float)
            if force is not None:
                F = F + force[:, src]
            g = orc.fluid_normals(p.seed, int(src), step, p.box) if p.kT > 0 else None
            out[k, i] = orc.collide_site(p, n_flat[:, src], F, g)[i]
    return out


def test_bench_workload_256_coupled(orc, lat):
    """The 256^3 coupled workload of bench.py (64 chains x 32 beads, kT 1e-4,
    FP32, launch configuration searched as in bench.py): bead update and the forced collision
    at bead-touched and random sites match the oracle."""
    import torch
    import bench
    from paper_0803_2826_amd.inputs import random_walk_chains
    L = 256
    N = L ** 3
    pos, mom, bonds = random_walk_chains(64, 32, (L, L, L), seed=0)
    nb = pos.shape[0]
    pd = lat.FluidParams(nx=L, ny=L, nz=L, storage="f32", kT=bench.KT, seed=0, track_totals=True, block=-1)
    dev = lat.Lattice(pd)
    dev.init_equilibrium()
    beads = lat.DeviceBeads(pos, mom, np.ones(nb), np.full(nb, 20.0), bonds, bench.K_BOND, 1.0)
    for _ in range(4):
        dev.coupled_step(beads)
    t = dev.step_count
    n_t = dev.get_populations(dtype=torch.float32).reshape(19, N).cpu().numpy().astype(np.float64)
    bo = orc.Beads(beads.pos.cpu().numpy().copy(), beads.mom.cpu().numpy().copy(), np.ones(nb), np.full(nb, 20.0),
                   bonds.copy(), bench.K_BOND, 1.0)
    dev.couple(beads)
    dev.step(1)
    n_t1 = dev.get_populations(dtype=torch.float32).reshape(19, N).cpu().numpy()
    po = orc.Params(nx=L, ny=L, nz=L, kT=bench.KT, seed=0)
    force = np.zeros((3, L, L, L))
    orc.couple(po, n_t.reshape(19, L, L, L), t, bo, force)
    np.testing.assert_allclose(beads.pos.cpu().numpy(), bo.pos, atol=1e-7)
    np.testing.assert_allclose(beads.mom.cpu().numpy(), bo.mom, atol=1e-7)
    force = force.reshape(3, N)
    touched = np.nonzero(np.abs(force).sum(0))[0]
    rng = np.random.default_rng(0)
    sites = np.concatenate([rng.choice(touched, 300, replace=False), rng.integers(0, N, 300)])
    # the collisions at the neighbours of the sampled sites use the force there
    ref = sampled_step_reference(orc, po, n_t, (L, L, L), sites, t, force=force)
    got = n_t1[:, sites].T
    assert np.abs(got - ref).max() <= 1e-6


@pytest.mark.parametrize("storage,tol", [("f32", 1e-6), ("bf16", 1e-3), ("f16", 1.5e-4)])
def test_precision_workload_512(orc, lat, storage, tol):
    """512^3 with the precision form's storage types: one step from the device
    state, sampled sites."""
    import torch
    from paper_0803_2826_amd.inputs import shear_wave
    L = 512
    N = L ** 3
    pd = lat.FluidParams(nx=L, ny=L, nz=L, storage=storage, kT=1e-4, seed=1, track_totals=False)
    dev = lat.Lattice(pd)
    dev.init_equilibrium(u=torch.from_numpy(shear_wave(L, L, L, 0.01)).cuda())
    dev.step(3)
    t = dev.step_count
    rng = np.random.default_rng(1)
    sites = np.concatenate([rng.integers(0, N, 300), [0, N - 1, L - 1, L * L - 1]])
    n_t = dev.get_populations(dtype=torch.float32).reshape(19, N)
    # the 19 upstream neighbours of every sampled site
    nx = ny = nz = L
    need = set()
    for s in sites:
        x, y, z = s % nx, (s // nx) % ny, s // (nx * ny)
        for i in range(19):
            need.add(((x - C[i, 0]) % nx) + nx * (((y - C[i, 1]) % ny) + ny * ((z - C[i, 2]) % nz)))
    need = np.array(sorted(need))
    sub = n_t[:, torch.from_numpy(need).cuda()].cpu().numpy().astype(np.float64)
    full = {int(s): sub[:, k] for k, s in enumerate(need)}
    dev.step(1)
    n_t1 = dev.get_populations(dtype=torch.float32).reshape(19, N)[:, torch.from_numpy(sites).cuda()].cpu().numpy()
    dev.close()
    po = orc.Params(nx=L, ny=L, nz=L, kT=1e-4, seed=1)

    class Lookup:
        def __getitem__(self, idx):
            return full[int(idx[1])]
    ref = sampled_step_reference(orc, po, Lookup(), (L, L, L), sites, t)
    err = np.abs(n_t1.T - ref).max()
    print(storage, "512^3 sampled one-step err", err)
    assert err <= tol


def test_batched_workload_512_replicas(orc, lat):
    """512 replicas with edges drawn from {24,32,40,48,64}, autotuned launch,
    graph replay: one step from the device state on sampled sites of sampled
    boxes (each box keyed by its own box id)."""
    import torch
    from paper_0803_2826_amd.forms import edge_draws
    dims = edge_draws(512, seed=0)
    pd = lat.FluidParams(nx=2, ny=2, nz=2, kT=1e-4, seed=0, graph_steps=10, block=0)
    B = lat.BatchLattice(pd, dims)
    B.init_equilibrium()
    B.step(10)
    t = B.step_count
    state = B.split(B.get_populations(dtype=torch.float32))
    rng = np.random.default_rng(2)
    boxes = rng.choice(len(dims), 6, replace=False)
    before = {int(b): state[b].reshape(19, -1).cpu().numpy().astype(np.float64) for b in boxes}
    B.step(1)
    after = B.split(B.get_populations(dtype=torch.float32))
    for b in boxes:
        nx, ny, nz = dims[b]
        Nb = nx * ny * nz
        po = orc.Params(nx=nx, ny=ny, nz=nz, kT=1e-4, seed=0, box=int(b))
        sites = rng.integers(0, Nb, 40)
        ref = sampled_step_reference(orc, po, before[int(b)], (nx, ny, nz), sites, t)
        got = after[b].reshape(19, -1)[:, torch.from_numpy(sites).cuda()].cpu().numpy().T
        assert np.abs(got - ref).max() <= 1e-6, b
    B.close()
