"""Checkpoint / resume through the C ABI (lb_save / lb_load): a run that is
saved, reloaded into a fresh context and continued reproduces the
uninterrupted run bit for bit (the noise and the stochastic rounding are
keyed by site and step), for a single box in each storage form and for a
batch; files of another layout, truncated or missing files are refused."""
import numpy as np
import pytest

from conftest import gpu_available

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lat():
    if not gpu_available():
        pytest.skip("no GPU")
    from paper_0803_2826_amd import lattice
    return lattice


@pytest.mark.parametrize("storage,rounding", [("f32", "nearest"), ("bf16", "stochastic"), ("f16", "nearest")])
def test_resume_is_bitwise(lat, tmp_path, storage, rounding):
    import torch
    from paper_0803_2826_amd.inputs import shear_wave
    p = lat.FluidParams(nx=20, ny=16, nz=12, storage=storage, rounding=rounding, kT=1e-4, seed=7,
                        body_force=(1e-5, 0.0, 0.0))
    a = lat.Lattice(p)
    a.init_equilibrium(u=torch.from_numpy(shear_wave(20, 16, 12, 0.01)).cuda())
    a.step(7)
    path = str(tmp_path / "state.lbck")
    a.save(path)
    a.step(5)
    b = lat.Lattice(p)
    b.init_equilibrium()
    b.load(path)
    assert b.step_count == 7
    b.step(5)
    assert torch.equal(a.get_populations(dtype=torch.float32), b.get_populations(dtype=torch.float32))
    a.close()
    b.close()


def test_coupled_resume_is_bitwise(lat, tmp_path):
    """Coupled steps with many beads sharing nodes: the spread force is summed
    in fixed point with integer atomics, so a resumed run (fluid from the
    checkpoint, bead state kept by the caller) repeats the original bit for
    bit, and so do two runs from the same start."""
    import numpy as np
    import torch
    from paper_0803_2826_amd.inputs import random_walk_chains
    L = 12
    p = lat.FluidParams(nx=L, ny=L, nz=L, kT=1e-4, seed=3, body_force=(1e-5, 0.0, 0.0))
    pos, mom, bonds = random_walk_chains(8, 16, (L, L, L), seed=2)     # 128 beads in 1728 sites
    nb = pos.shape[0]

    def beads(P, M):
        return lat.DeviceBeads(P, M, np.ones(nb), np.full(nb, 2.0), bonds, 1e-3, 1.0)

    a = lat.Lattice(p)
    a.init_equilibrium()
    ba = beads(pos, mom)
    for _ in range(6):
        a.coupled_step(ba)
    path = str(tmp_path / "coupled.lbck")
    a.save(path)
    P6, M6 = ba.pos.clone(), ba.mom.clone()
    for _ in range(8):
        a.coupled_step(ba)
    b = lat.Lattice(p)
    b.init_equilibrium()
    b.load(path)
    bb = beads(P6.cpu().numpy(), M6.cpu().numpy())
    for _ in range(8):
        b.coupled_step(bb)
    assert torch.equal(a.get_populations(dtype=torch.float32), b.get_populations(dtype=torch.float32))
    assert torch.equal(ba.pos, bb.pos) and torch.equal(ba.mom, bb.mom)
    # a third run from the very start agrees too
    c = lat.Lattice(p)
    c.init_equilibrium()
    bc = beads(pos, mom)
    for _ in range(14):
        c.coupled_step(bc)
    assert torch.equal(a.get_populations(dtype=torch.float32), c.get_populations(dtype=torch.float32))
    assert torch.equal(ba.mom, bc.mom)
    for x in (a, b, c):
        x.close()


def test_batch_resume_is_bitwise(lat, tmp_path):
    import torch
    dims = [(12, 12, 12), (16, 8, 10), (24, 24, 24)]
    p = lat.FluidParams(nx=2, ny=2, nz=2, kT=1e-4, seed=3, block=256, graph_steps=4)
    a = lat.BatchLattice(p, dims)
    a.init_equilibrium()
    a.step(6)
    path = str(tmp_path / "batch.lbck")
    a.save(path)
    a.step(8)
    b = lat.BatchLattice(p, dims)
    b.init_equilibrium()
    b.load(path)
    assert b.step_count == 6
    b.step(8)
    assert torch.equal(a.get_populations(dtype=torch.float32), b.get_populations(dtype=torch.float32))
    a.close()
    b.close()


def test_checkpoint_errors(lat, tmp_path):
    from paper_0803_2826_amd._lib import LB_EIO, LB_ESTATE, LBError
    a = lat.Lattice(lat.FluidParams(nx=8, ny=8, nz=8, kT=1e-4))
    a.init_equilibrium()
    a.step(2)
    path = tmp_path / "s.lbck"
    a.save(str(path))
    other = lat.Lattice(lat.FluidParams(nx=8, ny=8, nz=10, kT=1e-4))
    with pytest.raises(LBError) as ei:
        other.load(str(path))
    assert ei.value.code == LB_EIO
    other.close()
    half = tmp_path / "half.lbck"
    half.write_bytes(path.read_bytes()[: path.stat().st_size // 2])
    with pytest.raises(LBError) as ei:
        a.load(str(half))
    assert ei.value.code == LB_EIO
    with pytest.raises(LBError) as ei:
        a.load(str(tmp_path / "missing.lbck"))
    assert ei.value.code == LB_EIO
    beads = lat.DeviceBeads(np.array([[1.5, 2.5, 3.5]]), np.zeros((1, 3)), np.ones(1), np.ones(1))
    a.couple(beads)
    with pytest.raises(LBError) as ei:
        a.save(str(path))
    assert ei.value.code == LB_ESTATE
    a.step(1)
    a.save(str(path))
    a.close()
