"""The low-Mach guard lb_negative_count (sites with a negative population
n_i = a_i rho0 + d_i and the smallest n_i), through the C ABI.

- At rest every population is a_i rho0 > 0: no site, smallest 1/36 rho0.
- Planted negatives (the rest population, which also reads the FP32
  residual plane, and moving ones) in FP32 and BF16 storage: exactly the
  planted sites, the smallest planted value (to the storage rounding).
- A batch of two boxes with negatives planted in the second box only.
- A thermal run hot enough that noise drives populations negative: the
  count and the minimum equal a host recount of the populations read back
  (the same stored values, bit for bit).
"""
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


def host_count(n):
    m = n.min(axis=0)
    return int((m < 0).sum()), float(m.min())


def test_rest_has_no_negative_population(lat):
    dev = lat.Lattice(lat.FluidParams(nx=20, ny=16, nz=12))
    dev.init_equilibrium()
    count, mn = dev.negative_count()
    dev.close()
    assert count == 0 and mn == pytest.approx(1.0 / 36.0, abs=1e-15)


@pytest.mark.parametrize("storage,tol", [("f32", 1e-8), ("bf16", 1e-3)])
def test_planted_negatives(lat, storage, tol):
    import torch
    dev = lat.Lattice(lat.FluidParams(nx=20, ny=16, nz=12, storage=storage))
    dev.init_equilibrium()
    n = dev.get_populations().cpu()
    planted = [(0, 3, 4, 5, -0.03), (7, 0, 0, 0, -0.01), (12, 11, 15, 19, -0.05), (18, 6, 2, 9, -0.002)]
    for i, z, y, x, v in planted:
        n[i, z, y, x] = v
    dev.set_populations(n.to(dev.device))
    count, mn = dev.negative_count()
    dev.close()
    print(storage, count, mn)
    assert count == len(planted)
    assert mn == pytest.approx(-0.05, abs=tol)


def test_batch_counts_every_box(lat):
    import torch
    dims = [(12, 10, 8), (16, 12, 10)]
    dev = lat.BatchLattice(lat.FluidParams(nx=12, ny=10, nz=8), dims)
    dev.init_equilibrium()
    n = dev.get_populations().cpu().reshape(-1)
    n0 = 19 * 12 * 10 * 8  # box 1 follows box 0, each [19][N_b]
    second = n[n0:].reshape(19, -1)
    second[3, 17] = -0.02
    second[0, 400] = -0.04
    dev.set_populations(n.to(dev.device))
    count, mn = dev.negative_count()
    dev.close()
    assert count == 2
    assert mn == pytest.approx(-0.04, abs=1e-8)


def test_hot_noise_count_matches_host_recount(lat):
    """kT = 3e-3 at rho0 = 1: the noise on the populations with a_i = 1/36
    is about half of a_i rho0, so a few per cent go negative within a few
    steps (the run stays finite)."""
    dev = lat.Lattice(lat.FluidParams(nx=24, ny=24, nz=24, kT=3e-3, seed=5, gamma_shear=0.2, gamma_bulk=0.2))
    dev.init_equilibrium()
    dev.step(5)
    count, mn = dev.negative_count()
    n = dev.get_populations().cpu().numpy().reshape(19, -1)
    dev.close()
    assert np.isfinite(n).all()
    hc, hm = host_count(n)
    print("device", count, mn, "host", hc, hm)
    assert hc > 0
    assert count == hc and mn == hm
