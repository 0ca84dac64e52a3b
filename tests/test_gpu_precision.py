"""Precision form: populations stored as shifted deviations in FP32, BF16 or
FP16 (FP16 scaled by 2^8), FP32 collision arithmetic.  Through the C ABI.

Tolerances from the storage rounding (round to nearest even; significant
bits 24 / 8 / 11 for FP32 / BF16 / FP16, i.e. relative half spacing
2^-24 / 2^-8 / 2^-11, on values |d| <= 0.05):
- parity with the FP64 oracle after 20 steps, from the device's rounded
  initial state: the collision output rounds by at most 0.05 * 2^-8 = 2e-4
  (BF16) and 2.4e-5 (FP16) per step and the roundings of successive steps
  are independent; bounds 1e-3 (BF16), 1.5e-4 (FP16), 1e-6 (FP32);
- shear-wave decay rate (k = 2 pi / 512, 2000 steps, 64 x 64 x 512 sites,
  noise cancelled by a second run with the same seed and no wave): the
  rounding noise of the difference (spacing ~6e-5 at |d| ~ 1e-2 for BF16)
  projected on the mode random-walks to ~2 % of the total decay for BF16,
  ~0.1 % for FP16; bounds 1e-3 (FP32), 1 % (FP16), 8 % (BF16);
- stationary mode variances within 3 % of 3 kT w_k rho0 for every storage.
"""
import numpy as np
import pytest

from conftest import gpu_available

pytestmark = pytest.mark.gpu

PARITY_TOL = {"f32": 1e-6, "bf16": 1e-3, "f16": 1.5e-4}
DECAY_TOL = {"f32": 1e-3, "bf16": 0.08, "f16": 0.01}


@pytest.fixture(scope="module")
def lat():
    if not gpu_available():
        pytest.skip("no GPU")
    from paper_0803_2826_amd import lattice
    return lattice


@pytest.mark.parametrize("storage", ["f32", "bf16", "f16"])
def test_storage_parity(orc, lat, storage):
    import torch
    from paper_0803_2826_amd.inputs import shear_wave
    L = 24
    po = orc.Params(nx=L, ny=L, nz=L, kT=1e-4, seed=3, g=(1e-5, 0, 0))
    pd = lat.FluidParams(nx=L, ny=L, nz=L, storage=storage, kT=1e-4, seed=3, body_force=(1e-5, 0, 0))
    n = orc.init_equilibrium(po, u=shear_wave(L, L, L, 0.01))
    dev = lat.Lattice(pd)
    dev.set_populations(torch.from_numpy(n))
    # the oracle starts from the device's rounded initial state
    n = dev.get_populations().cpu().numpy()
    orc.run(po, n, 20)
    dev.step(20)
    err = np.abs(dev.get_populations().cpu().numpy() - n).max()
    print(f"{storage}: max|dn| after 20 steps = {err:.3e}")
    assert err <= PARITY_TOL[storage]
    dev.close()


@pytest.mark.parametrize("storage", ["f32", "bf16", "f16"])
def test_shear_decay_rate_per_storage(lat, storage):
    from paper_0803_2826_amd.forms import decay_rate
    d = decay_rate(storage, 64, 64, 512, steps=2000, kT=1e-4)
    print(storage, d)
    assert abs(d["rel_err"]) <= DECAY_TOL[storage]


@pytest.mark.parametrize("storage", ["f32", "bf16", "f16"])
def test_noise_variance_per_storage(lat, storage):
    from paper_0803_2826_amd.forms import mode_variances
    v = mode_variances(storage, 32, 1e-4, 300)
    print(storage, np.round(v, 4))
    np.testing.assert_allclose(v, 1.0, atol=0.03)


@pytest.mark.parametrize("storage", ["bf16", "f16"])
def test_mass_with_16bit_storage(lat, storage):
    """The rest-population residual keeps each site's stored mass equal to its
    stored input mass up to one rounding of the residual to the storage type:
    drift ~ half-ulp * sqrt(N T) at most."""
    pd = lat.FluidParams(nx=32, ny=32, nz=32, storage=storage, kT=1e-4, seed=4)
    dev = lat.Lattice(pd)
    dev.init_equilibrium()
    m0 = dev.totals(exact=True)[0]
    dev.step(100)
    m1 = dev.totals(exact=True)[0]
    half_ulp = {"bf16": 0.05 * 2.0 ** -8, "f16": 0.05 * 2.0 ** -11}[storage]
    print(storage, "relative mass drift", (m1 - m0) / m0)
    assert abs(m1 - m0) <= 6 * half_ulp * np.sqrt(32 ** 3 * 100) / np.sqrt(3)
    dev.close()
