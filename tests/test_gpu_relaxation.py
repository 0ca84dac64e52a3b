"""General relaxation on the GPU: the device's linearised dynamics equal the
19 x 19 stability operator A(k) = S(k) E^-1 diag(gamma) E (built from the
golden Table 1 fixture, eq. lco_eigen / eq. lco_update) for every eigenvalue
set of the oracle pins, including the two-rate relaxation.

Tolerance: the perturbation amplitude eps = 1e-5 makes the collision's
quadratic terms a relative 1e-5 effect; FP32 arithmetic on deviations of that
size rounds at ~1e-7 relative per step.  Bound 5e-5 relative to eps * max|v|.
"""
import numpy as np
import pytest

from conftest import gpu_available
from test_oracle_dynamics import RELAX_SETS, _mode_gammas, linear_operator

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lat():
    if not gpu_available():
        pytest.skip("no GPU")
    from paper_0803_2826_amd import lattice
    return lattice


@pytest.mark.parametrize("name", list(RELAX_SETS))
def test_gpu_linear_dynamics_equal_operator_power(orc, lat, name):
    import torch
    gs, gv, g3a, g3b, g4a, g4b = RELAX_SETS[name]
    nx, ny, nz = 6, 8, 10
    pd = lat.FluidParams(nx=nx, ny=ny, nz=nz, gamma_shear=gs, gamma_bulk=gv, gamma_3a=g3a, gamma_3b=g3b,
                         gamma_4a=g4a, gamma_4b=g4b, track_totals=False)
    c, a, e, w = orc.tables()
    rng = np.random.default_rng(3)
    kvec = 2 * np.pi * np.array([1 / nx, 2 / ny, 1 / nz])
    A = linear_operator(c, _mode_gammas(gs, gv, g3a, g3b, g4a, g4b), kvec)
    v = rng.normal(size=19) + 1j * rng.normal(size=19)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    phase = np.exp(1j * (kvec[0] * x + kvec[1] * y + kvec[2] * z))
    eps, T = 1e-5, 9
    n0 = a[:, None, None, None] + eps * np.real(v[:, None, None, None] * phase[None])
    dev = lat.Lattice(pd)
    dev.set_populations(torch.from_numpy(np.ascontiguousarray(n0)))
    dev.step(T)
    got = dev.get_populations().cpu().numpy()
    dev.close()
    vT = np.linalg.matrix_power(A, T) @ v
    expect = a[:, None, None, None] + eps * np.real(vT[:, None, None, None] * phase[None])
    err = np.abs(got - expect).max() / (eps * np.abs(v).max())
    print(name, "rel err", err)
    assert err < 5e-5


def test_two_rate_parameters(lat):
    p = lat.FluidParams(nx=4, ny=4, nz=4, **lat.two_rate(0.3))
    te, to = 1 / (1 - p.gamma_shear), 1 / (1 - p.gamma_3a)
    assert (te - 0.5) * (to - 0.5) == pytest.approx(3 / 16, rel=1e-14)
    assert p.gamma_bulk == p.gamma_4a == p.gamma_4b == p.gamma_shear == 0.3 and p.gamma_3b == p.gamma_3a
