"""Three- and four-point interpolation kernels (eq. 3point, eq. 4point) and
external bead forces on the GPU, against the oracle (pinned by the kernels'
moment conditions, momentum accounting and central finite differences of
its adjoint), and the settling experiment of Sec. "Interpolating functions".

Tolerances as for the two-point coupling: populations 1e-6 absolute, bead
positions and momenta 1e-7, the coupled adjoint 2e-5 relative.
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


def beads_pair(orc, lat, rng, L, W, nb=12):
    pos = rng.uniform(0, L, size=(nb, 3))
    mom = rng.normal(scale=0.01, size=(nb, 3))
    fext = rng.normal(scale=1e-4, size=(nb, 3))
    bonds = np.array([[k, k + 1] for k in range(0, nb - 1, 2)], dtype=np.int32)
    zeta = np.where(np.arange(nb) % 2 == 0, 2.0, 8.0)
    ob = orc.Beads(pos.copy(), mom.copy(), np.ones(nb), zeta, bonds.copy(), 1e-3, 1.0, W, fext.copy())
    db = lat.DeviceBeads(pos, mom, np.ones(nb), zeta, bonds, 1e-3, 1.0, stencil=W, fext=fext)
    return ob, db


@pytest.mark.parametrize("W", [2, 3, 4])
def test_coupled_parity_wide_kernels(orc, lat, W):
    import torch
    rng = np.random.default_rng(W)
    L = 12
    po = orc.Params(nx=L, ny=L, nz=L, kT=1e-4, seed=2, g=(1e-5, 0, -1e-5))
    pd = lat.FluidParams(nx=L, ny=L, nz=L, kT=1e-4, seed=2, body_force=(1e-5, 0, -1e-5))
    n = orc.init_equilibrium(po, u=rng.normal(scale=0.01, size=(3, L, L, L)))
    dev = lat.Lattice(pd)
    dev.set_populations(torch.from_numpy(n))
    n = dev.get_populations().cpu().numpy()
    ob, db = beads_pair(orc, lat, rng, L, W)
    for t in range(20):
        dev.coupled_step(db)
        orc.coupled_step(po, n, t, ob)
    assert np.abs(dev.get_populations().cpu().numpy() - n).max() <= 1e-6
    assert np.abs(db.pos.cpu().numpy() - ob.pos).max() <= 1e-7
    assert np.abs(db.mom.cpu().numpy() - ob.mom).max() <= 1e-7
    dev.close()


@pytest.mark.parametrize("W", [3, 4])
def test_coupled_adjoint_wide_kernels(orc, lat, W):
    import torch
    rng = np.random.default_rng(10 + W)
    L = 10
    po = orc.Params(nx=L, ny=L, nz=L, kT=1e-4, seed=4, g=(1e-4, 0, 2e-5))
    pd = lat.FluidParams(nx=L, ny=L, nz=L, kT=1e-4, seed=4, body_force=(1e-4, 0, 2e-5), track_totals=False)
    n0 = orc.init_equilibrium(po, u=rng.normal(scale=0.02, size=(3, L, L, L)))
    ob, db = beads_pair(orc, lat, rng, L, W, nb=6)
    T = 6
    w = rng.normal(size=n0.shape)
    a, b = rng.normal(size=(6, 3)), rng.normal(size=(6, 3))
    dev = lat.Lattice(pd)
    dev.set_populations(torch.from_numpy(n0))
    n0r = dev.get_populations().cpu().numpy()
    dev.tape_begin(4)
    for _ in range(T):
        dev.coupled_step(db)
    dn0, dg, dR0, dP0 = dev.backward_coupled(torch.from_numpy(w), torch.from_numpy(a), torch.from_numpy(b))
    dev.close()
    lam0, gbar, pb0, mb0 = orc.backward_coupled(po, n0r, T, ob, w, a, b)
    rel = lambda x, y: np.abs(np.asarray(x) - y).max() / np.abs(y).max()
    errs = [rel(dn0.cpu().numpy(), lam0), rel(dg, gbar), rel(dR0.cpu().numpy(), pb0), rel(dP0.cpu().numpy(), mb0)]
    print(W, "wide-kernel coupled adjoint rel errors", ["%.2e" % e for e in errs])
    assert max(errs) <= 2e-5


@pytest.mark.slow
def test_settling_mobility_grid_dependence(lat):
    """The settling experiment of Sec. "Interpolating functions": the radius
    parameter g of eq. aeffcorr (from the steady velocity of a held particle
    of input radius a0 = b) varies with the particle's position relative to
    the grid by up to ~20 % for phi_2, ~3 % for phi_3 and under 1 % for
    phi_4 (the text's figures; the curves themselves are not in the text, so
    the pin is the ordering and these sizes within a factor ~1.5)."""
    from paper_0803_2826_amd.forms import settling_study
    res = settling_study(L=16, steps=2500)
    dev = {W: res[W]["g_max_dev"] for W in (2, 3, 4)}
    print("largest relative deviation of g over 56 grid positions:", {W: round(v, 4) for W, v in dev.items()},
          "mean g:", {W: round(res[W]["g_mean"], 3) for W in (2, 3, 4)})
    assert dev[2] > dev[3] > dev[4]
    assert 0.12 < dev[2] < 0.3
    assert 0.015 < dev[3] < 0.05
    assert dev[4] < 0.015
