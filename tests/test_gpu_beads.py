"""GPU parity of the point-particle coupling against the FP64 oracle, through
the C ABI.  Tolerances: bead positions/momenta 1e-7 absolute (velocities
interpolated from FP32 populations; the spread force summed in fixed point
with 2^-44 resolution and rounded to FP32 where the step reads it);
populations 1e-6 as for the fluid path."""
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


def chains_setup(orc, lat, L, n_chains, length, kT, seed, g=(0.0, 0.0, 0.0), zeta=20.0, k=1.0, p0=0.0,
                 noise="gaussian"):
    """Bead-spring chains.  k = 1 is the stiffest bond (lattice units) for which
    the explicit coupled scheme is stable at zeta = 20, m = 1, h = 1."""
    from paper_0803_2826_amd.inputs import random_walk_chains
    pos, mom, bonds = random_walk_chains(n_chains, length, (L, L, L), seed)
    if p0:
        mom = np.random.default_rng(seed + 1).normal(scale=p0, size=mom.shape)
    nb = pos.shape[0]
    po = orc.Params(nx=L, ny=L, nz=L, kT=kT, seed=seed, g=g)
    pd = lat.FluidParams(nx=L, ny=L, nz=L, kT=kT, seed=seed, body_force=g)
    bo = orc.Beads(pos.copy(), mom.copy(), np.ones(nb), np.full(nb, zeta), bonds.copy(), k, 1.0,
                   three_point=(noise == "three_point"))
    bd = lat.DeviceBeads(pos, mom, np.ones(nb), np.full(nb, zeta), bonds, k, 1.0, noise=noise)
    return po, pd, bo, bd


@pytest.mark.parametrize("kT,noise", [(0.0, "gaussian"), (1e-4, "gaussian"), (1e-4, "three_point")])
def test_coupled_parity(orc, lat, kT, noise):
    """Twenty coupled steps of 4 chains x 8 beads in a 16^3 box, with either
    bead noise (the three-point variates of Sec. "Force coupling" come from
    the same Philox words on both sides, so the noise is identical)."""
    import torch
    L = 16
    po, pd, bo, bd = chains_setup(orc, lat, L, 4, 8, kT, seed=7, g=(1e-5, 0, 0), p0=0.01, noise=noise)
    n = orc.init_equilibrium(po)
    dev = lat.Lattice(pd)
    dev.set_populations(torch.from_numpy(n))
    for t in range(20):
        orc.coupled_step(po, n, t, bo)
        dev.coupled_step(bd)
    got = dev.get_populations().cpu().numpy()
    print("bead pos err", np.abs(bd.pos.cpu().numpy() - bo.pos).max(),
          "mom err", np.abs(bd.mom.cpu().numpy() - bo.mom).max(), "pop err", np.abs(got - n).max())
    np.testing.assert_allclose(bd.pos.cpu().numpy(), bo.pos, atol=1e-7)
    np.testing.assert_allclose(bd.mom.cpu().numpy(), bo.mom, atol=1e-7)
    assert np.abs(got - n).max() <= 1e-6
    dev.close()


def test_total_momentum_with_beads(orc, lat):
    """Fluid + bead momentum grows by exactly N g per coupled step (bond forces
    are pairwise); fluid mass is unchanged."""
    import torch
    L = 20
    g = (1e-5, -2e-5, 0.0)
    po, pd, bo, bd = chains_setup(orc, lat, L, 6, 10, 1e-4, seed=3, g=g)
    dev = lat.Lattice(pd)
    dev.init_equilibrium()
    t0 = np.array(dev.totals(exact=True))
    P0 = bd.mom.sum(0).cpu().numpy()
    for t in range(25):
        dev.coupled_step(bd)
    fused = np.array(dev.totals())
    t1 = np.array(dev.totals(exact=True))
    P1 = bd.mom.sum(0).cpu().numpy()
    N = L ** 3
    assert abs(fused[0] - t1[0]) <= 1e-12 * N
    np.testing.assert_allclose(fused[1:], t1[1:], atol=1e-8 * np.sqrt(N))
    dP = (t1[1:] - t0[1:]) + (P1 - P0)
    # FP32 rounding of the stored populations random-walks the fluid momentum
    # (~2e-8 sqrt(N T)); the bead momenta are FP64
    np.testing.assert_allclose(dP, 25 * N * np.array(g), atol=2e-8 * np.sqrt(N * 25))
    # mass: the FP32 state keeps each site's mass exactly (rest residual plane)
    assert abs(t1[0] - t0[0]) <= 1e-12 * t0[0]
    dev.close()


def test_couple_twice_is_state_error(orc, lat):
    from paper_0803_2826_amd._lib import LB_ESTATE, LBError
    po, pd, bo, bd = chains_setup(orc, lat, 8, 1, 4, 0.0, seed=1)
    dev = lat.Lattice(pd)
    dev.init_equilibrium()
    dev.couple(bd)
    with pytest.raises(LBError) as ei:
        dev.couple(bd)
    assert ei.value.code == LB_ESTATE
    dev.step(1)
    dev.couple(bd)  # allowed again after the step consumed the force
    dev.step(1)
    dev.close()


def test_bead_on_node_and_wrapping(orc, lat):
    """Beads exactly on nodes, on the periodic boundary and far outside the
    box (unwrapped coordinates) agree with the oracle."""
    import torch
    L = 8
    pos = np.array([[0.0, 0.0, 0.0], [7.999999, 3.5, 0.25], [-3.25, 17.5, 8.0], [4.0, 4.0, 4.0]])
    nb = pos.shape[0]
    mom = np.array([[0.01, 0, 0], [0, -0.01, 0], [0, 0, 0.02], [0.003, 0.002, -0.001]])
    po = orc.Params(nx=L, ny=L, nz=L, kT=1e-4, seed=4)
    pd = lat.FluidParams(nx=L, ny=L, nz=L, kT=1e-4, seed=4)
    bo = orc.Beads(pos.copy(), mom.copy(), np.ones(nb), np.full(nb, 5.0))
    bd = lat.DeviceBeads(pos, mom, np.ones(nb), np.full(nb, 5.0))
    rng = np.random.default_rng(0)
    n = orc.init_equilibrium(po, u=rng.normal(scale=0.01, size=(3, L, L, L)))
    dev = lat.Lattice(pd)
    dev.set_populations(torch.from_numpy(n))
    for t in range(10):
        orc.coupled_step(po, n, t, bo)
        dev.coupled_step(bd)
    np.testing.assert_allclose(bd.pos.cpu().numpy(), bo.pos, atol=1e-7)
    np.testing.assert_allclose(bd.mom.cpu().numpy(), bo.mom, atol=1e-7)
    assert np.abs(dev.get_populations().cpu().numpy() - n).max() <= 1e-6
    dev.close()


def test_changing_bead_sets_and_plain_steps(orc, lat):
    """Bead sets of different sizes in consecutive coupled steps (a larger one
    after a smaller one reuses the bond accumulators), plain steps after a
    coupled one (the step consumes the spread force: nothing is left for the
    next step), an external force on one set, all against the oracle."""
    import torch
    from paper_0803_2826_amd.inputs import random_walk_chains
    L, kT = 16, 1e-4
    po = orc.Params(nx=L, ny=L, nz=L, kT=kT, seed=11, g=(0.0, 2e-6, 0.0))
    pd = lat.FluidParams(nx=L, ny=L, nz=L, kT=kT, seed=11, body_force=(0.0, 2e-6, 0.0))
    sets = []
    for n_chains, length, seed in ((6, 10, 1), (2, 5, 2), (6, 10, 3)):
        pos, mom, bonds = random_walk_chains(n_chains, length, (L, L, L), seed)
        nb = pos.shape[0]
        fext = np.random.default_rng(seed).normal(scale=1e-4, size=(nb, 3)) if seed == 2 else None
        sets.append((orc.Beads(pos.copy(), mom.copy(), np.ones(nb), np.full(nb, 5.0), bonds.copy(), 1e-3, 1.0,
                               fext=None if fext is None else fext.copy()),
                     lat.DeviceBeads(pos, mom, np.ones(nb), np.full(nb, 5.0), bonds, 1e-3, 1.0, fext=fext)))
    n = orc.init_equilibrium(po)
    dev = lat.Lattice(pd)
    dev.set_populations(torch.from_numpy(n))
    t = 0
    for rep in range(2):
        for ob, db in sets:
            orc.coupled_step(po, n, t, ob)
            dev.coupled_step(db)
            t += 1
            for _ in range(2):  # plain steps in between
                orc.step(po, n, t)
                t += 1
            dev.step(2)
    got = dev.get_populations().cpu().numpy()
    print("pop err", np.abs(got - n).max())
    assert np.abs(got - n).max() <= 1e-6
    for ob, db in sets:
        np.testing.assert_allclose(db.pos.cpu().numpy(), ob.pos, atol=1e-7)
        np.testing.assert_allclose(db.mom.cpu().numpy(), ob.mom, atol=1e-7)
    dev.close()
