"""Stationary mid-link walls on the GPU (lb_params.walls = 1: walls at
z = -1/2 and z = nz - 1/2, eq. MBB with the wall at rest), against the FP64
oracle with the same walls (pinned by plane Poiseuille flow) and against the
Poiseuille closed form.

Tolerances as for the periodic box: populations 1e-6 absolute after the
run (FP32 arithmetic on shifted populations, noise amplitude <= 1.1e-2 with
hardware transcendentals); the Poiseuille profile to 3e-5 relative: every
step adds g = 1e-5 to momentum densities of up to 5e-4 held in FP32, a
rounding of ~6e-11 per increment that random-walks over the ~1500-step
viscous relaxation time of the channel (~3e-9, 6e-6 relative); the adjoint
to 2e-5 relative to its largest entry.
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


def pair(orc, lat, nx, ny, nz, **kw):
    po = orc.Params(nx=nx, ny=ny, nz=nz, walls=True, **kw)
    pd = lat.FluidParams(nx=nx, ny=ny, nz=nz, walls=True, kT=po.kT, seed=po.seed, body_force=po.g,
                         gamma_shear=po.gamma_shear, gamma_bulk=po.gamma_bulk, gamma_3a=po.gamma_3a,
                         gamma_3b=po.gamma_3b, gamma_4a=po.gamma_4a, gamma_4b=po.gamma_4b, track_totals=False)
    return po, pd


def test_walls_parity_with_noise_and_general_relaxation(orc, lat):
    import torch
    rng = np.random.default_rng(0)
    po, pd = pair(orc, lat, 12, 10, 8, kT=1e-4, seed=4, g=(1e-4, -5e-5, 3e-5), gamma_shear=0.2, gamma_bulk=-0.1,
                  gamma_3a=0.3, gamma_3b=-0.2, gamma_4a=0.1, gamma_4b=0.4)
    n = orc.init_equilibrium(po, u=rng.normal(scale=0.02, size=(3, 8, 10, 12)))
    dev = lat.Lattice(pd)
    dev.set_populations(torch.from_numpy(n))
    n = dev.get_populations().cpu().numpy()
    orc.run(po, n, 60)
    dev.step(60)
    got = dev.get_populations().cpu().numpy()
    err = np.abs(got - n).max()
    print("walls parity after 60 steps", err)
    assert err <= 1e-6
    rho, u = dev.moments()
    rr, uu = orc.fields(po, n)
    assert np.abs(rho.cpu().numpy() - rr).max() <= 1e-6
    assert np.abs(u.cpu().numpy() - uu).max() <= 1e-5
    dev.close()


def test_set_get_roundtrip_with_walls(orc, lat):
    import torch
    rng = np.random.default_rng(1)
    po, pd = pair(orc, lat, 6, 5, 7)
    n = orc.init_equilibrium(po, u=rng.normal(scale=0.05, size=(3, 7, 5, 6))) + rng.normal(scale=1e-3,
                                                                                          size=(19, 7, 5, 6))
    dev = lat.Lattice(pd)
    dev.set_populations(torch.from_numpy(n))
    assert np.abs(dev.get_populations().cpu().numpy() - n).max() <= 1e-8
    u = rng.normal(scale=0.02, size=(3, 7, 5, 6))
    dev.init_equilibrium(u=torch.from_numpy(u).cuda())
    np.testing.assert_allclose(dev.get_populations().cpu().numpy(), orc.init_equilibrium(po, u=u), atol=1e-8)
    dev.close()


@pytest.mark.parametrize("relax", ["gamma0", "two_rate_0.3"])
def test_gpu_poiseuille_closed_form(orc, lat, relax):
    import torch
    kw = {} if relax == "gamma0" else lat.two_rate(0.3)
    N, g = 16, 1e-5
    pd = lat.FluidParams(nx=2, ny=3, nz=N, walls=True, body_force=(g, 0, 0), track_totals=True, **kw)
    gs = pd.gamma_shear
    nu = (1 / 6) * (1 + gs) / (1 - gs)
    lam = (1 / (1 - gs) - 0.5) * (1 / (1 - pd.gamma_3a) - 0.5)
    z = np.arange(N)
    expect = g / (2 * nu) * (z + 0.5) * (N - 0.5 - z) + 2 * g / (3 * nu) * (lam - 3 / 16)
    u0 = np.zeros((3, N, 3, 2))
    u0[0] = (g / (2 * nu) * (z + 0.5) * (N - 0.5 - z))[:, None, None]
    dev = lat.Lattice(pd)
    dev.init_equilibrium(u=torch.from_numpy(u0).cuda())
    m0 = dev.totals(exact=True)[0]
    dev.step(8000)
    rho, u = dev.moments()
    j = (u[0] * rho).cpu().numpy()[:, 0, 0]
    err = np.abs(j - expect).max() / expect.max()
    print(relax, "GPU Poiseuille rel err", err)
    assert err < 3e-5
    assert abs(dev.totals(exact=True)[0] - m0) <= 1e-9 * m0
    dev.close()


def test_gpu_adjoint_with_walls_matches_oracle(orc, lat):
    import torch
    rng = np.random.default_rng(2)
    po, pd = pair(orc, lat, 8, 6, 10, kT=1e-4, seed=6, g=(1e-4, 2e-5, -4e-5), gamma_shear=0.1, gamma_3a=0.2)
    n0 = orc.init_equilibrium(po, u=rng.normal(scale=0.02, size=(3, 10, 6, 8)))
    T = 10
    w = rng.normal(size=n0.shape)
    dev = lat.Lattice(pd)
    dev.set_populations(torch.from_numpy(n0))
    n0r = dev.get_populations().cpu().numpy()
    dev.tape_begin(4)
    dev.step(T)
    dn0, dg = dev.backward(torch.from_numpy(w))
    dev.close()
    ref, gref = orc.backward(po, n0r, T, w)
    err = np.abs(dn0.cpu().numpy() - ref).max() / np.abs(ref).max()
    print("adjoint with walls rel err", err)
    assert err <= 2e-5
    np.testing.assert_allclose(dg, gref, rtol=2e-4)


def test_coupled_parity_with_walls(orc, lat):
    """Beads kept inside the channel (stencil within 0 <= z <= nz - 1)."""
    import torch
    rng = np.random.default_rng(3)
    po, pd = pair(orc, lat, 12, 12, 14, kT=1e-4, seed=8, g=(2e-5, 0, 0))
    pos = np.column_stack([rng.uniform(0, 12, 16), rng.uniform(0, 12, 16), rng.uniform(4, 9, 16)])
    nb = pos.shape[0]
    mom = np.zeros((nb, 3))
    bonds = np.array([[k, k + 1] for k in range(0, nb - 1, 2)], dtype=np.int32)
    n = orc.init_equilibrium(po)
    dev = lat.Lattice(pd)
    dev.set_populations(torch.from_numpy(n))
    db = lat.DeviceBeads(pos, mom, np.ones(nb), np.full(nb, 5.0), bonds, 1e-3, 1.0)
    ob = orc.Beads(pos.copy(), mom.copy(), np.ones(nb), np.full(nb, 5.0), bonds.copy(), 1e-3, 1.0)
    for t in range(20):
        dev.coupled_step(db)
        orc.coupled_step(po, n, t, ob)
    assert np.abs(dev.get_populations().cpu().numpy() - n).max() <= 1e-6
    assert np.abs(db.pos.cpu().numpy() - ob.pos).max() <= 1e-7
    assert np.abs(db.mom.cpu().numpy() - ob.mom).max() <= 1e-7
    dev.close()


@pytest.mark.parametrize("K", [4, 0])
def test_coupled_adjoint_with_walls_matches_oracle(orc, lat, K):
    """Taped coupled steps in a channel (beads kept off the walls): the
    reverse sweep with the walls' reflected adjoint and the particle
    adjoint, against the oracle's FP64 adjoint of whole coupled steps;
    checkpoints every 4 steps, and a moments tape (K = 0)."""
    import torch
    rng = np.random.default_rng(5)
    po, pd = pair(orc, lat, 10, 8, 12, kT=1e-4, seed=3, g=(1e-4, 0.0, -2e-5), gamma_shear=0.1)
    n0 = orc.init_equilibrium(po, u=rng.normal(scale=0.02, size=(3, 12, 8, 10)))
    nb = 12
    pos = np.column_stack([rng.uniform(0, 10, nb), rng.uniform(0, 8, nb), rng.uniform(3.5, 7.5, nb)])
    mom = rng.normal(scale=0.01, size=(nb, 3))
    bonds = np.array([[k, k + 1] for k in range(0, nb - 1, 2)], dtype=np.int32)
    zeta = np.full(nb, 1.0)
    ob = orc.Beads(pos.copy(), mom.copy(), np.ones(nb), zeta, bonds.copy(), 1e-3, 1.0)
    db = lat.DeviceBeads(pos, mom, np.ones(nb), zeta, bonds, 1e-3, 1.0)
    T = 6
    w = rng.normal(size=n0.shape)
    a, b = rng.normal(size=(nb, 3)), rng.normal(size=(nb, 3))
    dev = lat.Lattice(pd)
    dev.set_populations(torch.from_numpy(n0))
    n0r = dev.get_populations().cpu().numpy()
    dev.tape_begin(K)
    for _ in range(T):
        dev.coupled_step(db)
    dn0, dg, dR0, dP0 = dev.backward_coupled(torch.from_numpy(w), torch.from_numpy(a), torch.from_numpy(b))
    dev.close()
    lam0, gbar, pb0, mb0 = orc.backward_coupled(po, n0r, T, ob, w, a, b)

    def rel(x, ref):
        return np.abs(np.asarray(x) - ref).max() / np.abs(ref).max()

    errs = [rel(dn0.cpu().numpy(), lam0), rel(dg, gbar), rel(dR0.cpu().numpy(), pb0), rel(dP0.cpu().numpy(), mb0)]
    print("coupled adjoint with walls rel errors (n0, g, R0, P0):", ["%.2e" % e for e in errs])
    assert max(errs) <= 2e-5


def test_batch_rejects_walls(lat):
    from paper_0803_2826_amd._lib import LB_EINVAL, LB_EUNSUPPORTED, LBError
    with pytest.raises(LBError) as ei:
        lat.BatchLattice(lat.FluidParams(nx=2, ny=2, nz=2, walls=True), [(8, 8, 8)])
    assert ei.value.code == LB_EUNSUPPORTED
    p = lat.FluidParams(nx=8, ny=8, nz=8)
    c = p.to_c()
    c.walls = 2
    from paper_0803_2826_amd import _lib
    import ctypes
    import torch
    L = _lib.load()
    ctx = ctypes.c_void_p()
    rc = L.lb_create(ctypes.byref(c), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream), ctypes.byref(ctx))
    assert rc == LB_EINVAL
