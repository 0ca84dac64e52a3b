"""Pins of the oracle's stationary walls (eq. MBB with the wall at rest,
u_b = 0; walls half way along the links at z = -1/2 and z = nz - 1/2).

Plane Poiseuille flow under a uniform body force g along x has a closed
form for the discrete scheme with odd kinetic modes relaxing at a common
rate (gamma_3a = gamma_3b): the steady momentum density
j(z) = (g / 2 nu)(z + 1/2)(N - 1/2 - z) + (2 g / 3 nu)(Lambda - 3/16),
nu = (1/6)(1 + gamma_s)/(1 - gamma_s), Lambda = (tau_e - 1/2)(tau_o - 1/2),
tau = 1/(1 - gamma) for the shear (even) and odd kinetic rates: the
continuum parabola plus a constant slip that vanishes at Lambda = 3/16
(the two-rate choice Sec. "D3Q19 model II" refers to).  At gamma = 0 this is
3 g (z + 1/2)(N - 1/2 - z) + g/4.
"""
import numpy as np
import pytest


def _two_rate(gamma_e, magic=3 / 16):
    te = 1 / (1 - gamma_e)
    go = 1 - 1 / (0.5 + magic / (te - 0.5))
    return dict(gamma_shear=gamma_e, gamma_bulk=gamma_e, gamma_4a=gamma_e, gamma_4b=gamma_e, gamma_3a=go, gamma_3b=go)


POISEUILLE = {
    "gamma0": {},
    "tau0.8_ghosts0": dict(gamma_shear=-0.25, gamma_bulk=-0.25),
    "two_rate_0.3": _two_rate(0.3),
    "two_rate_-0.25": _two_rate(-0.25),
    "two_rate_0.3_Lambda0.25": _two_rate(0.3, magic=0.25),
    "odd0.5_even-0.1": dict(gamma_shear=-0.1, gamma_bulk=0.2, gamma_3a=0.5, gamma_3b=0.5, gamma_4a=-0.3, gamma_4b=0.1),
}


@pytest.mark.parametrize("name", list(POISEUILLE))
def test_poiseuille_closed_form(orc, name):
    kw = POISEUILLE[name]
    N, g = 16, 1e-5
    p = orc.Params(nx=2, ny=3, nz=N, g=(g, 0, 0), walls=True, **kw)
    gs = p.gamma_shear
    nu = (1 / 6) * (1 + gs) / (1 - gs)
    te, to = 1 / (1 - gs), 1 / (1 - p.gamma_3a)
    lam = (te - 0.5) * (to - 0.5)
    z = np.arange(N)
    expect = g / (2 * nu) * (z + 0.5) * (N - 0.5 - z) + 2 * g / (3 * nu) * (lam - 3 / 16)
    u0 = np.zeros((3, N, 3, 2))
    u0[0] = (g / (2 * nu) * (z + 0.5) * (N - 0.5 - z))[:, None, None]
    n = orc.init_equilibrium(p, u=u0)
    orc.run(p, n, 8000)
    rho, u = orc.fields(p, n)
    j = (u[0] * rho)[:, 0, 0]
    err = np.abs(j - expect).max() / expect.max()
    print(name, "Lambda", lam, "rel err", err)
    assert err < 1e-10
    # uniform across the periodic x, y directions; no transverse flow (FP64
    # rounding on a flow of 1e-4)
    assert np.abs(u[0] - u[0][:, :1, :1]).max() < 1e-13
    assert np.abs(u[1:]).max() < 1e-13


def test_walls_conserve_mass_with_noise(orc):
    rng = np.random.default_rng(0)
    p = orc.Params(nx=6, ny=5, nz=7, kT=1e-4, seed=3, g=(1e-4, 2e-5, -3e-5), walls=True, gamma_shear=0.2)
    n = orc.init_equilibrium(p, u=rng.normal(scale=0.02, size=(3, 7, 5, 6)))
    m0 = n.sum()
    orc.run(p, n, 200)
    assert abs(n.sum() - m0) <= 1e-12 * m0


def test_wall_momentum_exchange(orc):
    """At rest with walls and no force nothing moves; a body force along z
    (normal to the walls) is balanced by the walls: the fluid stays at rest
    up to the hydrostatic density gradient, with zero steady momentum."""
    p = orc.Params(nx=2, ny=2, nz=12, walls=True)
    n = orc.init_equilibrium(p)
    ref = n.copy()
    orc.run(p, n, 50)
    assert np.abs(n - ref).max() < 1e-16
    p = orc.Params(nx=2, ny=2, nz=12, walls=True, g=(0, 0, 1e-5))
    n = orc.init_equilibrium(p)
    orc.run(p, n, 4000)
    rho, u = orc.fields(p, n)
    assert np.abs(u).max() < 1e-12
    # hydrostatic balance c_s^2 d rho / dz = g: rho grows linearly along +z
    drho = np.diff(rho[:, 0, 0])
    np.testing.assert_allclose(drho, 3 * 1e-5, rtol=1e-6)


def test_step_adjoint_with_walls_matches_finite_differences(orc):
    rng = np.random.default_rng(1)
    p = orc.Params(nx=3, ny=4, nz=5, kT=1e-4, seed=7, g=(1e-4, -2e-4, 5e-5), gamma_shear=0.2, gamma_bulk=0.1,
                   gamma_3a=-0.1, gamma_3b=0.3, gamma_4a=0.2, gamma_4b=-0.4, walls=True)
    n0 = orc.init_equilibrium(p, u=rng.normal(scale=0.02, size=(3, 5, 4, 3)))
    T = 6
    w = rng.normal(size=n0.shape)
    lam0, gbar = orc.backward(p, n0, T, w)
    eps = 1e-6

    def run(pp, x):
        y = x.copy()
        orc.run(pp, y, T)
        return (w * y).sum()
    for _ in range(3):
        v = rng.normal(size=n0.shape)
        fd = (run(p, n0 + eps * v) - run(p, n0 - eps * v)) / (2 * eps)
        assert (lam0 * v).sum() == pytest.approx(fd, rel=1e-6)
    for a in range(3):
        gp, gm = list(p.g), list(p.g)
        gp[a] += eps
        gm[a] -= eps
        fd = (run(orc.Params(**{**p.__dict__, "g": tuple(gp)}), n0) -
              run(orc.Params(**{**p.__dict__, "g": tuple(gm)}), n0)) / (2 * eps)
        assert gbar[a] == pytest.approx(fd, rel=1e-6)
