"""Pins of the oracle's single-site stochastic collision with forcing.

Expected values follow from the paper's statements of what the collision
must do: exact conservation of mass and momentum (the constraints after
eq. LBE and eq. moment_zero/one_external_force), the stress update rule
with force (eq. stress_updaterule_with_force with Sigma from
eq. moment_two_external_force), mode-wise relaxation (eq. lco_update) and the
noise amplitude sqrt(w_k mu rho (1 - gamma_k^2)) of eq. stochupdaterule1 /
eq. detailedbalance1 with the normalisation eq. normalized_mk.
"""
import numpy as np
import pytest


def rand_state(rng, orc, rho=1.0, uscale=0.03, dev=1e-3):
    u = rng.normal(scale=uscale, size=3)
    n = orc.equilibrium(rho, u) + rng.normal(scale=dev, size=19)
    return n


def params(orc, **kw):
    base = dict(nx=4, ny=4, nz=4, kT=0.0)
    base.update(kw)
    return orc.Params(**base)


@pytest.mark.parametrize("kT", [0.0, 1e-4])
def test_mass_and_momentum_change(orc, kT):
    """sum_i Delta_i = 0 and sum_i Delta_i c_i = h f, with and without noise."""
    c, a, e, w = orc.tables()
    rng = np.random.default_rng(10)
    p = params(orc, kT=kT, gamma_shear=0.3, gamma_bulk=-0.2, gamma_3a=0.1, gamma_3b=0.5, gamma_4a=-0.4,
               gamma_4b=0.7)
    for _ in range(30):
        n = rand_state(rng, orc)
        F = rng.normal(scale=1e-3, size=3)
        g = rng.normal(size=16)
        ns = orc.collide_site(p, n, F, g)
        assert (ns - n).sum() == pytest.approx(0.0, abs=1e-15)
        np.testing.assert_allclose((ns - n) @ c.astype(float), F, atol=1e-15)


def test_stress_update_rule_with_force(orc):
    """eq. stress_updaterule_with_force: pi*neq = gamma_s bar(pi neq)
    + gamma_v/3 tr(pi neq) delta + h Sigma, where pi^neq is measured against
    pi^eq = rho c_s^2 delta + rho u u (eq. MBeq2) with u from
    eq. special_choice_momentum_density, and Sigma from
    eq. moment_two_external_force."""
    c, a, e, w = orc.tables()
    cf = c.astype(float)
    rng = np.random.default_rng(11)
    gs, gv = 0.35, -0.25
    p = params(orc, gamma_shear=gs, gamma_bulk=gv, gamma_3a=0.2, gamma_3b=0.1, gamma_4a=0.3, gamma_4b=0.4)
    I3 = np.eye(3)
    for _ in range(30):
        n = rand_state(rng, orc)
        F = rng.normal(scale=1e-3, size=3)
        ns = orc.collide_site(p, n, F)
        rho = n.sum()
        u = (n @ cf + F / 2) / rho
        pieq = rho / 3 * I3 + rho * np.outer(u, u)
        pi = np.einsum("i,ia,ib->ab", n, cf, cf)
        pis = np.einsum("i,ia,ib->ab", ns, cf, cf)
        pneq = pi - pieq
        tr = np.trace(pneq)
        bar = pneq - tr / 3 * I3
        uf = u @ F
        Sig = 0.5 * (1 + gs) * (np.outer(u, F) + np.outer(F, u) - 2 / 3 * uf * I3) + (1 + gv) / 3 * uf * I3
        expect = gs * bar + gv / 3 * tr * I3 + Sig
        np.testing.assert_allclose(pis - pieq, expect, atol=3e-16)


def test_kinetic_modes_relax_with_own_eigenvalue(orc):
    """eq. lco_update for the kinetic groups 10-12, 13-15, 16, 17-18
    (their equilibrium projection is zero), deterministic case."""
    rng = np.random.default_rng(12)
    gam = dict(gamma_3a=0.11, gamma_3b=-0.37, gamma_4a=0.52, gamma_4b=-0.81)
    p = params(orc, gamma_shear=0.2, gamma_bulk=0.1, **gam)
    expect = [gam["gamma_3a"]] * 3 + [gam["gamma_3b"]] * 3 + [gam["gamma_4a"]] + [gam["gamma_4b"]] * 2
    for _ in range(10):
        n = rand_state(rng, orc)
        F = rng.normal(scale=1e-3, size=3)
        m = orc.moments_site(n)
        ms = orc.moments_site(orc.collide_site(p, n, F))
        np.testing.assert_allclose(ms[10:], np.array(expect) * m[10:], atol=1e-16)


def test_bgk_tau1_projects_to_equilibrium(orc):
    """All gamma = 0 and no force: the collision returns n^eq(rho, u)
    (BGK with tau = 1 as the special case of eq. linear_collision_operator)."""
    c, a, e, w = orc.tables()
    rng = np.random.default_rng(13)
    p = params(orc)
    for _ in range(10):
        n = rand_state(rng, orc)
        rho = n.sum()
        u = (n @ c.astype(float)) / rho
        np.testing.assert_allclose(orc.collide_site(p, n), orc.equilibrium(rho, u), atol=1e-16)


@pytest.mark.parametrize("noise_rho0", [False, True])
def test_noise_enters_each_mode_with_fdt_amplitude(orc, noise_rho0):
    """Replay: n*(noise) - n*(no noise) has moments sqrt(w_k mu rho)
    sqrt(1 - gamma_k^2) r_k for k >= 4 and zero for the conserved modes
    (eq. stochupdaterule1, eq. detailedbalance1, eq. normalized_mk,
    mu = kT / c_s^2)."""
    c, a, e, w = orc.tables()
    rng = np.random.default_rng(14)
    kT = 2e-5
    gam = np.array([1, 1, 1, 1, -0.3] + [0.45] * 5 + [0.1] * 3 + [0.2] * 3 + [0.3] + [0.6] * 2)
    p = params(orc, kT=kT, gamma_bulk=gam[4], gamma_shear=gam[5], gamma_3a=gam[10], gamma_3b=gam[13],
               gamma_4a=gam[16], gamma_4b=gam[17], noise_rho0=noise_rho0, rho0=1.0)
    pdet = params(orc, kT=0.0, gamma_bulk=gam[4], gamma_shear=gam[5], gamma_3a=gam[10], gamma_3b=gam[13],
                  gamma_4a=gam[16], gamma_4b=gam[17])
    for _ in range(10):
        n = rand_state(rng, orc, rho=1.0 + 0.1 * rng.normal())
        F = rng.normal(scale=1e-3, size=3)
        g = rng.normal(size=16)
        d = orc.moments_site(orc.collide_site(p, n, F, g) - orc.collide_site(pdet, n, F))
        rho = 1.0 if noise_rho0 else n.sum()
        expect = np.zeros(19)
        expect[4:] = np.sqrt(w[4:] * 3 * kT * rho * (1 - gam[4:] ** 2)) * g[:15]
        np.testing.assert_allclose(d, expect, atol=1e-15)


def test_gamma_one_means_no_relaxation_no_noise(orc):
    """|gamma_k| = 1 leaves the mode untouched and adds no noise
    (phi_k = 0 by eq. detailedbalance3)."""
    rng = np.random.default_rng(15)
    p = params(orc, kT=1e-4, gamma_shear=1.0, gamma_bulk=1.0, gamma_3a=1.0, gamma_3b=1.0, gamma_4a=1.0,
               gamma_4b=1.0)
    n = rand_state(rng, orc)
    np.testing.assert_allclose(orc.collide_site(p, n, np.zeros(3), rng.normal(size=16)), n, atol=1e-16)
