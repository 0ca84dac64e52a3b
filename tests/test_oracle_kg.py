"""Pins of the oracle's bead-spring (Kremer-Grest) interactions: the purely
repulsive Lennard-Jones (WCA) pair potential of eq. ulennardjones and the
FENE bond of eq. ufene, written out here as closed forms; forces must be
minus their gradients (central differences), pair forces must cancel, and
frictionless chains (no momentum exchange with the fluid) integrated with
the half-drift / kick / half-drift scheme of eq. pTrotter must conserve
their energy."""
import numpy as np
import pytest

EPS, SIG = 1e-4, 1.0
K_FENE, R0 = 30 * EPS / SIG ** 2, 1.5 * SIG


def v_wca(r):
    rc = 2 ** (1 / 6) * SIG
    return np.where(r < rc, 4 * EPS * ((SIG / r) ** 12 - (SIG / r) ** 6 + 0.25), 0.0)


def v_fene(r):
    return -0.5 * K_FENE * R0 ** 2 * np.log(1 - r ** 2 / R0 ** 2)


def energy(orc, p, beads, R):
    Lb = np.array([p.nx, p.ny, p.nz], float)
    E = 0.0
    n = R.shape[0]
    for i in range(n):
        for j in range(i + 1, n):
            d = R[j] - R[i]
            d -= Lb * np.floor(d / Lb + 0.5)
            E += float(v_wca(np.linalg.norm(d)))
    for a, b in beads.bonds:
        E += float(v_fene(np.linalg.norm(R[b] - R[a])))
    return E


def kg_beads(orc, pos, bonds, zeta=0.0):
    nb = pos.shape[0]
    return orc.Beads(pos.copy(), np.zeros((nb, 3)), np.ones(nb), np.full(nb, zeta), bonds, K_FENE, R0, fene=True,
                     wca_eps=EPS, wca_sigma=SIG)


def test_forces_are_minus_gradients(orc):
    """Two short chains placed so that beads interact across the periodic
    boundary; forces against central differences of the closed-form energy."""
    p = orc.Params(nx=6, ny=6, nz=6)
    rng = np.random.default_rng(0)
    pos = np.array([[0.3, 1.0, 1.0], [1.2, 1.3, 1.1], [2.0, 1.8, 1.4], [5.5, 1.1, 0.9], [5.6, 2.0, 1.5]])
    pos += rng.normal(scale=0.05, size=pos.shape)
    bonds = np.array([[0, 1], [1, 2], [3, 4]], np.int32)
    b = kg_beads(orc, pos, bonds)
    F = orc.bead_forces(p, b, pos)
    eps = 1e-6
    for k in range(pos.shape[0]):
        for a in range(3):
            Rp, Rm = pos.copy(), pos.copy()
            Rp[k, a] += eps
            Rm[k, a] -= eps
            fd = -(energy(orc, p, b, Rp) - energy(orc, p, b, Rm)) / (2 * eps)
            assert F[k, a] == pytest.approx(fd, rel=1e-6, abs=1e-12)
    # some pairs are inside the WCA range, across the boundary too (0 and 3)
    d03 = pos[3] - pos[0]
    d03 -= 6 * np.round(d03 / 6)
    assert np.linalg.norm(d03) < 2 ** (1 / 6)
    np.testing.assert_allclose(F.sum(0), 0.0, atol=1e-16)


def test_wca_vanishes_smoothly_at_cutoff(orc):
    p = orc.Params(nx=8, ny=8, nz=8)
    rc = 2 ** (1 / 6) * SIG
    for r, expect_zero in ((rc * (1 + 1e-9), True), (rc * (1 - 1e-9), False)):
        b = orc.Beads(np.array([[2.0, 2.0, 2.0], [2.0 + r, 2.0, 2.0]]), np.zeros((2, 3)), np.ones(2), np.zeros(2),
                      np.zeros((0, 2), np.int32), 0.0, 1.0, wca_eps=EPS, wca_sigma=SIG)
        F = orc.bead_forces(p, b, b.pos)
        if expect_zero:
            assert np.abs(F).max() == 0.0
        else:
            # V'(rc) = 0 and V''(rc) = 57.1 eps / sigma^2: |F| ~ 6e-8 eps / sigma here
            assert np.abs(F).max() < 1e-6 * EPS / SIG


def test_fene_overstretch_is_not_finite(orc):
    p = orc.Params(nx=8, ny=8, nz=8)
    b = orc.Beads(np.array([[1.0, 1.0, 1.0], [1.0 + 1.6, 1.0, 1.0]]), np.zeros((2, 3)), np.ones(2), np.zeros(2),
                  np.array([[0, 1]], np.int32), K_FENE, R0, fene=True)
    assert not np.isfinite(orc.bead_forces(p, b, b.pos)).all()


def test_frictionless_chains_conserve_energy(orc):
    """zeta = 0: P'' = P + h F^c and the fluid gets no impulse; the scheme is
    the leapfrog (drift h/2, kick h, drift h/2).  Its energy error is bounded
    and does not drift: the stiffest motion, a bond near its minimum (FENE
    plus WCA curvature ~180 eps / sigma^2, so h omega = 0.13 at m = 1,
    eps = 1e-4), makes the energy fluctuate by ~(h omega)^2 = 2 % of the
    kinetic energy; bounds: 5 % of the initial kinetic energy for the
    fluctuation, 1 % for the drift between the first and last tenth of
    2000 steps.  The momentum is conserved."""
    from paper_0803_2826_amd.inputs import kremer_grest_chains
    L = 6
    p = orc.Params(nx=L, ny=L, nz=L)
    pos, mom, bonds = kremer_grest_chains(3, 8, (L, L, L), seed=1)
    b = kg_beads(orc, pos, bonds)
    rng = np.random.default_rng(2)
    b.mom = rng.normal(scale=np.sqrt(EPS), size=pos.shape)
    b.mom -= b.mom.mean(0)
    n = orc.init_equilibrium(p)
    force = np.zeros((3, L, L, L))

    def total():
        return 0.5 * (b.mom ** 2).sum() + energy(orc, p, b, b.pos)
    E0, P0, mom0 = total(), b.mom.sum(0).copy(), b.mom.copy()
    Es = []
    for t in range(2000):
        orc.couple(p, n, t, b, force)
        if t % 50 == 0:
            Es.append(total())
    # the impulse -(P'' - P - h F^c) is zero up to the rounding of momenta ~1e-2
    assert np.abs(force).max() < 1e-15
    np.testing.assert_allclose(b.mom.sum(0), P0, atol=1e-15)
    Es = np.array(Es)
    ke0 = 0.5 * (mom0 ** 2).sum()
    assert np.abs(Es - E0).max() < 0.05 * ke0
    assert abs(Es[-4:].mean() - Es[:4].mean()) < 0.01 * ke0


def test_wca_does_not_act_through_walls(orc):
    """With walls at z = -1/2 and z = nz - 1/2 the z axis is not periodic:
    beads close to opposite walls, 0.7 apart through the periodic image,
    do not interact; the same pair near the middle does, and its force is
    minus the gradient of the closed-form energy."""
    p = orc.Params(nx=8, ny=8, nz=8, walls=True)
    pos = np.array([[2.0, 2.0, 0.2], [2.1, 2.0, 7.5]])
    b = orc.Beads(pos.copy(), np.zeros((2, 3)), np.ones(2), np.zeros(2), np.zeros((0, 2), np.int32), 0.0, 1.0,
                  wca_eps=EPS, wca_sigma=SIG)
    assert np.abs(orc.bead_forces(p, b, pos)).max() == 0.0
    pp = orc.Params(nx=8, ny=8, nz=8)          # periodic: the image pair interacts
    assert np.abs(orc.bead_forces(pp, b, pos)).max() > 0.0
    mid = np.array([[2.0, 2.0, 3.6], [2.1, 2.0, 4.3]])
    F = orc.bead_forces(p, b, mid)
    r = np.linalg.norm(mid[1] - mid[0])
    e = 1e-6
    dVdr = (v_wca(r + e) - v_wca(r - e)) / (2 * e)
    np.testing.assert_allclose(F[1], -dVdr * (mid[1] - mid[0]) / r, rtol=1e-6)
    np.testing.assert_allclose(F[0], -F[1], rtol=1e-15)
