"""Pins of the oracle's hand-written adjoint against central finite
differences of the oracle's own forward map (FP64, eps = 1e-6, truncation
O(eps^2)); the loss is a random linear functional of the final populations
or the kinetic energy in a probe region (the loss of the differentiation
form: mean |u|^2 over a sub-box, u = (sum n c + g/2)/rho)."""
import numpy as np
import pytest


def test_collision_adjoint_is_transpose_of_jacobian(orc):
    rng = np.random.default_rng(0)
    p = orc.Params(nx=4, ny=4, nz=4, kT=1e-4, gamma_shear=0.3, gamma_bulk=-0.2, gamma_3a=0.1, gamma_3b=0.4,
                   gamma_4a=-0.3, gamma_4b=0.6)
    eps = 1e-6
    for noise_rho0 in (False, True):
        p.noise_rho0 = noise_rho0
        for _ in range(10):
            n = orc.equilibrium(1 + 0.05 * rng.normal(), rng.normal(scale=0.03, size=3)) + rng.normal(scale=1e-3,
                                                                                                        size=19)
            F = rng.normal(scale=1e-3, size=3)
            g = rng.normal(size=16)
            w = rng.normal(size=19)
            v = rng.normal(size=19)
            vF = rng.normal(size=3)
            nb, Fb = orc.collide_site_adjoint(p, n, F, g, w)
            fd = (w @ orc.collide_site(p, n + eps * v, F, g) - w @ orc.collide_site(p, n - eps * v, F, g)) / (2 * eps)
            assert nb @ v == pytest.approx(fd, rel=1e-7, abs=1e-10)
            fdF = (w @ orc.collide_site(p, n, F + eps * vF, g) - w @ orc.collide_site(p, n, F - eps * vF, g)) / (2 * eps)
            assert Fb @ vF == pytest.approx(fdF, rel=1e-7, abs=1e-10)


def _run(orc, p, n0, T):
    n = n0.copy()
    orc.run(p, n, T)
    return n


@pytest.mark.parametrize("noise_rho0", [False, True])
def test_backward_matches_finite_differences_linear_loss(orc, noise_rho0):
    rng = np.random.default_rng(1)
    p = orc.Params(nx=3, ny=4, nz=5, kT=1e-4, seed=7, g=(1e-4, -2e-4, 5e-5), gamma_shear=0.2, gamma_bulk=0.1,
                   gamma_3a=-0.1, gamma_3b=0.3, gamma_4a=0.2, gamma_4b=-0.4, noise_rho0=noise_rho0)
    n0 = orc.init_equilibrium(p, u=rng.normal(scale=0.02, size=(3, 5, 4, 3)))
    T = 6
    w = rng.normal(size=n0.shape)
    lam0, gbar = orc.backward(p, n0, T, w)
    eps = 1e-6
    for _ in range(3):
        v = rng.normal(size=n0.shape)
        fd = ((w * _run(orc, p, n0 + eps * v, T)).sum() - (w * _run(orc, p, n0 - eps * v, T)).sum()) / (2 * eps)
        assert (lam0 * v).sum() == pytest.approx(fd, rel=1e-6)
    for a in range(3):
        gp, gm = list(p.g), list(p.g)
        gp[a] += eps
        gm[a] -= eps
        pp = orc.Params(**{**p.__dict__, "g": tuple(gp)})
        pm = orc.Params(**{**p.__dict__, "g": tuple(gm)})
        fd = ((w * _run(orc, pp, n0, T)).sum() - (w * _run(orc, pm, n0, T)).sum()) / (2 * eps)
        assert gbar[a] == pytest.approx(fd, rel=1e-6)


def probe_loss(orc, p, n, lo, hi):
    rho, u = orc.fields(p, n)
    sl = (slice(None), slice(lo, hi), slice(lo, hi), slice(lo, hi))
    return (u[sl] ** 2).sum(axis=0).mean()


def probe_loss_grad(orc, p, n, lo, hi):
    """dL/dn of L = mean over the probe of |u|^2 (u = J/rho, J = sum n c + g/2):
    dL/dn_i = (2/P)(u.c_i - |u|^2)/rho, and dL/dg = (1/P) sum u/rho."""
    c, a, e, w = orc.tables()
    rho, u = orc.fields(p, n)
    mask = np.zeros(rho.shape, bool)
    mask[lo:hi, lo:hi, lo:hi] = True
    P = mask.sum()
    uc = np.einsum("ia,azyx->izyx", c.astype(float), u)
    usq = (u ** 2).sum(axis=0)
    grad = 2.0 / P * (uc - usq) / rho * mask
    gdir = (u / rho * mask).sum(axis=(1, 2, 3)) / P
    return grad, gdir


def test_backward_probe_kinetic_energy_loss(orc):
    rng = np.random.default_rng(2)
    L = 6
    p = orc.Params(nx=L, ny=L, nz=L, kT=1e-4, seed=3, g=(2e-4, 0.0, -1e-4))
    n0 = orc.init_equilibrium(p, u=rng.normal(scale=0.02, size=(3, L, L, L)))
    T = 8
    lo, hi = 2, 4
    nT = _run(orc, p, n0, T)
    lamT, g_direct = probe_loss_grad(orc, p, nT, lo, hi)
    lam0, gbar = orc.backward(p, n0, T, lamT)
    gbar = gbar + g_direct
    eps = 1e-6
    v = rng.normal(size=n0.shape)
    fd = (probe_loss(orc, p, _run(orc, p, n0 + eps * v, T), lo, hi) -
          probe_loss(orc, p, _run(orc, p, n0 - eps * v, T), lo, hi)) / (2 * eps)
    assert (lam0 * v).sum() == pytest.approx(fd, rel=1e-6)
    for a in range(3):
        gp, gm = list(p.g), list(p.g)
        gp[a] += eps
        gm[a] -= eps
        pp = orc.Params(**{**p.__dict__, "g": tuple(gp)})
        pm = orc.Params(**{**p.__dict__, "g": tuple(gm)})
        fd = (probe_loss(orc, pp, _run(orc, pp, n0, T), lo, hi) - probe_loss(orc, pm, _run(orc, pm, n0, T), lo, hi)) / (
            2 * eps)
        assert gbar[a] == pytest.approx(fd, rel=1e-5, abs=1e-12)


def _bead_system(orc, rng, L=(8, 7, 6), chains=2, length=3, zeta=(0.5, 2.0)):
    """Chains of unit-ish bonds placed well inside the box, positions kept at
    least 0.05 away from the node planes so that the stencil weights are
    differentiable along the finite-difference path."""
    nb = chains * length
    pos = np.zeros((nb, 3))
    for c in range(chains):
        start = rng.uniform(1.0, min(L) - 3.0, size=3)
        for k in range(length):
            pos[c * length + k] = start + np.array([0.9 * k, 0.3 * k, 0.2 * k])
    frac = pos - np.floor(pos)
    pos = np.floor(pos) + np.clip(frac, 0.05, 0.95)
    mom = rng.normal(scale=0.01, size=(nb, 3))
    bonds = np.array([[c * length + k, c * length + k + 1] for c in range(chains) for k in range(length - 1)],
                     dtype=np.int32)
    z = np.array([zeta[b % len(zeta)] for b in range(nb)])
    return orc.Beads(pos, mom, np.ones(nb), z, bonds, 0.05, 1.0)


def test_couple_adjoint_matches_finite_differences(orc):
    """One particle half-step (interpolation, OU update, bonds, spreading):
    the adjoint w.r.t. n, g, R, P of L = wf.force + a.R_new + b.P_new."""
    rng = np.random.default_rng(5)
    p = orc.Params(nx=8, ny=7, nz=6, kT=1e-4, seed=4, g=(1e-4, -5e-5, 2e-5))
    n = orc.init_equilibrium(p, u=rng.normal(scale=0.02, size=(3, 6, 7, 8)))
    beads = _bead_system(orc, rng)
    nb = beads.pos.shape[0]
    wf = rng.normal(size=(3, 6, 7, 8))
    a, b = rng.normal(size=(nb, 3)), rng.normal(size=(nb, 3))

    def loss(nn, pp, bb):
        force = np.zeros((3, 6, 7, 8))
        c = bb.copy()
        orc.couple(pp, nn, 3, c, force)
        return (wf * force).sum() + (a * c.pos).sum() + (b * c.mom).sum()

    lam = np.zeros_like(n)
    gbar = np.zeros(3)
    pb, mb = a.copy(), b.copy()
    orc.couple_adjoint(p, n, 3, beads, wf, pb, mb, lam, gbar)
    eps = 1e-6
    v = rng.normal(size=n.shape)
    fd = (loss(n + eps * v, p, beads) - loss(n - eps * v, p, beads)) / (2 * eps)
    assert (lam * v).sum() == pytest.approx(fd, rel=1e-6, abs=1e-12)
    for name, bar in (("pos", pb), ("mom", mb)):
        vb = rng.normal(size=(nb, 3))
        bp_, bm_ = beads.copy(), beads.copy()
        setattr(bp_, name, getattr(beads, name) + eps * vb)
        setattr(bm_, name, getattr(beads, name) - eps * vb)
        fd = (loss(n, p, bp_) - loss(n, p, bm_)) / (2 * eps)
        assert (bar * vb).sum() == pytest.approx(fd, rel=1e-6, abs=1e-12), name
    for k in range(3):
        gp, gm = list(p.g), list(p.g)
        gp[k] += eps
        gm[k] -= eps
        pp = orc.Params(**{**p.__dict__, "g": tuple(gp)})
        pm = orc.Params(**{**p.__dict__, "g": tuple(gm)})
        fd = (loss(n, pp, beads) - loss(n, pm, beads)) / (2 * eps)
        assert gbar[k] == pytest.approx(fd, rel=1e-6, abs=1e-12)


def test_coupled_backward_matches_finite_differences(orc):
    """Whole coupled steps (particles + fluid with the spread force): the
    adjoint w.r.t. n(0), g, R(0), P(0) of L = w.n(T) + a.R(T) + b.P(T)."""
    rng = np.random.default_rng(6)
    p = orc.Params(nx=8, ny=7, nz=6, kT=1e-4, seed=8, g=(1e-4, -5e-5, 2e-5), gamma_shear=0.2, gamma_bulk=-0.1)
    n0 = orc.init_equilibrium(p, u=rng.normal(scale=0.02, size=(3, 6, 7, 8)))
    beads = _bead_system(orc, rng)
    nb = beads.pos.shape[0]
    T = 4
    w = rng.normal(size=n0.shape)
    a, b = rng.normal(size=(nb, 3)), rng.normal(size=(nb, 3))

    def loss(nn, pp, bb):
        n = nn.copy()
        c = bb.copy()
        for t in range(T):
            orc.coupled_step(pp, n, t, c)
        return (w * n).sum() + (a * c.pos).sum() + (b * c.mom).sum()

    lam0, gbar, pb0, mb0 = orc.backward_coupled(p, n0, T, beads, w, a, b)
    eps = 1e-6
    v = rng.normal(size=n0.shape)
    fd = (loss(n0 + eps * v, p, beads) - loss(n0 - eps * v, p, beads)) / (2 * eps)
    assert (lam0 * v).sum() == pytest.approx(fd, rel=1e-6)
    for name, bar in (("pos", pb0), ("mom", mb0)):
        vb = rng.normal(size=(nb, 3))
        bp_, bm_ = beads.copy(), beads.copy()
        setattr(bp_, name, getattr(beads, name) + eps * vb)
        setattr(bm_, name, getattr(beads, name) - eps * vb)
        fd = (loss(n0, p, bp_) - loss(n0, p, bm_)) / (2 * eps)
        assert (bar * vb).sum() == pytest.approx(fd, rel=1e-6), name
    for k in range(3):
        gp, gm = list(p.g), list(p.g)
        gp[k] += eps
        gm[k] -= eps
        pp = orc.Params(**{**p.__dict__, "g": tuple(gp)})
        pm = orc.Params(**{**p.__dict__, "g": tuple(gm)})
        fd = (loss(n0, pp, beads) - loss(n0, pm, beads)) / (2 * eps)
        assert gbar[k] == pytest.approx(fd, rel=1e-6)


def _kg_system(orc, rng, L):
    """Four Kremer-Grest chains of 8 (FENE + WCA at eps = 1e-3, sigma = 1): bonded
    neighbours sit at 0.97, inside the WCA range, and a few unbonded pairs
    too."""
    from paper_0803_2826_amd.inputs import kremer_grest_chains
    pos, _, bonds = kremer_grest_chains(4, 8, L, seed=int(rng.integers(1 << 30)))
    nb = pos.shape[0]
    eps = 1e-3
    return orc.Beads(pos, rng.normal(scale=0.01, size=(nb, 3)), np.ones(nb), np.full(nb, 0.5), bonds, 30 * eps, 1.5,
                     fene=True, wca_eps=eps, wca_sigma=1.0)


def test_kg_couple_adjoint_matches_finite_differences(orc):
    """One particle half-step with FENE bonds and WCA pairs: the adjoint
    w.r.t. n, g, R, P of L = wf.force + a.R_new + b.P_new (central
    differences, eps = 1e-6; no pair lies within 1e-5 of the WCA cutoff,
    where the force's derivative jumps)."""
    rng = np.random.default_rng(15)
    dims = (8, 8, 8)
    p = orc.Params(nx=8, ny=8, nz=8, kT=1e-4, seed=4, g=(1e-4, -5e-5, 2e-5))
    n = orc.init_equilibrium(p, u=rng.normal(scale=0.02, size=(3, 8, 8, 8)))
    beads = _kg_system(orc, rng, dims)
    nb = beads.pos.shape[0]
    half = beads.pos + 0.5 * beads.mom
    dd = half[:, None, :] - half[None, :, :]
    dd -= 8 * np.round(dd / 8)
    r = np.linalg.norm(dd, axis=2)
    assert np.abs(r[np.triu_indices(nb, 1)] - 2 ** (1 / 6)).min() > 1e-5
    assert (r[np.triu_indices(nb, 1)] < 2 ** (1 / 6)).sum() > len(beads.bonds)   # unbonded pairs interact too
    wf = rng.normal(size=(3, 8, 8, 8))
    a, b = rng.normal(size=(nb, 3)), rng.normal(size=(nb, 3))

    def loss(nn, pp, bb):
        force = np.zeros((3, 8, 8, 8))
        c = bb.copy()
        orc.couple(pp, nn, 3, c, force)
        return (wf * force).sum() + (a * c.pos).sum() + (b * c.mom).sum()

    lam = np.zeros_like(n)
    gbar = np.zeros(3)
    pb, mb = a.copy(), b.copy()
    orc.couple_adjoint(p, n, 3, beads, wf, pb, mb, lam, gbar)
    eps = 1e-6
    for name, bar in (("pos", pb), ("mom", mb)):
        vb = rng.normal(size=(nb, 3))
        bp_, bm_ = beads.copy(), beads.copy()
        setattr(bp_, name, getattr(beads, name) + eps * vb)
        setattr(bm_, name, getattr(beads, name) - eps * vb)
        fd = (loss(n, p, bp_) - loss(n, p, bm_)) / (2 * eps)
        assert (bar * vb).sum() == pytest.approx(fd, rel=1e-6, abs=1e-12), name
    v = rng.normal(size=n.shape)
    fd = (loss(n + eps * v, p, beads) - loss(n - eps * v, p, beads)) / (2 * eps)
    assert (lam * v).sum() == pytest.approx(fd, rel=1e-6, abs=1e-12)


def test_kg_coupled_backward_matches_finite_differences(orc):
    """Whole coupled steps with FENE + WCA chains: the adjoint w.r.t. n(0),
    g, R(0), P(0) of L = w.n(T) + a.R(T) + b.P(T)."""
    rng = np.random.default_rng(16)
    p = orc.Params(nx=8, ny=8, nz=8, kT=1e-4, seed=8, g=(1e-4, -5e-5, 2e-5))
    n0 = orc.init_equilibrium(p, u=rng.normal(scale=0.02, size=(3, 8, 8, 8)))
    beads = _kg_system(orc, rng, (8, 8, 8))
    nb = beads.pos.shape[0]
    T = 4
    w = rng.normal(size=n0.shape)
    a, b = rng.normal(size=(nb, 3)), rng.normal(size=(nb, 3))

    def loss(nn, pp, bb):
        n = nn.copy()
        c = bb.copy()
        for t in range(T):
            orc.coupled_step(pp, n, t, c)
        return (w * n).sum() + (a * c.pos).sum() + (b * c.mom).sum()

    lam0, gbar, pb0, mb0 = orc.backward_coupled(p, n0, T, beads, w, a, b)
    eps = 1e-6
    for name, bar in (("pos", pb0), ("mom", mb0)):
        vb = rng.normal(size=(nb, 3))
        bp_, bm_ = beads.copy(), beads.copy()
        setattr(bp_, name, getattr(beads, name) + eps * vb)
        setattr(bm_, name, getattr(beads, name) - eps * vb)
        fd = (loss(n0, p, bp_) - loss(n0, p, bm_)) / (2 * eps)
        assert (bar * vb).sum() == pytest.approx(fd, rel=1e-6), name
    v = rng.normal(size=n0.shape)
    fd = (loss(n0 + eps * v, p, beads) - loss(n0 - eps * v, p, beads)) / (2 * eps)
    assert (lam0 * v).sum() == pytest.approx(fd, rel=1e-6)
    gp, gm = list(p.g), list(p.g)
    gp[0] += eps
    gm[0] -= eps
    pp = orc.Params(**{**p.__dict__, "g": tuple(gp)})
    pm = orc.Params(**{**p.__dict__, "g": tuple(gm)})
    fd = (loss(n0, pp, beads) - loss(n0, pm, beads)) / (2 * eps)
    assert gbar[0] == pytest.approx(fd, rel=1e-6)


def test_composed_reverse_sweep_equals_backward_coupled(orc):
    """The oracle's step and particle adjoints, composed by hand step by step,
    give the same gradients as orc_backward_coupled (the composition used by
    the GPU tests of mixed tapes)."""
    rng = np.random.default_rng(7)
    p = orc.Params(nx=8, ny=7, nz=6, kT=1e-4, seed=2, g=(1e-4, 0.0, 3e-5))
    n0 = orc.init_equilibrium(p, u=rng.normal(scale=0.02, size=(3, 6, 7, 8)))
    beads = _bead_system(orc, rng)
    nb = beads.pos.shape[0]
    T = 3
    w = rng.normal(size=n0.shape)
    a, b = rng.normal(size=(nb, 3)), rng.normal(size=(nb, 3))
    ref = orc.backward_coupled(p, n0, T, beads, w, a, b)
    states, bstates = [n0.copy()], [beads.copy()]
    n, bb = n0.copy(), beads.copy()
    for t in range(T):
        orc.coupled_step(p, n, t, bb)
        states.append(n.copy())
        bstates.append(bb.copy())
    lam, gbar, pb, mb = w.copy(), np.zeros(3), a.copy(), b.copy()
    for t in range(T - 1, -1, -1):
        force = np.zeros((3, 6, 7, 8))
        orc.couple(p, states[t], t, bstates[t].copy(), force)
        fbar = np.zeros((3, 6, 7, 8))
        orc.step_adjoint(p, states[t], lam, t, gbar, extra_force=force, extra_bar=fbar)
        orc.couple_adjoint(p, states[t], t, bstates[t], fbar, pb, mb, lam, gbar)
    for x, y in zip((lam, gbar, pb, mb), ref):
        np.testing.assert_allclose(x, y, rtol=1e-12, atol=1e-14 * np.abs(y).max())


@pytest.mark.parametrize("W", [3, 4])
def test_coupled_backward_wide_stencils_match_finite_differences(orc, W):
    """The coupled adjoint with the three- and four-point kernels (their
    derivatives enter through the weights) and an external bead force."""
    rng = np.random.default_rng(20 + W)
    p = orc.Params(nx=10, ny=9, nz=8, kT=1e-4, seed=5, g=(1e-4, -5e-5, 2e-5))
    n0 = orc.init_equilibrium(p, u=rng.normal(scale=0.02, size=(3, 8, 9, 10)))
    beads = _bead_system(orc, rng, L=(10, 9, 8))
    beads.stencil = W
    beads.fext = rng.normal(scale=1e-4, size=beads.pos.shape)
    nb = beads.pos.shape[0]
    T = 3
    w = rng.normal(size=n0.shape)
    a, b = rng.normal(size=(nb, 3)), rng.normal(size=(nb, 3))

    def loss(nn, pp, bb):
        n = nn.copy()
        c = bb.copy()
        for t in range(T):
            orc.coupled_step(pp, n, t, c)
        return (w * n).sum() + (a * c.pos).sum() + (b * c.mom).sum()

    lam0, gbar, pb0, mb0 = orc.backward_coupled(p, n0, T, beads, w, a, b)
    eps = 1e-6
    v = rng.normal(size=n0.shape)
    fd = (loss(n0 + eps * v, p, beads) - loss(n0 - eps * v, p, beads)) / (2 * eps)
    assert (lam0 * v).sum() == pytest.approx(fd, rel=1e-6)
    for name, bar in (("pos", pb0), ("mom", mb0)):
        vb = rng.normal(size=(nb, 3))
        bp_, bm_ = beads.copy(), beads.copy()
        setattr(bp_, name, getattr(beads, name) + eps * vb)
        setattr(bm_, name, getattr(beads, name) - eps * vb)
        fd = (loss(n0, p, bp_) - loss(n0, p, bm_)) / (2 * eps)
        assert (bar * vb).sum() == pytest.approx(fd, rel=1e-6), name


def test_c5_references_agree():
    """The two stored references of the differentiation workload pin each
    other: the directional derivatives of the oracle's FP64 adjoint of the
    500 coupled steps (c5_adjoint.json: dL/dx . v for each seeded direction,
    summed over n(0), g, R(0), P(0)) equal the central differences of the
    oracle's forward along the same directions (c5_directional.json,
    eps = 3e-5) to 1e-6 relative (measured 3e-7 and 6e-7)."""
    import json
    import os
    here = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
    with open(os.path.join(here, "c5_adjoint.json")) as f:
        adj = json.load(f)
    with open(os.path.join(here, "c5_directional.json")) as f:
        fd = json.load(f)
    assert adj["workload"] == fd["workload"]
    by_seed = {d["seed"]: d["d_v_L"] for d in fd["directions"]}
    assert set(by_seed) == {d["seed"] for d in adj["dots"]}
    for d in adj["dots"]:
        dot = d["dn0_dot_vn"] + d["dg_dot_vg"] + d["dR0_dot_vR"] + d["dP0_dot_vP"]
        assert abs(dot - by_seed[d["seed"]]) <= 1e-6 * abs(by_seed[d["seed"]]), (d["seed"], dot, by_seed[d["seed"]])
