"""Pins of the oracle's full time step (collide + stream) against closed forms
and invariants that the paper fixes.

- Shear wave at gamma = 0: the transverse momentum obeys
  j(z, t+1) = (2/3) j(z) + (1/6)(j(z-1) + j(z+1)) exactly (from
  eq. original_equil_distrib with the D3Q19 weights streamed by eq. LBE), so
  j_x(z,t) = A lambda^t sin(kz) with lambda = 1 - (2/3) sin^2(k/2); its
  long-wave limit is exp(-nu k^2) with nu = 1/6 (eq. shearviscosity).
- General gamma_s: the decay rate tends to nu k^2 with
  nu = (c_s^2/2)(1+gamma_s)/(1-gamma_s) (eq. shearviscosity).
- Kolmogorov forcing f_x = g sin(kz) at gamma = 0: the physical momentum of
  eq. special_choice_momentum_density reaches g (1+lambda)/(2(1-lambda)).
- Mass is conserved and momentum grows by exactly N g per step.
- Stationary statistics: every mode has variance mu w_k rho0 (the Gaussian
  eq. Pdistneq has variance mu n_i^eq per population; for the conserved modes
  this is the ideal-gas value, <delta rho^2> = mu rho, <j^2> = kT rho).
- Counter-based noise: 2k steps equal k + k steps bit for bit.
"""
import math

import numpy as np
import pytest


def shear_init(orc, p, amp, axis_flow=0, axis_var=2):
    L = [p.nx, p.ny, p.nz][axis_var]
    coords = np.arange(L)
    prof = amp * np.sin(2 * np.pi * coords / L)
    u = np.zeros((3, p.nz, p.ny, p.nx))
    shape = [1, 1, 1]
    shape[2 - axis_var] = L
    u[axis_flow] = prof.reshape(shape)
    return orc.init_equilibrium(p, u=u), prof


def momentum(orc, n):
    c, a, e, w = orc.tables()
    return np.einsum("ia,izyx->azyx", c.astype(float), n)


@pytest.mark.parametrize("flow,var", [(0, 2), (1, 0), (2, 1)])
def test_shear_wave_gamma0_exact(orc, flow, var):
    dims = [2, 2, 2]
    dims[var] = 32
    p = orc.Params(nx=dims[0], ny=dims[1], nz=dims[2])
    n, prof = shear_init(orc, p, 0.01, flow, var)
    lam = 1 - (2 / 3) * math.sin(math.pi / 32) ** 2
    orc.run(p, n, 200)
    j = momentum(orc, n)[flow]
    shape = [1, 1, 1]
    shape[2 - var] = 32
    np.testing.assert_allclose(j, (lam ** 200 * prof).reshape(shape) * np.ones_like(j), atol=2e-16)
    rho, _ = orc.fields(p, n)
    np.testing.assert_allclose(rho, 1.0, atol=1e-12)
    # long-wave limit of lambda is exp(-nu k^2), nu = 1/6
    assert lam ** 200 == pytest.approx(math.exp(-(1 / 6) * (2 * math.pi / 32) ** 2 * 200), rel=1e-5)


@pytest.mark.parametrize("gs", [0.5, -0.5])
def test_shear_viscosity_general_gamma(orc, gs):
    """Decay rate of a long shear wave -> nu k^2, nu = (1/6)(1+g)/(1-g)."""
    L = 128
    p = orc.Params(nx=2, ny=2, nz=L, gamma_shear=gs, gamma_bulk=gs)
    n, prof = shear_init(orc, p, 1e-4)
    orc.run(p, n, 50)  # let the non-hydrodynamic transient die out
    j0 = momentum(orc, n)[0, :, 0, 0]
    orc.run(p, n, 400, step0=50)
    j1 = momentum(orc, n)[0, :, 0, 0]
    s = np.sin(2 * np.pi * np.arange(L) / L)
    rate = -math.log((j1 @ s) / (j0 @ s)) / 400
    nu = (1 / 6) * (1 + gs) / (1 - gs)
    k = 2 * math.pi / L
    assert rate == pytest.approx(nu * k * k, rel=5e-3)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_uniform_flow_advects_a_transverse_wave(orc, axis):
    """Direction of streaming: a transverse velocity wave riding on a uniform
    flow U along its wave vector is carried downstream (the advective term of
    the Navier-Stokes limit, eq. LBE with the second-order equilibrium of
    eq. original_equil_distrib): the phase of its Fourier mode moves by
    k U t.  A standing wave alone cannot tell pull from push streaming; this
    fixes the sign along each axis.  U = 0.05 leaves O(U^2) corrections of a
    few per cent; bound 10 %."""
    L, U, A, T = 32, 0.05, 1e-3, 40
    dims = [2, 2, 2]
    dims[axis] = L
    nx, ny, nz = dims
    p = orc.Params(nx=nx, ny=ny, nz=nz)
    trans = (axis + 1) % 3
    k = 2 * np.pi / L
    coord = np.arange(L)
    shape = [1, 1, 1]
    shape[2 - axis] = L
    u = np.zeros((3, nz, ny, nx))
    u[axis] = U
    u[trans] = np.broadcast_to((A * np.sin(k * coord)).reshape(shape), (nz, ny, nx))
    n = orc.init_equilibrium(p, u=u)

    def phase():
        rho, uu = orc.fields(p, n)
        j = (rho * uu[trans]).mean(axis=tuple(a for a in range(3) if a != 2 - axis))
        return np.angle(np.sum(j * np.exp(-1j * k * coord)))

    ph0 = phase()
    orc.run(p, n, T)
    shift = -(np.angle(np.exp(1j * (phase() - ph0))))
    assert shift == pytest.approx(k * U * T, rel=0.1)


def test_kolmogorov_steady_amplitude(orc):
    L = 32
    g = 1e-6
    p = orc.Params(nx=2, ny=2, nz=L)
    n = orc.init_equilibrium(p)
    z = np.arange(L)
    f = np.zeros((3, L, 2, 2))
    f[0] = (g * np.sin(2 * np.pi * z / L))[:, None, None]
    for t in range(6000):  # transient lambda^t has decayed below 1e-16
        orc.step(p, n, t, extra_force=f)
    jraw = momentum(orc, n)[0]
    jphys = jraw + 0.5 * f[0]  # eq. special_choice_momentum_density
    lam = 1 - (2 / 3) * math.sin(math.pi / L) ** 2
    amp = g * (1 + lam) / (2 * (1 - lam))
    np.testing.assert_allclose(jphys, amp * np.sin(2 * np.pi * z / L)[:, None, None] * np.ones((L, 2, 2)),
                               rtol=0, atol=1e-9 * amp + 1e-20)


def test_conservation_with_body_force_and_noise(orc):
    p = orc.Params(nx=6, ny=5, nz=4, kT=1e-4, g=(1e-5, -2e-5, 3e-6), seed=7, gamma_shear=0.2, gamma_bulk=-0.1)
    rng = np.random.default_rng(5)
    u = rng.normal(scale=0.01, size=(3, 4, 5, 6))
    n = orc.init_equilibrium(p, u=u)
    t0 = orc.totals(p, n)
    N = p.N
    orc.run(p, n, 25)
    t1 = orc.totals(p, n)
    assert t1[0] == pytest.approx(t0[0], rel=1e-14)
    np.testing.assert_allclose(t1[1:] - t0[1:], 25 * N * np.array(p.g), atol=1e-13)


def test_step_split_is_bitwise(orc):
    p = orc.Params(nx=5, ny=4, nz=3, kT=1e-4, seed=123)
    n = orc.init_equilibrium(p)
    n2 = n.copy()
    orc.run(p, n, 20)
    orc.run(p, n2, 10, step0=0)
    orc.run(p, n2, 10, step0=10)
    assert np.array_equal(n, n2)


@pytest.mark.slow
def test_stationary_mode_variances(orc):
    """<delta m_k^2> = mu w_k rho0 for all 19 modes (mu = 3 kT)."""
    c, a, e, w = orc.tables()
    L = 12
    kT = 1e-4
    p = orc.Params(nx=L, ny=L, nz=L, kT=kT, seed=11)
    n = orc.init_equilibrium(p)
    orc.run(p, n, 150)
    acc = np.zeros(19)
    cnt = 0
    for t in range(150, 450, 3):
        orc.run(p, n, 3, step0=t)
        m = orc.mode_field(p, n)
        dm = m - m.mean(axis=(1, 2, 3), keepdims=True)
        acc += (dm ** 2).mean(axis=(1, 2, 3))
        cnt += 1
    ratio = acc / cnt / (3 * kT * w * p.rho0)
    # conserved modes: the box-average is removed, correction (N-1)/N
    np.testing.assert_allclose(ratio, 1.0, atol=0.03)


@pytest.mark.slow
def test_transverse_current_autocorrelation(orc):
    """At gamma = 0 the transverse current of the lowest Fourier mode decays by
    lambda(k) per step on average (linear dynamics, eq. LBE), and its equal-time
    variance is N kT rho0 (equipartition of eq. Pdistneq)."""
    L = 12
    kT = 1e-4
    p = orc.Params(nx=L, ny=L, nz=L, kT=kT, seed=3)
    n = orc.init_equilibrium(p)
    orc.run(p, n, 100)
    k = 2 * np.pi / L
    z = np.arange(L)
    phase = np.exp(-1j * k * z)[:, None, None]
    lam = 1 - (2 / 3) * math.sin(k / 2) ** 2
    c0 = c1 = 0.0
    prev = None
    for t in range(100, 1300):
        orc.step(p, n, t)
        jx = momentum(orc, n)[0]
        jk = (jx * phase).sum()
        if prev is not None:
            c0 += abs(prev) ** 2
            c1 += (jk * np.conj(prev)).real
        prev = jk
    assert c1 / c0 == pytest.approx(lam, abs=0.02)
    N = L ** 3
    assert c0 / 1199 / (N * kT) == pytest.approx(1.0, rel=0.2)


# ---------------------------------------------------------------------------
# Linear stability operator (eq. lco_eigen, eq. lco_update): the 19 x 19 map
# of a Fourier mode exp(i k.r) of population deviations through one step,
# A(k) = S(k) E^-1 diag(gamma) E with S = diag(exp(-i k.c_i)) (streaming) and
# E the Table 1 basis (equilibrium moments of order >= 2 vanish at linear
# order around rest).  Built from the golden Table 1 fixture and numpy's
# eigensolver only.
# ---------------------------------------------------------------------------

def _table1_basis(c):
    from test_oracle_lattice import load_table1
    rows = load_table1()
    E = np.zeros((19, 19))
    w = np.zeros(19)
    for k, poly, wk in rows:
        for i in range(19):
            cx, cy, cz = (float(v) for v in c[i])
            E[k, i] = eval(poly, {}, {"cx": cx, "cy": cy, "cz": cz, "c2": cx * cx + cy * cy + cz * cz})
        w[k] = float(wk)
    return E, w


def _mode_gammas(gs, gv, g3a, g3b, g4a, g4b):
    return np.array([1, 1, 1, 1, gv] + [gs] * 5 + [g3a] * 3 + [g3b] * 3 + [g4a] + [g4b] * 2, dtype=float)


def linear_operator(c, gam, kvec):
    E, w = _table1_basis(c)
    a = np.array([{0: 1 / 3, 1: 1 / 18, 2: 1 / 36}[int((ci ** 2).sum())] for ci in c])
    Einv = (a[:, None] * E.T) / w[None, :]         # back-transformation n_i = a_i sum_k e_ki m_k / w_k
    Cl = Einv @ np.diag(gam) @ E
    S = np.diag(np.exp(-1j * (c.astype(float) @ kvec)))
    return S @ Cl


def two_rate(gamma_e, magic=3.0 / 16.0):
    """Odd kinetic eigenvalue from the even one for a given
    Lambda = (1/(1 - gamma_e) - 1/2)(1/(1 - gamma_o) - 1/2)."""
    te = 1.0 / (1.0 - gamma_e)
    to = 0.5 + magic / (te - 0.5)
    return 1.0 - 1.0 / to


RELAX_SETS = {
    "gamma0": (0.0, 0.0, 0.0, 0.0, 0.0, 0.0),
    "tau0.8": (-0.25, -0.25, 0.0, 0.0, 0.0, 0.0),
    "general": (0.3, -0.2, 0.1, -0.4, 0.5, 0.2),
    "two_rate_magic": (0.3, 0.3, two_rate(0.3), two_rate(0.3), 0.3, 0.3),
}


def test_linear_operator_reproduces_closed_form_shear_rate(orc):
    """At gamma = 0 the shear eigenvalue is 1 - (2/3) sin^2(k/2), and for small
    k at general gamma_s it approaches exp(-nu k^2), nu = (1/6)(1+g)/(1-g)
    (eq. shearviscosity with rho c_s^2 h / 2 and rho = 1)."""
    c, a, e, w = orc.tables()
    for L in (16, 32):
        k = 2 * np.pi / L
        lam = np.linalg.eigvals(linear_operator(c, _mode_gammas(*RELAX_SETS["gamma0"]), np.array([0, 0, k])))
        assert np.min(np.abs(lam - (1 - (2 / 3) * np.sin(k / 2) ** 2))) < 1e-14
    gs = 0.3
    k = 2 * np.pi / 512
    lam = np.linalg.eigvals(linear_operator(c, _mode_gammas(gs, -0.2, 0.1, -0.4, 0.5, 0.2), np.array([0, 0, k])))
    nu = (1 / 6) * (1 + gs) / (1 - gs)
    # the hydrodynamic limit holds to O(k^4) = 2.3e-8 at k = 2 pi / 512
    assert np.min(np.abs(lam - np.exp(-nu * k * k))) < 1e-8


@pytest.mark.parametrize("name", list(RELAX_SETS))
def test_shear_eigenmode_evolves_by_its_eigenvalue(orc, name):
    """T5: a shear eigenmode of A(k), k = 2 pi / L along z, seeded at amplitude
    1e-8 into the oracle (kT = 0), is multiplied by its eigenvalue every
    step: after T steps the state equals lambda^T times the mode to 1e-7
    relative (the collision's quadratic terms are O(amplitude))."""
    gs, gv, g3a, g3b, g4a, g4b = RELAX_SETS[name]
    p = orc.Params(nx=4, ny=4, nz=16, gamma_shear=gs, gamma_bulk=gv, gamma_3a=g3a, gamma_3b=g3b, gamma_4a=g4a,
                   gamma_4b=g4b)
    c, a, e, w = orc.tables()
    k = 2 * np.pi / p.nz
    lam, V = np.linalg.eig(linear_operator(c, _mode_gammas(gs, gv, g3a, g3b, g4a, g4b), np.array([0, 0, k])))
    jx = c[:, 0].astype(float) @ V                  # x-momentum of each eigenvector
    m = int(np.argmax(np.abs(jx) * (np.abs(lam) > 0.5)))
    v = V[:, m] / jx[m]                             # normalised to unit j_x
    assert abs(lam[m].imag) < 1e-12
    eps, T = 1e-8, 12
    z = np.arange(p.nz)
    mode = np.real(v[:, None] * np.exp(1j * k * z)[None, :])      # [19, nz]
    n = (a[:, None, None, None] + eps * mode[:, :, None, None] * np.ones((1, 1, p.ny, p.nx)))
    n = np.ascontiguousarray(n)
    orc.run(p, n, T)
    expect = a[:, None, None, None] + eps * np.real(lam[m] ** T * v[:, None] * np.exp(1j * k * z)[None, :])[:, :, None,
                                                                                                              None]
    err = np.abs(n - expect).max() / eps
    print(name, "eigenvalue", lam[m].real, "rel err", err)
    assert err < 1e-7


@pytest.mark.parametrize("name", list(RELAX_SETS))
def test_linear_dynamics_equal_operator_power(orc, name):
    """The whole linearised step: a random complex population perturbation on
    an oblique wave vector k = 2 pi (1/nx, 2/ny, 1/nz), seeded at amplitude
    1e-8, after T oracle steps equals A(k)^T applied to it (every eigenvalue
    group and direction enters: bulk, shear, both odd and both even kinetic
    groups)."""
    gs, gv, g3a, g3b, g4a, g4b = RELAX_SETS[name]
    p = orc.Params(nx=6, ny=8, nz=10, gamma_shear=gs, gamma_bulk=gv, gamma_3a=g3a, gamma_3b=g3b, gamma_4a=g4a,
                   gamma_4b=g4b)
    c, a, e, w = orc.tables()
    rng = np.random.default_rng(3)
    kvec = 2 * np.pi * np.array([1 / p.nx, 2 / p.ny, 1 / p.nz])
    A = linear_operator(c, _mode_gammas(gs, gv, g3a, g3b, g4a, g4b), kvec)
    v = rng.normal(size=19) + 1j * rng.normal(size=19)
    z, y, x = np.meshgrid(np.arange(p.nz), np.arange(p.ny), np.arange(p.nx), indexing="ij")
    phase = np.exp(1j * (kvec[0] * x + kvec[1] * y + kvec[2] * z))
    eps, T = 1e-8, 9
    n = np.ascontiguousarray(a[:, None, None, None] + eps * np.real(v[:, None, None, None] * phase[None]))
    orc.run(p, n, T)
    vT = np.linalg.matrix_power(A, T) @ v
    expect = a[:, None, None, None] + eps * np.real(vT[:, None, None, None] * phase[None])
    err = np.abs(n - expect).max() / (eps * np.abs(v).max())
    print(name, "rel err", err)
    assert err < 1e-7
