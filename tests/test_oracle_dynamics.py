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
