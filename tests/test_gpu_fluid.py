"""GPU parity of the fused stream-collide path against the FP64 oracle.

All calls go through liblbmi's C ABI (ctypes binding).  Tolerances:
- populations: 1e-6 absolute after the run (FP32 arithmetic on shifted
  populations of size ~1e-2 rounds at ~1e-9 per step; the noise uses hardware
  log2/sqrt/sin/cos whose error is ~1e-6 relative on a unit Gaussian times an
  amplitude sqrt(w mu rho) <= 1.1e-2, i.e. <= 1e-8 per step);
- device Gaussians vs oracle Gaussians: 2e-5 absolute (same 24-bit integer
  fields, FP32 hardware transcendentals vs FP64 libm).
"""
import math

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


def make_pair(orc, lat, **kw):
    """Matching oracle and device parameter objects."""
    p_or = orc.Params(nx=kw["nx"], ny=kw["ny"], nz=kw["nz"], rho0=kw.get("rho0", 1.0),
                      gamma_shear=kw.get("gs", 0.0), gamma_bulk=kw.get("gb", 0.0),
                      gamma_3a=kw.get("g3a", 0.0), gamma_3b=kw.get("g3b", 0.0),
                      gamma_4a=kw.get("g4a", 0.0), gamma_4b=kw.get("g4b", 0.0),
                      kT=kw.get("kT", 0.0), g=kw.get("g", (0.0, 0.0, 0.0)), seed=kw.get("seed", 0),
                      noise_rho0=kw.get("noise_rho0", False))
    p_dev = lat.FluidParams(nx=kw["nx"], ny=kw["ny"], nz=kw["nz"], storage=kw.get("storage", "f32"),
                            rho0=p_or.rho0, gamma_shear=p_or.gamma_shear, gamma_bulk=p_or.gamma_bulk,
                            gamma_3a=p_or.gamma_3a, gamma_3b=p_or.gamma_3b, gamma_4a=p_or.gamma_4a,
                            gamma_4b=p_or.gamma_4b, kT=p_or.kT, body_force=p_or.g, seed=p_or.seed,
                            noise_rho0=p_or.noise_rho0, block=kw.get("block", 0),
                            track_totals=kw.get("track_totals", True))
    return p_or, p_dev


def test_device_gaussians_match_oracle(orc, lat):
    import torch
    _, pd = make_pair(orc, lat, nx=16, ny=16, nz=16, kT=1e-4, seed=0xDEADBEEF12345)
    L = lat.Lattice(pd)
    for step in (0, 7, 123456):
        g = L.noise_sample(0, 2000, step).cpu().numpy().astype(np.float64)
        ref = np.array([orc.fluid_normals(pd.seed, s, step)[:15] for s in range(2000)])
        np.testing.assert_allclose(g, ref, atol=2e-5, rtol=0)
    L.close()


def run_parity(orc, lat, steps, u0=None, rho0_field=None, **kw):
    import torch
    po, pd = make_pair(orc, lat, **kw)
    n = orc.init_equilibrium(po, rho=rho0_field, u=u0)
    L = lat.Lattice(pd)
    L.set_populations(torch.from_numpy(n))
    orc.run(po, n, steps)
    L.step(steps)
    got = L.get_populations().cpu().numpy()
    return po, pd, L, n, got


def test_config1_parity_200_steps(orc, lat):
    """32^3, rho=1, tau=1 (all gamma 0), kT=1e-5, u_x = 0.01 sin(2 pi z/32),
    200 steps, Philox seed 0: |n_gpu - n_oracle| <= 1e-6, and the total mass
    of the stored state conserved to 1e-12 relative (the collision keeps each
    site's mass, constraint after eq. LBE; FP32 storage keeps the rest
    population's rounding residual, so only FP64 rounding, ~1e-16 per site
    and step, remains)."""
    import torch
    from paper_0803_2826_amd.inputs import shear_wave
    u0 = shear_wave(32, 32, 32, 0.01)
    po, pd = make_pair(orc, lat, nx=32, ny=32, nz=32, kT=1e-5, seed=0)
    n = orc.init_equilibrium(po, u=u0)
    L = lat.Lattice(pd)
    L.set_populations(torch.from_numpy(n))
    m_start = L.totals(exact=True)[0]
    orc.run(po, n, 200)
    L.step(200)
    got = L.get_populations().cpu().numpy()
    err = np.abs(got - n).max()
    print(f"config-1 parity: max|dn| = {err:.3e}")
    assert err <= 1e-6
    t_dev = L.totals(exact=True)
    t_or = orc.totals(po, n)
    M0 = 32 ** 3
    drift = (t_dev[0] - m_start) / m_start
    print(f"mass drift over 200 steps (device, relative) = {drift:.3e}; oracle {(t_or[0] - M0) / M0:.3e}")
    assert abs(drift) <= 1e-12
    assert abs(t_dev[0] - t_or[0]) / M0 < 1e-9
    L.close()


@pytest.mark.parametrize("noise_rho0", [False, True])
def test_ragged_box_general_relaxation(orc, lat, noise_rho0):
    """N = 37*29*23 (not a multiple of the block), all six eigenvalues
    distinct, body force, noise, 30 steps."""
    from paper_0803_2826_amd.inputs import random_velocity
    u0 = random_velocity(37, 29, 23, 0.01, seed=3)
    po, pd, L, n, got = run_parity(orc, lat, 30, u0=u0, nx=37, ny=29, nz=23, gs=0.3, gb=-0.2, g3a=0.1,
                                   g3b=-0.5, g4a=0.7, g4b=-0.9, kT=1e-4, g=(1e-5, -2e-5, 3e-6), seed=99,
                                   noise_rho0=noise_rho0)
    err = np.abs(got - n).max()
    print(f"ragged parity: max|dn| = {err:.3e}")
    assert err <= 1e-6
    L.close()


def test_minimal_box(orc, lat):
    po, pd, L, n, got = run_parity(orc, lat, 10, u0=np.full((3, 2, 2, 2), 0.01), nx=2, ny=2, nz=2, kT=1e-4,
                                   seed=5, g=(1e-4, 0, 0))
    assert np.abs(got - n).max() <= 1e-6
    L.close()


def test_zero_steps_and_roundtrip(orc, lat):
    import torch
    po, pd = make_pair(orc, lat, nx=9, ny=7, nz=5)
    rng = np.random.default_rng(0)
    n = orc.init_equilibrium(po, u=rng.normal(scale=0.01, size=(3, 5, 7, 9)))
    L = lat.Lattice(pd)
    L.set_populations(torch.from_numpy(n))
    L.step(0)
    got = L.get_populations().cpu().numpy()
    # only FP32 rounding of the shifted values
    assert np.abs(got - n).max() <= 1e-9
    L.close()


@pytest.mark.parametrize("block", [64, 128, 512, 1024])
def test_block_size_and_totals_flag_do_not_change_results(orc, lat, block):
    import torch
    kw = dict(nx=40, ny=24, nz=17, kT=1e-4, seed=3, gs=0.1, gb=0.1)
    po, pd_ref = make_pair(orc, lat, **kw)
    n = orc.init_equilibrium(po)
    ref = lat.Lattice(pd_ref)
    ref.set_populations(torch.from_numpy(n))
    ref.step(12)
    a = ref.get_populations(dtype=torch.float32)
    _, pd = make_pair(orc, lat, block=block, track_totals=False, **kw)
    L = lat.Lattice(pd)
    L.set_populations(torch.from_numpy(n))
    L.step(12)
    b = L.get_populations(dtype=torch.float32)
    assert torch.equal(a, b)
    ref.close()
    L.close()


def test_step_split_bitwise(orc, lat):
    import torch
    po, pd = make_pair(orc, lat, nx=20, ny=20, nz=20, kT=1e-4, seed=11)
    n = orc.init_equilibrium(po)
    A = lat.Lattice(pd)
    B = lat.Lattice(pd)
    A.set_populations(torch.from_numpy(n))
    B.set_populations(torch.from_numpy(n))
    A.step(20)
    B.step(10)
    B.step(10)
    assert torch.equal(A.get_populations(dtype=torch.float32), B.get_populations(dtype=torch.float32))
    assert A.step_count == 20
    A.close()
    B.close()


def test_totals_fused_exact_and_oracle(orc, lat):
    """Fused per-step totals vs the exact FP64 pass vs the oracle.
    Tolerances from the arithmetic: the fused mass is an FP64 sum of the
    stored values (agrees with the exact pass to FP64 rounding); the fused
    momentum is summed in FP32 per site (error ~1e-8 per site, random:
    1e-8 sqrt(N)); stored populations round at <= 3e-9 per value per step,
    so momentum totals random-walk by ~2e-8 sqrt(N T) against the oracle."""
    g = (2e-5, -1e-5, 5e-6)
    T = 40
    po, pd, L, n, got = run_parity(orc, lat, T, nx=24, ny=20, nz=16, kT=1e-4, seed=1, g=g)
    fused = np.array(L.totals())
    exact = np.array(L.totals(exact=True))
    ref = orc.totals(po, n)
    N = 24 * 20 * 16
    assert abs(fused[0] - exact[0]) <= 1e-12 * N
    np.testing.assert_allclose(fused[1:], exact[1:], rtol=0, atol=1e-8 * np.sqrt(N))
    tol = 2e-8 * np.sqrt(N * T)
    np.testing.assert_allclose(exact[1:], ref[1:], rtol=0, atol=tol)
    np.testing.assert_allclose(exact[1:], T * N * np.array(g), rtol=0, atol=tol)
    # mass: the stored state conserves it to FP64 rounding; the start differs
    # from N by the FP32 rounding of the 18 moving populations on the way in
    # (|error| <= 2^-25 * 0.05 each, random)
    assert abs(exact[0] - N) <= 6 * 1.5e-9 * np.sqrt(18 * N) / np.sqrt(3)
    L.close()


def test_moments_match_oracle_fields(orc, lat):
    from paper_0803_2826_amd.inputs import random_velocity
    po, pd, L, n, got = run_parity(orc, lat, 5, u0=random_velocity(12, 10, 8, 0.02, 4), nx=12, ny=10, nz=8,
                                   kT=1e-4, g=(1e-4, 0, -1e-4), seed=2)
    rho, u = L.moments()
    r_or, u_or = orc.fields(po, n)
    np.testing.assert_allclose(rho.cpu().numpy(), r_or, atol=1e-6)
    np.testing.assert_allclose(u.cpu().numpy(), u_or, atol=1e-6)
    L.close()


def test_mode_stats_thermal_equilibrium(orc, lat):
    """Stationary per-mode variances mu w_k rho0 (variance of eq. Pdistneq)."""
    c, a, e, w = orc.tables()
    kT = 1e-4
    _, pd = make_pair(orc, lat, nx=32, ny=32, nz=32, kT=kT, seed=17)
    L = lat.Lattice(pd)
    L.init_equilibrium()
    L.step(300)
    acc = np.zeros(19)
    for _ in range(20):
        L.step(5)
        acc += np.array(L.mode_stats())
    ratio = acc / 20 / (3 * kT * w)
    print("mode variance ratios:", np.round(ratio, 4))
    np.testing.assert_allclose(ratio, 1.0, atol=0.02)
    L.close()


def test_shear_wave_decay_matches_closed_form(orc, lat):
    """kT = 0, gamma = 0: j_x = A lambda^t sin(kz), lambda = 1 - (2/3) sin^2(k/2)."""
    from paper_0803_2826_amd.inputs import shear_wave
    _, pd = make_pair(orc, lat, nx=8, ny=8, nz=64)
    L = lat.Lattice(pd)
    L.init_equilibrium(u=shear_wave(8, 8, 64, 0.01))
    L.step(500)
    rho, u = L.moments()
    ux = (u[0] * rho).cpu().numpy()[:, 0, 0]
    lam = 1 - (2 / 3) * math.sin(math.pi / 64) ** 2
    np.testing.assert_allclose(ux, 0.01 * lam ** 500 * np.sin(2 * np.pi * np.arange(64) / 64), atol=2e-8)
    L.close()


def test_error_paths(orc, lat):
    import torch
    from paper_0803_2826_amd._lib import LB_EINVAL, LB_ENONFINITE, LBError
    for bad in (dict(nx=1, ny=4, nz=4), dict(nx=4, ny=4, nz=4, gamma_shear=1.0),
                dict(nx=4, ny=4, nz=4, kT=-1.0), dict(nx=4, ny=4, nz=4, gamma_3a=1.5),
                dict(nx=4, ny=4, nz=4, block=100), dict(nx=4, ny=4, nz=4, rho0=0.0)):
        with pytest.raises(LBError) as ei:
            lat.Lattice(lat.FluidParams(**bad))
        assert ei.value.code == LB_EINVAL
    L = lat.Lattice(lat.FluidParams(nx=4, ny=4, nz=4, kT=1e-4))
    with pytest.raises(LBError) as ei:
        L.step(-1)
    assert ei.value.code == LB_EINVAL
    n = torch.zeros((19, 4, 4, 4), dtype=torch.float64)
    n[3, 1, 2, 3] = float("nan")
    L.set_populations(n, shifted=True)
    L.step(1)
    with pytest.raises(LBError) as ei:
        L.sync()
    assert ei.value.code == LB_ENONFINITE
    L.close()
