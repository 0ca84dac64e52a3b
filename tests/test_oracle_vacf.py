"""Pins of the oracle's transverse Fourier amplitudes (orc_transverse_modes),
the observable of the batch form's ensemble VACF:
- against numpy's FFT of the momentum density j = sum_i c_i n_i of a random
  state on a ragged box (the k = 2 pi / L_a coefficient along axis a,
  index 1 of that axis and 0 of the other two);
- a single shear wave j_x(z) = A cos(kz) + B sin(kz): amplitude
  (N / 2)(A - iB) in the (k along z, j_x) mode and zero in every other;
- a uniform momentum has no k != 0 component.
"""
import numpy as np


def test_transverse_modes_match_fft(orc):
    rng = np.random.default_rng(4)
    p = orc.Params(nx=7, ny=5, nz=6)
    n = rng.normal(scale=0.1, size=(19, p.nz, p.ny, p.nx)) + 0.05
    c, _, _, _ = orc.tables()
    j = np.einsum("ia,izyx->azyx", c.astype(float), n)
    F = [np.fft.fftn(j[a]) for a in range(3)]  # axes (z, y, x)
    want = np.array([F[0][1, 0, 0], F[1][1, 0, 0],   # k along z: j_x, j_y
                     F[0][0, 1, 0], F[2][0, 1, 0],   # k along y: j_x, j_z
                     F[1][0, 0, 1], F[2][0, 0, 1]])  # k along x: j_y, j_z
    got = orc.transverse_modes(p, n)
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-12 * np.abs(want).max())


def test_transverse_modes_shear_wave_and_uniform_flow(orc):
    p = orc.Params(nx=4, ny=3, nz=8)
    A, B, k = 0.01, -0.004, 2 * np.pi / 8
    z = np.arange(8)
    u = np.zeros((3, 8, 3, 4))
    u[0] = (A * np.cos(k * z) + B * np.sin(k * z))[:, None, None]
    n = orc.init_equilibrium(p, u=u)   # rho = 1: j = u
    got = orc.transverse_modes(p, n)
    want = np.zeros(6, complex)
    want[0] = (p.N / 2) * (A - 1j * B)
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-14)
    u = np.zeros((3, 8, 3, 4))
    u[:] = np.array([0.01, -0.02, 0.03])[:, None, None, None]
    assert np.abs(orc.transverse_modes(p, orc.init_equilibrium(p, u=u))).max() < 1e-14
