"""Differentiation form on the GPU (lb_tape_begin / lb_backward and the
torch.autograd.Function), checked against the oracle's FP64 adjoint (itself
pinned by central finite differences) and, at 128^3, against a central
finite difference of the FP64 oracle forward along one random direction.

Tolerance: the GPU computes forward and adjoint in FP32; each step rounds
the adjoint at ~1e-7 relative and the rounding of T steps random-walks, so
the gradient error relative to its largest entry is ~1e-7 sqrt(T) (<= 1e-5
for T <= 1e4); bound 2e-5.
"""
import numpy as np
import pytest

from conftest import gpu_available

pytestmark = pytest.mark.gpu

REL_TOL = 2e-5


@pytest.fixture(scope="module")
def lat():
    if not gpu_available():
        pytest.skip("no GPU")
    from paper_0803_2826_amd import lattice
    return lattice


def pair(orc, lat, nx, ny, nz, **kw):
    po = orc.Params(nx=nx, ny=ny, nz=nz, **kw)
    pd = lat.FluidParams(nx=nx, ny=ny, nz=nz, kT=po.kT, seed=po.seed, body_force=po.g, gamma_shear=po.gamma_shear,
                         gamma_bulk=po.gamma_bulk, gamma_3a=po.gamma_3a, gamma_3b=po.gamma_3b,
                         gamma_4a=po.gamma_4a, gamma_4b=po.gamma_4b, noise_rho0=po.noise_rho0, track_totals=False)
    return po, pd


@pytest.mark.parametrize("noise_rho0", [False, True])
def test_gpu_adjoint_matches_oracle_adjoint(orc, lat, noise_rho0):
    import torch
    rng = np.random.default_rng(0)
    po, pd = pair(orc, lat, 12, 10, 8, kT=1e-4, seed=5, g=(1e-4, -5e-5, 2e-5), gamma_shear=0.2, gamma_bulk=-0.1,
                  gamma_3a=0.3, gamma_3b=-0.2, gamma_4a=0.1, gamma_4b=0.4, noise_rho0=noise_rho0)
    n0 = orc.init_equilibrium(po, u=rng.normal(scale=0.02, size=(3, 8, 10, 12)))
    T = 20
    w = rng.normal(size=n0.shape)
    dev = lat.Lattice(pd)
    dev.set_populations(torch.from_numpy(n0))
    n0r = dev.get_populations().cpu().numpy()   # the device's rounded start
    dev.tape_begin(7)                            # segments of 7, 7, 6 steps
    dev.step(T)
    dn0, dg = dev.backward(torch.from_numpy(w))
    ref, gref = orc.backward(po, n0r, T, w)
    err = np.abs(dn0.cpu().numpy() - ref).max() / np.abs(ref).max()
    print(f"adjoint rel err {err:.2e}, dg {dg} vs {gref}")
    assert err <= REL_TOL
    np.testing.assert_allclose(dg, gref, rtol=REL_TOL * 10, atol=1e-6 * np.abs(gref).max())
    dev.close()


def test_checkpoint_interval_does_not_change_gradient(orc, lat):
    import torch
    rng = np.random.default_rng(1)
    po, pd = pair(orc, lat, 10, 9, 8, kT=1e-4, seed=2)
    n0 = orc.init_equilibrium(po, u=rng.normal(scale=0.02, size=(3, 8, 9, 10)))
    w = torch.from_numpy(rng.normal(size=n0.shape))
    outs = []
    # 2^31 - 1: too many step buffers to allocate at lb_tape_begin, so the
    # taped steps write none of them and the sweep allocates the 13 it needs
    for K in (1, 4, 13, 100, 2 ** 31 - 1):
        dev = lat.Lattice(pd)
        dev.set_populations(torch.from_numpy(n0))
        dev.tape_begin(K)
        dev.step(13)
        outs.append(dev.backward(w))
        dev.close()
    for dn, dg in outs[1:]:
        assert torch.equal(dn, outs[0][0])
        assert dg == outs[0][1]


def velocity_table(device):
    import torch
    c = [[0, 0, 0], [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1], [1, 1, 0], [-1, -1, 0],
         [1, -1, 0], [-1, 1, 0], [1, 0, 1], [-1, 0, -1], [1, 0, -1], [-1, 0, 1], [0, 1, 1], [0, -1, -1], [0, 1, -1],
         [0, -1, 1]]
    return torch.tensor(c, dtype=torch.float64, device=device)


def probe_loss_torch(nT, g, lo, hi):
    """Mean |u|^2 over a probe sub-box, u = (sum n c + g/2)/rho."""
    import torch
    c = velocity_table(nT.device)
    J = torch.einsum("ia,izyx->azyx", c, nT) + 0.5 * g.reshape(3, 1, 1, 1)
    rho = nT.sum(0)
    u = J / rho
    return (u[:, lo:hi, lo:hi, lo:hi] ** 2).sum(0).mean()


def test_autograd_probe_loss_matches_oracle(orc, lat):
    import torch
    from paper_0803_2826_amd.autograd import rollout
    import test_oracle_adjoint as toa
    rng = np.random.default_rng(3)
    L = 12
    po, pd = pair(orc, lat, L, L, L, kT=1e-4, seed=9, g=(2e-4, 0.0, -1e-4))
    n0 = orc.init_equilibrium(po, u=rng.normal(scale=0.02, size=(3, L, L, L)))
    T, lo, hi = 30, 4, 8
    n0_t = torch.tensor(n0, device="cuda", requires_grad=True)
    g_t = torch.tensor(po.g, dtype=torch.float64, device="cuda", requires_grad=True)
    nT = rollout(n0_t, g_t, pd, T, checkpoint_every=10)
    loss = probe_loss_torch(nT, g_t, lo, hi)
    loss.backward()
    # oracle: forward, loss gradient, FP64 adjoint
    nT_ref = n0.copy()
    orc.run(po, nT_ref, T)
    lamT, g_direct = toa.probe_loss_grad(orc, po, nT_ref, lo, hi)
    lam0, gbar = orc.backward(po, n0, T, lamT)
    err = np.abs(n0_t.grad.cpu().numpy() - lam0).max() / np.abs(lam0).max()
    print(f"probe-loss gradient rel err {err:.2e}")
    assert err <= REL_TOL
    np.testing.assert_allclose(g_t.grad.cpu().numpy(), gbar + g_direct, rtol=1e-4)


def test_backward_error_paths(orc, lat):
    import torch
    from paper_0803_2826_amd._lib import LB_EINVAL, LB_ESTATE, LB_EUNSUPPORTED, LBError
    dev = lat.Lattice(lat.FluidParams(nx=8, ny=8, nz=8, kT=1e-4))
    dev.init_equilibrium()
    dev.step(2)
    with pytest.raises(LBError) as ei:
        dev.backward(torch.zeros(19 * 512, dtype=torch.float64))
    assert ei.value.code == LB_ESTATE
    with pytest.raises(LBError) as ei:
        dev.tape_begin(-1)
    assert ei.value.code == LB_EINVAL
    dev.close()
    B = lat.BatchLattice(lat.FluidParams(nx=2, ny=2, nz=2, kT=1e-4, block=256), [(8, 8, 8)])
    with pytest.raises(LBError) as ei:
        B.tape_begin(4)
    assert ei.value.code == LB_EUNSUPPORTED
    B.close()


@pytest.mark.parametrize("replace", ["set_populations", "init_equilibrium", "step_count"])
def test_replacing_the_state_ends_the_tape(orc, lat, replace):
    """A call that replaces the state or the step counter in the middle of a
    tape ends it: lb_backward then returns LB_ESTATE from its host-side
    checks (it never indexes a tape that does not match the steps).  A new
    tape after such a call differentiates as usual, matching the oracle."""
    import torch
    from paper_0803_2826_amd._lib import LB_ESTATE, LBError
    rng = np.random.default_rng(6)
    po = orc.Params(nx=8, ny=6, nz=5, kT=1e-4, seed=3)
    pd = lat.FluidParams(nx=8, ny=6, nz=5, kT=1e-4, seed=3, track_totals=False)
    n0 = orc.init_equilibrium(po, u=rng.normal(scale=0.02, size=(3, 5, 6, 8)))
    w = rng.normal(size=n0.shape)
    dev = lat.Lattice(pd)
    dev.set_populations(torch.from_numpy(n0))
    dev.tape_begin(2)                       # the forward writes its step buffers into the segment slots
    dev.step(3)
    if replace == "set_populations":
        dev.set_populations(torch.from_numpy(n0))
    elif replace == "init_equilibrium":
        dev.init_equilibrium()
    else:
        dev.step_count = 7
    dev.step(2)
    with pytest.raises(LBError) as ei:
        dev.backward(torch.from_numpy(w))
    assert ei.value.code == LB_ESTATE
    # a fresh tape on the same context
    dev.step_count = 0
    dev.set_populations(torch.from_numpy(n0))
    n0r = dev.get_populations().cpu().numpy()
    dev.tape_begin(2)
    dev.step(5)
    dn0, dg = dev.backward(torch.from_numpy(w))
    lam0, gbar = orc.backward(po, n0r, 5, w)
    dev.close()
    assert np.abs(dn0.cpu().numpy() - lam0).max() / np.abs(lam0).max() <= REL_TOL


@pytest.mark.slow
def test_full_size_directional_derivative(orc, lat):
    """128^3 (the differentiation workload's box), 10 steps: <dL/dn0, v> from the
    GPU adjoint against a central difference of the FP64 oracle forward
    (eps = 1e-4 along a unit-scale random v; truncation O(eps^2))."""
    import torch
    L, T = 128, 10
    rng = np.random.default_rng(4)
    po, pd = pair(orc, lat, L, L, L, kT=1e-4, seed=1, g=(1e-5, 0.0, 0.0))
    n0 = orc.init_equilibrium(po, u=rng.normal(scale=0.01, size=(3, L, L, L)))
    w = rng.normal(size=n0.shape)
    dev = lat.Lattice(pd)
    dev.set_populations(torch.from_numpy(n0))
    n0 = dev.get_populations().cpu().numpy()
    dev.tape_begin(5)
    dev.step(T)
    dn0, _ = dev.backward(torch.from_numpy(w))
    dev.close()
    v = rng.normal(size=n0.shape) * 1e-3
    eps = 1e-4

    def fwd(x):
        y = x.copy()
        orc.run(po, y, T)
        return (w * y).sum()
    fd = (fwd(n0 + eps * v) - fwd(n0 - eps * v)) / (2 * eps)
    got = (dn0.cpu().numpy() * v).sum()
    print(f"directional derivative: gpu {got:.10e} fd {fd:.10e}")
    assert got == pytest.approx(fd, rel=1e-4)


def test_repeated_backward_and_continued_tape(orc, lat):
    """The taped steps leave the last segment's step buffers in place for the
    reverse sweep; a second backward over the same tape (after a sweep that
    recomputed over them, or one that did not) and a backward after more
    taped steps must give what a fresh tape gives, and no sweep may change
    the forward state."""
    import torch
    rng = np.random.default_rng(5)
    po, pd = pair(orc, lat, 9, 8, 10, kT=1e-4, seed=4)
    n0 = orc.init_equilibrium(po, u=rng.normal(scale=0.02, size=(3, 10, 8, 9)))
    w = torch.from_numpy(rng.normal(size=n0.shape))

    def fresh(K, T):
        dev = lat.Lattice(pd)
        dev.set_populations(torch.from_numpy(n0))
        dev.tape_begin(K)
        dev.step(T)
        return dev

    for K in (4, 20):
        ref9, ref13 = fresh(K, 9), fresh(K, 13)
        g9, g13 = ref9.backward(w), ref13.backward(w)
        n13 = ref13.get_populations()
        ref9.close()
        ref13.close()
        dev = fresh(K, 9)
        n9 = dev.get_populations()
        plain = lat.Lattice(pd)  # the same steps with no tape: ping-pong buffers only
        plain.set_populations(torch.from_numpy(n0))
        plain.step(9)
        assert torch.equal(plain.get_populations(), n9), K
        plain.close()
        for _ in range(2):
            dn, dg = dev.backward(w)
            assert torch.equal(dn, g9[0]) and dg == g9[1], K
            assert torch.equal(dev.get_populations(), n9), K
        dev.step(4)
        dn, dg = dev.backward(w)
        assert torch.equal(dn, g13[0]) and dg == g13[1], K
        assert torch.equal(dev.get_populations(), n13), K
        dev.close()
