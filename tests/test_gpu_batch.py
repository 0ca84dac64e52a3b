"""GPU tests of the batched replica form (lb_create_batch) through the C ABI:
per-box parity with the FP64 oracle (box b draws its noise with box id b),
graph replay == eager launches bit for bit, the launch-configuration search
does not change results, and the on-device ensemble VACF of the lowest
transverse modes follows lambda(k)^tau (eq. LBE, gamma = 0) with equal-time
value N kT rho0 (equipartition of eq. Pdistneq)."""
import math

import numpy as np
import pytest

from conftest import gpu_available

pytestmark = pytest.mark.gpu

DIMS = [(8, 8, 8), (12, 10, 6), (5, 7, 9), (16, 4, 3)]


@pytest.fixture(scope="module")
def lat():
    if not gpu_available():
        pytest.skip("no GPU")
    from paper_0803_2826_amd import lattice
    return lattice


def oracle_boxes(orc, kT, seed, g=(0.0, 0.0, 0.0), gs=0.0):
    return [orc.Params(nx=d[0], ny=d[1], nz=d[2], kT=kT, seed=seed, box=b, g=g, gamma_shear=gs, gamma_bulk=gs)
            for b, d in enumerate(DIMS)]


def test_batch_parity_per_box(orc, lat):
    import torch
    kT, seed, g = 1e-4, 17, (1e-5, 0.0, -1e-5)
    pos = oracle_boxes(orc, kT, seed, g, gs=0.2)
    rng = np.random.default_rng(0)
    ns = [orc.init_equilibrium(p, u=rng.normal(scale=0.01, size=(3, p.nz, p.ny, p.nx))) for p in pos]
    pd = lat.FluidParams(nx=2, ny=2, nz=2, kT=kT, seed=seed, body_force=g, gamma_shear=0.2, gamma_bulk=0.2, block=128)
    B = lat.BatchLattice(pd, DIMS)
    B.set_populations(torch.from_numpy(np.concatenate([n.reshape(-1) for n in ns])))
    for p, n in zip(pos, ns):
        orc.run(p, n, 15)
    B.step(15)
    got = B.split(B.get_populations())
    for b, (gb, n) in enumerate(zip(got, ns)):
        err = np.abs(gb.cpu().numpy() - n).max()
        assert err <= 1e-6, (b, err)
    tot = B.totals()
    ref = sum(orc.totals(p, n) for p, n in zip(pos, ns))
    np.testing.assert_allclose(tot, ref, rtol=0, atol=1e-6)
    B.close()


def test_graph_replay_equals_eager(lat):
    import torch
    dims = DIMS * 3
    base = dict(nx=2, ny=2, nz=2, kT=1e-4, seed=5, vacf_lags=8, block=256)
    A = lat.BatchLattice(lat.FluidParams(**base, graph_steps=0), dims)
    G = lat.BatchLattice(lat.FluidParams(**base, graph_steps=4), dims)
    for X in (A, G):
        X.init_equilibrium()
        X.step(7)   # one graph replay + 3 eager steps (parity flips)
        X.step(9)   # graph for the other buffer parity
    assert A.step_count == G.step_count == 16
    assert torch.equal(A.get_populations(dtype=torch.float32), G.get_populations(dtype=torch.float32))
    va, na = A.vacf()
    vg, ng = G.vacf()
    assert na == ng == 16
    np.testing.assert_allclose(va, vg, rtol=1e-5, atol=1e-12)
    A.close()
    G.close()


def test_autotune_does_not_change_results(lat):
    import torch
    base = dict(nx=2, ny=2, nz=2, kT=1e-4, seed=9)
    F = lat.BatchLattice(lat.FluidParams(**base, block=256), DIMS)
    T = lat.BatchLattice(lat.FluidParams(**base, block=0), DIMS)
    for X in (F, T):
        X.init_equilibrium()
        X.step(6)
    blk, grid, chunk, _ = T.launch_config()
    assert blk in (128, 256, 512, 1024) and grid >= 1 and chunk >= 1
    assert torch.equal(F.get_populations(dtype=torch.float32), T.get_populations(dtype=torch.float32))
    F.close()
    T.close()


def test_single_box_autotune(orc, lat):
    """The searched launch configurations (without and with bead force) give
    the same state as a fixed one, bit for bit."""
    import torch
    from paper_0803_2826_amd.inputs import random_walk_chains
    p = dict(nx=40, ny=32, nz=24, kT=1e-4, seed=2)
    pos, mom, bonds = random_walk_chains(4, 8, (40, 32, 24), seed=1)
    nb = pos.shape[0]
    A = lat.Lattice(lat.FluidParams(**p, block=256))
    T = lat.Lattice(lat.FluidParams(**p, block=-1))
    for X in (A, T):
        X.init_equilibrium()
        X.step(3)
        beads = lat.DeviceBeads(pos, mom, np.ones(nb), np.full(nb, 5.0), bonds, 1e-3, 1.0)
        for _ in range(3):
            X.coupled_step(beads)
        X.step(2)
    for force in (False, True):
        blk, grid, tiles, remap = T.launch_config(force)
        assert blk in (64, 128, 256, 512, 1024) and tiles == 1 and remap in (0, 1)
        assert grid * blk >= 40 * 32 * 24
    assert torch.equal(A.get_populations(dtype=torch.float32), T.get_populations(dtype=torch.float32))
    assert A.totals(exact=True) == T.totals(exact=True)
    A.close()
    T.close()


def test_batch_vacf_amplitudes_match_oracle(orc, lat):
    """Two sampled steps of the on-device VACF (vacf_lags = 2) against the
    oracle's amplitudes of the populations at the start of each step (the
    momentum the step's collision sees; the kernel forms it from the stored
    post-collision values less the body force): per box,
    C_b(0) 6 N_b kT rho0 = (|j_hat(0)|^2 + |j_hat(1)|^2) / 2 and
    C_b(1) 6 N_b kT rho0 = Re[j_hat(1) conj(j_hat(0))], summed over the six
    modes (ragged boxes, so tiles span box ends)."""
    import torch
    kT, seed, g = 1e-4, 31, (1e-5, -2e-5, 0.0)
    pos = oracle_boxes(orc, kT, seed, g)
    rng = np.random.default_rng(2)
    ns = [orc.init_equilibrium(p, u=rng.normal(scale=0.01, size=(3, p.nz, p.ny, p.nx))) for p in pos]
    pd = lat.FluidParams(nx=2, ny=2, nz=2, kT=kT, seed=seed, body_force=g, vacf_lags=2)
    B = lat.BatchLattice(pd, DIMS)
    B.set_populations(torch.from_numpy(np.concatenate([n.reshape(-1) for n in ns])))
    start = [x.cpu().numpy() for x in B.split(B.get_populations())]
    B.step(2)
    C, nsamp = B.vacf()
    B.close()
    assert nsamp == 2
    for b, (p, n) in enumerate(zip(pos, start)):
        a0 = orc.transverse_modes(p, n)
        n1 = n.copy()
        orc.run(p, n1, 1)
        a1 = orc.transverse_modes(p, n1)
        norm = 6 * p.N * kT * p.rho0
        want = [float((np.abs(a0) ** 2 + np.abs(a1) ** 2).sum() / (2 * norm)),
                float((a1 * np.conj(a0)).real.sum() / norm)]
        print(b, C[b], want)
        assert C[b] == pytest.approx(want, rel=1e-4), (b, C[b], want)


def test_batch_vacf_decay(lat):
    """64 replicas of 16^3 at gamma = 0: C(tau) ~ lambda(k)^tau, C(0) ~ 1."""
    kT = 1e-4
    L = 16
    dims = [(L, L, L)] * 64
    B = lat.BatchLattice(lat.FluidParams(nx=2, ny=2, nz=2, kT=kT, seed=123, vacf_lags=12, graph_steps=10), dims)
    B.init_equilibrium()
    B.step(300)   # thermalise (samples of the transient are included but few)
    B.step(1200)
    C, nsamp = B.vacf()
    assert nsamp == 1500
    lam = 1 - (2 / 3) * math.sin(math.pi / L) ** 2
    Cm = C.mean(axis=0)
    print("C(tau):", np.round(Cm, 4), "lambda:", lam)
    assert Cm[0] == pytest.approx(1.0, rel=0.1)
    np.testing.assert_allclose(Cm[1:] / Cm[0], lam ** np.arange(1, 12), atol=0.03)
    B.close()


def test_batch_rejects_coupling_and_bad_args(lat):
    from paper_0803_2826_amd._lib import LB_EINVAL, LB_EUNSUPPORTED, LBError
    with pytest.raises(LBError) as ei:
        lat.BatchLattice(lat.FluidParams(nx=2, ny=2, nz=2, graph_steps=3), DIMS)
    assert ei.value.code == LB_EINVAL
    with pytest.raises(LBError) as ei:
        lat.BatchLattice(lat.FluidParams(nx=2, ny=2, nz=2), [(1, 4, 4)])
    assert ei.value.code == LB_EINVAL
    B = lat.BatchLattice(lat.FluidParams(nx=2, ny=2, nz=2, kT=1e-4), DIMS)
    B.init_equilibrium()
    beads = lat.DeviceBeads(np.zeros((1, 3)), np.zeros((1, 3)), np.ones(1), np.ones(1))
    with pytest.raises(LBError) as ei:
        B.couple(beads)
    assert ei.value.code == LB_EUNSUPPORTED
    B.close()
