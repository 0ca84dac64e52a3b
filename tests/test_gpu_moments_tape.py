"""The moments tape (lb_tape_begin(ctx, 0)): every taped step writes the
moments (rho - rho0, j) of the state it starts from, and the reverse sweep
reads them instead of recomputing states from checkpoints.

- Fluid only: the same gradients, bit for bit, as checkpointed tapes (a
  checkpoint every 4 steps, recomputed; and one segment the forward kept):
  the forward writes the moments with the summation the adjoint uses on a
  state, so the sweep sees the same values (FP32 and BF16 storage, walls,
  70 steps across a chunk of the tape).
- Coupled steps (fused and separate launches, harmonic and Kremer-Grest
  chains, plain steps interleaved, phi_3): against the oracle's FP64
  adjoint at the bar of test_gpu_adjoint_coupled (2e-5 of each gradient's
  largest entry), and against a checkpointed tape of the same run to 1e-5
  (the particle adjoint takes u at its nodes from the FP32 moments instead
  of an FP64 sum of the populations, and adds into lambda with FP32
  atomics).
- Book-keeping: a sweep over no steps, two sweeps over one tape, a tape
  ended by lb_set_populations, totals of taped steps (formed from the
  state, the steps take no fused totals).
"""
import numpy as np
import pytest

from conftest import gpu_available
from test_gpu_adjoint import pair
from test_gpu_adjoint_coupled import REL_TOL, oracle_mixed_backward, rel_err, system

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lat():
    if not gpu_available():
        pytest.skip("no GPU")
    from paper_0803_2826_amd import lattice
    return lattice


def fluid_grads(lat, pd, n0, w, K, T):
    import torch
    dev = lat.Lattice(pd)
    dev.set_populations(torch.from_numpy(n0))
    dev.tape_begin(K)
    dev.step(T)
    dn0, dg = dev.backward(w)
    dev.close()
    return dn0.cpu(), dg


@pytest.mark.parametrize("case", ["f32", "bf16", "f16", "walls", "long"])
def test_fluid_moments_tape_bitwise(orc, lat, case):
    import torch
    rng = np.random.default_rng(3)
    nz = 8
    po, pd = pair(orc, lat, 12, 10, nz, kT=1e-4, seed=7, g=(1e-4, -5e-5, 2e-5), gamma_shear=0.2, gamma_bulk=-0.1,
                  gamma_3a=0.3, gamma_3b=-0.2, gamma_4a=0.1, gamma_4b=0.4)
    if case in ("bf16", "f16"):
        pd.storage = case
    if case == "walls":
        pd.walls = True
    T = 70 if case == "long" else 13  # 70: past the first 64-step chunk of the tape
    n0 = orc.init_equilibrium(po, u=rng.normal(scale=0.02, size=(3, nz, 10, 12)))
    w = torch.from_numpy(rng.normal(size=n0.shape))
    ref = fluid_grads(lat, pd, n0, w, 4, T)
    kept = fluid_grads(lat, pd, n0, w, T, T)
    got = fluid_grads(lat, pd, n0, w, 0, T)
    for other in (ref, kept):
        assert torch.equal(got[0], other[0]), float((got[0] - other[0]).abs().max())
        assert tuple(got[1]) == tuple(other[1])
    if case in ("f32", "long"):
        dev = lat.Lattice(pd)
        dev.set_populations(torch.from_numpy(n0))
        n0r = dev.get_populations().cpu().numpy()
        dev.close()
        lam, gbar = orc.backward(po, n0r, T, w.numpy())
        err = rel_err(got[0].numpy(), lam)
        print(f"{case}: moments tape vs oracle adjoint {err:.2e}")
        assert err <= REL_TOL
        np.testing.assert_allclose(got[1], gbar, rtol=REL_TOL * 10, atol=1e-6 * np.abs(gbar).max())


def coupled_grads(lat, pd, n0, make_beads, T, K, w, a, b, fused, plain=()):
    import torch
    dev = lat.Lattice(pd)
    dev.set_populations(torch.from_numpy(n0))
    n0r = dev.get_populations().cpu().numpy()
    db = make_beads()
    dev.tape_begin(K)
    if fused and not plain:
        dev.coupled_steps(db, T)
    else:
        for t in range(T):
            if t in plain:
                dev.step(1)
            else:
                dev.coupled_step(db)
    dn0, dg, dR0, dP0 = dev.backward_coupled(torch.from_numpy(w), torch.from_numpy(a), torch.from_numpy(b))
    out = dn0.cpu().numpy(), np.array(dg), dR0.cpu().numpy(), dP0.cpu().numpy()
    dev.close()
    return n0r, out


def compare(got, ref, tol, what):
    errs = [rel_err(x, y) for x, y in zip(got, ref)]
    print(what, "(n0, g, R0, P0):", ["%.2e" % e for e in errs])
    assert max(errs) <= tol


@pytest.mark.parametrize("fused,storage", [(True, "f32"), (False, "f32"), (True, "bf16")])
def test_coupled_moments_tape_matches_oracle(orc, lat, fused, storage):
    """BF16 storage: against the checkpointed tape only (the oracle runs in
    FP64, the stored trajectory in BF16)."""
    rng = np.random.default_rng(5)
    po, pd, n0, ob, db = system(orc, lat, rng, kT=1e-4, seed=5, g=(1e-4, -5e-5, 2e-5), gamma_shear=0.2,
                                gamma_bulk=-0.1)
    pd.storage = storage
    T = 8
    w = rng.normal(size=n0.shape)
    a, b = rng.normal(size=(ob.pos.shape[0], 3)), rng.normal(size=(ob.pos.shape[0], 3))

    def make():
        return lat.DeviceBeads(ob.pos.copy(), ob.mom.copy(), ob.mass.copy(), ob.zeta.copy(), ob.bonds.copy(), 0.05,
                               1.0)

    n0r, got = coupled_grads(lat, pd, n0, make, T, 0, w, a, b, fused)
    _, ref = coupled_grads(lat, pd, n0, make, T, 3, w, a, b, fused)
    if storage == "f32":
        lam0, gbar, pb0, mb0 = orc.backward_coupled(po, n0r, T, ob, w, a, b)
        compare(got, (lam0, gbar, pb0, mb0), REL_TOL, "moments tape vs oracle")
    compare(got, ref, 1e-5, "moments tape vs checkpoints every 3")


@pytest.mark.parametrize("fused", [True, False])
def test_kg_moments_tape_matches_oracle(orc, lat, fused):
    """Kremer-Grest chains (FENE bonds, WCA pairs): the fused launches build
    their cell lists and write the moments in the same launch."""
    from paper_0803_2826_amd.inputs import kremer_grest_chains
    rng = np.random.default_rng(11)
    L, eps = 10, 1e-3
    po = orc.Params(nx=L, ny=L, nz=L, kT=1e-4, seed=6, g=(1e-4, -5e-5, 2e-5))
    pd = lat.FluidParams(nx=L, ny=L, nz=L, kT=po.kT, seed=po.seed, body_force=po.g, track_totals=False)
    pos, _, bonds = kremer_grest_chains(4, 8, (L, L, L), seed=3)
    nb = pos.shape[0]
    mom = rng.normal(scale=0.01, size=(nb, 3))
    zeta = np.full(nb, 0.5)
    ob = orc.Beads(pos.copy(), mom.copy(), np.ones(nb), zeta, bonds.copy(), 30 * eps, 1.5, fene=True, wca_eps=eps,
                   wca_sigma=1.0)

    def make():
        return lat.DeviceBeads(pos.copy(), mom.copy(), np.ones(nb), zeta, bonds, 30 * eps, 1.5, bond="fene",
                               wca_epsilon=eps, wca_sigma=1.0)

    n0 = orc.init_equilibrium(po, u=rng.normal(scale=0.02, size=(3, L, L, L)))
    T = 8
    w = rng.normal(size=n0.shape)
    a, b = rng.normal(size=(nb, 3)), rng.normal(size=(nb, 3))
    n0r, got = coupled_grads(lat, pd, n0, make, T, 0, w, a, b, fused)
    lam0, gbar, pb0, mb0 = orc.backward_coupled(po, n0r, T, ob, w, a, b)
    compare(got, (lam0, gbar, pb0, mb0), REL_TOL, "KG moments tape vs oracle")


def test_mixed_moments_tape_matches_oracle(orc, lat):
    """Plain steps (lb_step on the tape) between coupled ones, a plain first
    and last step."""
    rng = np.random.default_rng(1)
    po, pd, n0, ob, db = system(orc, lat, rng, kT=1e-4, seed=9, g=(5e-5, 0.0, -2e-5))
    T, plain = 7, (0, 3, 6)
    w = rng.normal(size=n0.shape)
    a, b = rng.normal(size=(ob.pos.shape[0], 3)), rng.normal(size=(ob.pos.shape[0], 3))
    n0r, got = coupled_grads(lat, pd, n0, lambda: db, T, 0, w, a, b, False, plain=plain)
    lam0, gbar, pb0, mb0 = oracle_mixed_backward(orc, po, n0r, ob, T, plain, w, a, b)
    compare(got, (lam0, gbar, pb0, mb0), REL_TOL, "mixed moments tape vs oracle")


def test_phi3_moments_tape_matches_checkpoints(orc, lat):
    """phi_3 on a moments tape: lb_coupled_steps takes the separate
    launches; the gradients of a checkpointed tape to 1e-5."""
    rng = np.random.default_rng(21)
    po, pd, n0, ob, db = system(orc, lat, rng, kT=1e-4, seed=4, g=(2e-5, 1e-5, 0.0))
    T = 6
    w = rng.normal(size=n0.shape)
    a, b = rng.normal(size=(ob.pos.shape[0], 3)), rng.normal(size=(ob.pos.shape[0], 3))
    pos, mom = ob.pos.copy(), ob.mom.copy()

    def make():
        return lat.DeviceBeads(pos.copy(), mom.copy(), ob.mass.copy(), ob.zeta.copy(), ob.bonds.copy(), 0.05, 1.0,
                               stencil=3)

    _, got = coupled_grads(lat, pd, n0, make, T, 0, w, a, b, True)
    _, ref = coupled_grads(lat, pd, n0, make, T, 4, w, a, b, True)
    compare(got, ref, 1e-5, "phi_3 moments tape vs checkpoints every 4")


def test_moments_tape_bookkeeping(orc, lat):
    import torch
    from paper_0803_2826_amd._lib import LB_ESTATE, LBError
    rng = np.random.default_rng(8)
    po, pd = pair(orc, lat, 10, 9, 8, kT=1e-4, seed=2)
    pd.track_totals = True
    n0 = orc.init_equilibrium(po, u=rng.normal(scale=0.02, size=(3, 8, 9, 10)))
    w = torch.from_numpy(rng.normal(size=n0.shape))
    dev = lat.Lattice(pd)
    dev.set_populations(torch.from_numpy(n0))
    # no taped steps: the sweep hands dL/dn(T) back unchanged
    dev.tape_begin(0)
    dn0, dg = dev.backward(w)
    assert torch.allclose(dn0.cpu(), w.to(dn0.dtype), rtol=0, atol=1e-7 * float(w.abs().max()))
    assert tuple(dg) == (0.0, 0.0, 0.0)
    # taped steps take no fused totals: lb_totals forms them from the state
    dev.tape_begin(0)
    dev.step(5)
    tot = dev.totals()
    exact = dev.totals(exact=True)
    assert tuple(tot) == tuple(exact)
    # two sweeps over one tape agree
    first = dev.backward(w)
    second = dev.backward(w)
    assert torch.equal(first[0], second[0]) and tuple(first[1]) == tuple(second[1])
    # replacing the state ends the tape
    dev.set_populations(torch.from_numpy(n0))
    with pytest.raises(LBError) as ei:
        dev.backward(w)
    assert ei.value.code == LB_ESTATE
    dev.close()
