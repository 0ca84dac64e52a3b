"""The differentiation workload end to end on the GPU (inputs.DIFF_WORKLOAD:
128^3 from rest, kT 1e-4, 16 chains x 32 beads with zeta 20 and k 10 kT, the
probe + drag loss of the final state, gradients w.r.t. n(0), g, R(0), P(0)),
through forms.differentiation_study, the code path bench.py times (fused
coupled steps, lb_coupled_steps, taped with a checkpoint every 50 steps: the
restore and recompute run nine times; and taped with a moments tape, the
reverse sweep reading every step's moments, recomputing nothing).

- 500 coupled steps, directional derivatives <grad, v> along the two seeded
  directions of tests/golden/c5_directional.json against the FP64 oracle's
  central differences stored there (eps = 3e-5; written by
  make_c5_directional.py, oracle only).  Bar 1e-6, the workload's target, on
  the error relative to the scale of the dot product, sum_i |g_i v_i|: a
  random direction makes <grad, v> a sum of ~4e7 terms of both signs that
  cancel to ~1e-3 of their magnitudes, so the error relative to <grad, v>
  itself is that cancellation times larger (printed).  The loss: its FP32
  value against the mean of the oracle's L(x +- eps v) (L(x) up to
  O(eps^2)), bar 1e-5 (FP32 trajectory over 500 steps).
- 500 coupled steps, element by element against the oracle's FP64 adjoint
  (tests/golden/c5_adjoint.json, make_c5_adjoint.py: orc.backward_coupled
  over the same ten segments): dL/dn(0) at 20000 seeded indices, relative
  to its largest entry, bar 2e-5 (the FP32 adjoint state: ~6e-8 relative
  rounding per value and step, measured 3e-6); dL/dR(0), dL/dP(0) relative
  to their largest entries, bar 1e-4 (measured 8e-6, 2e-5); dL/dg relative
  to its largest entry, bar 5e-4 (measured 1.6e-4): it collects a term from
  every site and step (1e9 of them, summed in FP64 from FP32 per-site
  values) of the FP32 adjoint state, whose share of it cancels to ~1e-3 of
  its magnitude, so the per-value rounding shows up ~1e3-fold.
- 10 coupled steps (K = 5, two segments): dL/dn(0), dL/dg, dL/dR(0),
  dL/dP(0) element by element against the oracle's FP64 adjoint of whole
  coupled steps (orc.backward_coupled), bar 2e-5 relative to each
  gradient's largest entry, as in test_gpu_adjoint_coupled.
"""
import json
import os

import numpy as np
import pytest

from conftest import gpu_available

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c5_directional.json")
ADJOINT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c5_adjoint.json")


@pytest.fixture(scope="module")
def forms():
    if not gpu_available():
        pytest.skip("no GPU")
    from paper_0803_2826_amd import forms
    return forms


def rel_err(got, ref):
    return float(np.abs(np.asarray(got) - ref).max() / np.abs(ref).max())


@pytest.fixture(scope="module", params=["checkpoints", "moments_tape"])
def study500(forms, request):
    """The 500-step run taped with a checkpoint every 50 steps, and with a
    moments tape (lb_tape_begin(0): every step's (rho - rho0, j) kept,
    nothing recomputed)."""
    from paper_0803_2826_amd.inputs import DIFF_WORKLOAD as W
    K = W["checkpoint_every"] if request.param == "checkpoints" else 0
    print(f"differentiation workload: {W['L']}^3, {W['steps']} coupled steps, K = {K} ({request.param})", flush=True)
    return forms.differentiation_study(K)


def test_c5_500_steps_against_oracle_central_differences(forms, study500):
    from paper_0803_2826_amd.inputs import DIFF_WORKLOAD as W
    with open(GOLDEN) as f:
        golden = json.load(f)
    assert golden["workload"]["L"] == W["L"] and golden["workload"]["steps"] == W["steps"]
    d = study500
    errs = forms.directional_errors(d, golden)
    assert len(errs) == 2
    for e in errs:
        print(f"direction {e['seed']}: gpu {e['gpu']:.12e} oracle fd {e['oracle_fd']:.12e} error "
              f"{e['rel_err']:.2e} of sum |g v| ({e['rel_err_signed']:.2e} of <g, v>, cancellation "
              f"{e['cancellation']:.0f}); loss rel err {e['loss_rel_err']:.2e}", flush=True)
    assert all(np.all(np.isfinite(x)) for x in (d["dn0"], d["dg"], d["dR0"], d["dP0"]))
    assert max(e["rel_err"] for e in errs) <= 1e-6
    assert max(e["loss_rel_err"] for e in errs) <= 1e-5


def test_c5_500_steps_elementwise_against_oracle_adjoint(study500):
    from paper_0803_2826_amd.inputs import DIFF_WORKLOAD as W
    with open(ADJOINT) as f:
        ref = json.load(f)
    assert ref["workload"]["L"] == W["L"] and ref["workload"]["steps"] == W["steps"]
    d = study500
    dn = np.asarray(d["dn0"]).reshape(-1)
    idx = np.asarray(ref["dn0_index"])
    e_n = float(np.abs(dn[idx] - np.asarray(ref["dn0_sample"])).max() / ref["dn0_max_abs"])
    e_g, e_R, e_P = (rel_err(d[k], np.asarray(ref[k])) for k in ("dg", "dR0", "dP0"))
    print(f"500 steps vs the oracle adjoint: dn0 {e_n:.2e} (20000 samples), dg {e_g:.2e}, dR0 {e_R:.2e}, "
          f"dP0 {e_P:.2e} of each largest entry", flush=True)
    assert e_n <= 2e-5
    assert e_R <= 1e-4 and e_P <= 1e-4
    assert e_g <= 5e-4


def test_c5_10_steps_elementwise_against_oracle_adjoint(forms, orc):
    from paper_0803_2826_amd.inputs import DIFF_WORKLOAD as W, random_walk_chains
    from test_gpu_adjoint_coupled import drag_loss_grads
    T, K = 10, 5
    L = W["L"]
    lo, hi = W["probe"]
    d = forms.differentiation_study(K, steps=T)
    po = orc.Params(nx=L, ny=L, nz=L, kT=W["kT"], seed=W["seed"], g=W["g"])
    pos, mom, bonds = random_walk_chains(W["chains"], W["length"], (L, L, L), seed=W["chain_seed"])
    nb = pos.shape[0]
    ob = orc.Beads(pos, mom, np.full(nb, W["mass"]), np.full(nb, W["zeta"]), bonds, W["k_bond"], W["r0"])
    n0 = orc.init_equilibrium(po)  # at rest: n_i = a_i rho0, exact in the device's shifted storage
    n, bb = n0.copy(), ob.copy()
    for t in range(T):
        orc.coupled_step(po, n, t, bb)
    lamT, gdir, dRT, dPT = drag_loss_grads(orc, po, n, bb.pos, bb.mom, ob.mass, ob.zeta, lo, hi)
    del n
    lam0, gbar, dR0, dP0 = orc.backward_coupled(po, n0, T, ob, lamT, dRT, dPT)
    errs = [rel_err(d["dn0"], lam0.reshape(-1)), rel_err(d["dg"], gbar + gdir), rel_err(d["dR0"], dR0),
            rel_err(d["dP0"], dP0)]
    print("128^3, 10 coupled steps, K = 5: rel errors (n0, g, R0, P0):", ["%.2e" % e for e in errs], flush=True)
    assert max(errs) <= 2e-5
