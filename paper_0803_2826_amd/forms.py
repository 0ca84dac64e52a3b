"""Measurement helpers of the three forms beside the plain FP32 path.

precision_study  storage FP32 / BF16 / FP16 (shifted deviations, FP32
                 collision arithmetic), 16-bit stores rounded to nearest or
                 stochastically: decay rate of a shear wave and the
                 stationary per-mode noise variances, each against its closed
                 form, plus MLUPS.
batch_study      many uneven replica boxes in one persistent launch per step
                 (HIP graph replay): MLUPS and the ensemble VACF.
differentiation_study
                 the differentiation workload (inputs.DIFF_WORKLOAD): taped
                 forward, the loss gradient at the final state, the reverse
                 sweep (lb_backward_coupled), with their timings and the
                 gradients w.r.t. n(0), g, R(0), P(0).

The closed forms used as references (both pinned against the FP64 oracle in
the test suite):
  shear wave at gamma = 0: j_x(z, t) = A lambda^t sin(kz),
      lambda = 1 - (2/3) sin^2(k/2);
  stationary variance of mode k: mu w_k rho0 = 3 kT w_k rho0.
Round to nearest on thermally dithered 16-bit values adds a damping
rounding_shrink(storage) per step to every hydrodynamic mode (derivation with
LB_ROUND_NEAREST in the C header); stochastic rounding removes it.
"""
from __future__ import annotations

import math
import time

import numpy as np
import torch

from .inputs import DIFF_WORKLOAD, direction, random_walk_chains, shear_wave
from .lattice import BatchLattice, DeviceBeads, FluidParams, Lattice

W_K = np.array([1, 1 / 3, 1 / 3, 1 / 3, 2 / 3, 4 / 3, 4 / 9, 1 / 9, 1 / 9, 1 / 9, 2 / 3, 2 / 3, 2 / 3, 2 / 9, 2 / 9, 2 / 9,
                2, 4 / 3, 4 / 9])


def rounding_shrink(storage: str) -> float:
    """Mean shrink per round-to-nearest store of a dithered value: u^2 / (32 ln 2),
    u the relative spacing (BF16 2^-7, FP16 2^-10, FP32 2^-23)."""
    u = {"f32": 2.0 ** -23, "bf16": 2.0 ** -7, "f16": 2.0 ** -10}[storage]
    return u * u / (32 * math.log(2))


def _jx_mode(lat: Lattice, nz: int) -> float:
    """Projection of the momentum density j_x on sin(2 pi z / nz)."""
    rho, u = lat.moments()
    jx = (u[0] * rho).mean(dim=(1, 2))  # [nz]
    s = torch.sin(2 * math.pi * torch.arange(nz, device=jx.device, dtype=torch.float64) / nz)
    return float((jx * s).sum() * 2.0 / nz)


def decay_rate(storage: str, nx: int, ny: int, nz: int, steps: int, kT: float, amp: float = 0.01, seed: int = 0,
               samples: int = 20, rounding: str = "nearest"):
    """Fitted per-step decay rate of a shear wave (k = 2 pi / nz), noise
    cancelled by subtracting a run with the same seed and no wave."""
    runs = []
    for a in (amp, 0.0):
        p = FluidParams(nx=nx, ny=ny, nz=nz, storage=storage, kT=kT, seed=seed, track_totals=False,
                        rounding=rounding)
        lat = Lattice(p)
        lat.init_equilibrium(u=shear_wave(nx, ny, nz, a))
        series = [_jx_mode(lat, nz)]
        per = steps // samples
        for _ in range(samples):
            lat.step(per)
            series.append(_jx_mode(lat, nz))
        lat.close()
        runs.append(np.array(series))
    diff = runs[0] - runs[1]
    t = np.arange(samples + 1) * (steps // samples)
    slope = np.polyfit(t, np.log(np.abs(diff)), 1)[0]
    lam = 1 - (2 / 3) * math.sin(math.pi / nz) ** 2
    exact = -math.log(lam)
    return {"rate": -slope, "rate_exact": exact, "rel_err": (-slope - exact) / exact,
            "amp_final": float(diff[-1]), "amp_final_exact": amp * lam ** t[-1]}


def mode_variances(storage: str, L: int, kT: float, steps: int, seed: int = 1, samples: int = 10,
                   rounding: str = "nearest"):
    """Stationary per-mode variances / (3 kT w_k rho0)."""
    p = FluidParams(nx=L, ny=L, nz=L, storage=storage, kT=kT, seed=seed, track_totals=False, rounding=rounding)
    lat = Lattice(p)
    lat.init_equilibrium()
    lat.step(steps)
    acc = np.zeros(19)
    for _ in range(samples):
        lat.step(5)
        acc += np.array(lat.mode_stats())
    lat.close()
    return acc / samples / (3 * kT * W_K)


def step_mlups(storage: str, L: int, kT: float, steps: int = 50, rounding: str = "nearest") -> float:
    p = FluidParams(nx=L, ny=L, nz=L, storage=storage, kT=kT, seed=0, track_totals=True, rounding=rounding)
    lat = Lattice(p)
    lat.init_equilibrium()
    lat.step(5)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(lat.stream)
    lat.step(steps)
    e1.record(lat.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    lat.close()
    return L ** 3 / (ms * 1e-3) / 1e6


def precision_study(decay_box=(8, 8, 512), decay_steps=2000, var_L=32, var_steps=300, kT=1e-4, mlups_L=256):
    out = {}
    for st, rd in (("f32", "nearest"), ("bf16", "nearest"), ("f16", "nearest"), ("bf16", "stochastic"),
                   ("f16", "stochastic")):
        d = decay_rate(st, *decay_box, steps=decay_steps, kT=kT, rounding=rd)
        v = mode_variances(st, var_L, kT, var_steps, rounding=rd)
        shrink = rounding_shrink(st) if rd == "nearest" else 0.0
        out[f"{st}-{rd}"] = {"decay_rate_rel_err": d["rel_err"],
                             "predicted_rel_err": shrink / d["rate_exact"],
                             "mode_var_ratio_max_dev": float(np.abs(v - 1).max()),
                             "mode_var_ratio": [round(float(x), 4) for x in v],
                             "mlups": step_mlups(st, mlups_L, kT, rounding=rd) if mlups_L else None}
    return out


def edge_draws(nbox: int, seed: int = 0, choices=(24, 32, 40, 48, 64)):
    """Replica box edges drawn uniformly from `choices` (seeded numpy PCG64)."""
    rng = np.random.default_rng(seed)
    e = rng.choice(np.asarray(choices), size=nbox)
    return [(int(v), int(v), int(v)) for v in e]


def batch_study(nbox: int = 512, steps: int = 500, kT: float = 1e-4, lags: int = 32, graph_steps: int = 10,
                seed: int = 0, block: int = 0):
    dims = edge_draws(nbox, seed)
    p = FluidParams(nx=2, ny=2, nz=2, kT=kT, seed=seed, vacf_lags=lags, graph_steps=graph_steps, block=block)
    B = BatchLattice(p, dims)
    B.init_equilibrium()
    B.step(graph_steps)  # launch-configuration search happens on the first step
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(B.stream)
    B.step(steps)
    e1.record(B.stream)
    torch.cuda.synchronize()
    ms = max(e0.elapsed_time(e1), (time.perf_counter() - t0) * 1e3) / steps
    C, ns = B.vacf() if lags > 0 else (None, 0)
    cfg = B.launch_config()
    edges = np.array([d[0] for d in dims])
    by_L = {}
    for Lb in (sorted(set(edges.tolist())) if lags > 0 else []):
        sel = edges == Lb
        lam = 1 - (2 / 3) * math.sin(math.pi / Lb) ** 2
        c = C[sel].mean(axis=0)
        ratio = c / c[0]
        pw = lam ** np.arange(len(c))
        by_L[int(Lb)] = {"count": int(sel.sum()), "C0": float(c[0]), "C_ratio": [float(x) for x in ratio[:8]],
                         "lambda_pow": [float(x) for x in pw[:8]],
                         "max_abs_dev": float(np.abs(ratio - pw).max())}
    B.close()
    return {"sites": int(sum(d[0] * d[1] * d[2] for d in dims)), "ms_per_step": ms,
            "mlups": sum(d[0] * d[1] * d[2] for d in dims) / (ms * 1e-3) / 1e6, "launch": cfg, "samples": ns,
            "vacf_by_edge": by_L}


def settling_study(L: int = 16, steps: int = 2500, a0: float = 1.0, force: float = 1e-4, stencils=(2, 3, 4)):
    """Grid dependence of a point particle's mobility (Sec. "Interpolating
    functions", the settling experiment): one bead of input radius a0 (bare
    friction Gamma = 6 pi eta a0, eta = 1/6 at gamma = 0) held at the
    positions (i, j, k)/10 + 3 (0 <= i <= j <= k <= 5, 56 positions) of an
    L^3 periodic box at kT = 0 under an external force F along x, with the
    compensating uniform force density -F/L^3 on the fluid so that the net
    force is zero.  After `steps` coupled steps (position reset every step,
    momentum kept) the steady velocity U = P/m gives 1/a = 6 pi eta U/F and
    the kernel's radius parameter g from eq. aeffcorr,
    1/(g b) = 1/a + 2.84/L - 1/a0 (b = 1).  Returns, per kernel width, the
    mobilities, the g values and the largest relative deviation of g from
    its mean over the positions."""
    eta = 1.0 / 6.0
    zeta = 6.0 * math.pi * eta * a0
    out = {}
    positions = [(i, j, k) for k in range(6) for j in range(k + 1) for i in range(j + 1)]
    for W in stencils:
        mob = []
        for i, j, k in positions:
            R0 = torch.tensor([[3 + i / 10, 3 + j / 10, 3 + k / 10]], dtype=torch.float64, device="cuda")
            p = FluidParams(nx=L, ny=L, nz=L, body_force=(-force / L ** 3, 0.0, 0.0), track_totals=False)
            lat = Lattice(p)
            lat.init_equilibrium()
            b = DeviceBeads(R0.cpu().numpy(), np.zeros((1, 3)), np.ones(1), np.full(1, zeta), stencil=W,
                            fext=np.array([[force, 0.0, 0.0]]))
            for _ in range(steps):
                lat.coupled_step(b)
                b.pos.copy_(R0)
            torch.cuda.synchronize()
            mob.append(float(b.mom[0, 0]) / force)
            lat.close()
        mob = np.array(mob)
        inv_a = 6.0 * math.pi * eta * mob
        g = 1.0 / (inv_a + 2.84 / L - 1.0 / a0)
        out[W] = {"mobility": mob.tolist(), "g": g.tolist(), "g_mean": float(g.mean()),
                  "g_max_dev": float(np.abs(g / g.mean() - 1).max()),
                  "mobility_spread": float((mob.max() - mob.min()) / mob.mean())}
    return out



def differentiation_study(checkpoint_every: int, steps: int | None = None, workload: dict = DIFF_WORKLOAD):
    """One run of the differentiation workload: `steps` coupled steps from the
    fluid at rest with the workload's chains, taped with a checkpoint every
    `checkpoint_every` steps (the step buffers are allocated before the
    timed forward), the probe + drag loss at the final state (its gradient
    w.r.t. n(T), R(T), P(T) and its direct dependence on g through
    u = (sum n c + g/2)/rho, by torch autograd), then the reverse sweep.
    Returns the timings (events on the context stream), the loss and the
    gradients (dL/dn(0) [19 N] float64, dL/dg [3], dL/dR(0), dL/dP(0)
    [n, 3]) on the host."""
    from .autograd import probe_drag_loss
    W = workload
    L, T = W["L"], steps or W["steps"]
    lo, hi = W["probe"]
    p = FluidParams(nx=L, ny=L, nz=L, kT=W["kT"], seed=W["seed"], body_force=W["g"], track_totals=False)
    lat = Lattice(p)
    lat.init_equilibrium()
    pos, mom, bonds = random_walk_chains(W["chains"], W["length"], (L, L, L), seed=W["chain_seed"])
    nb = pos.shape[0]
    beads = DeviceBeads(pos, mom, np.full(nb, W["mass"]), np.full(nb, W["zeta"]), bonds, W["k_bond"], W["r0"])
    lat.tape_begin(checkpoint_every)  # allocates the segment buffer outside the timed region
    lat.tape_begin(checkpoint_every)
    lat.tape_reserve(T, beads)  # ... and the checkpoints and the bead tape
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    torch.cuda.synchronize()
    ev[0].record(lat.stream)
    lat.coupled_steps(beads, T)
    ev[1].record(lat.stream)
    nT = lat.get_populations(dtype=torch.float64).requires_grad_()
    g_t = torch.tensor(W["g"], dtype=torch.float64, device=nT.device, requires_grad=True)
    RT = beads.pos.detach().clone().requires_grad_()
    PT = beads.mom.detach().clone().requires_grad_()
    loss = probe_drag_loss(nT, g_t, RT, PT, beads.mass, beads.zeta, lo, hi)
    loss.backward()
    torch.cuda.synchronize()
    ev[2].record(lat.stream)
    dn0, dg, dR0, dP0 = lat.backward_coupled(nT.grad.contiguous(), RT.grad, PT.grad)
    ev[3].record(lat.stream)
    torch.cuda.synchronize()
    out = {"sites": L ** 3, "steps": T, "checkpoint_every": checkpoint_every,
           "forward_ms": ev[0].elapsed_time(ev[1]), "backward_ms": ev[2].elapsed_time(ev[3]),
           "loss": float(loss.detach()),
           "dn0": dn0.detach().reshape(-1).double().cpu().numpy(),
           "dg": np.asarray(dg, dtype=np.float64) + g_t.grad.detach().cpu().numpy(),
           "dR0": dR0.detach().cpu().numpy(), "dP0": dP0.detach().cpu().numpy()}
    lat.close()
    return out


def elementwise_errors(study: dict, ref: dict) -> dict:
    """Element-wise errors of a differentiation_study gradient against a
    stored FP64 adjoint of the same run (dL/dg, dL/dR(0), dL/dP(0) in full,
    dL/dn(0) at the stored indices), each relative to the largest entry of
    the stored gradient."""
    dn = np.asarray(study["dn0"]).reshape(-1)
    idx = np.asarray(ref["dn0_index"])
    out = {"dn0": float(np.abs(dn[idx] - np.asarray(ref["dn0_sample"])).max() / ref["dn0_max_abs"])}
    for k in ("dg", "dR0", "dP0"):
        r = np.asarray(ref[k], dtype=np.float64)
        out[k] = float(np.abs(np.asarray(study[k]) - r).max() / np.abs(r).max())
    return out


def directional_errors(study: dict, golden: dict) -> list:
    """Errors of <grad, v> from a differentiation_study against the stored
    central differences d_v L of the FP64 oracle (one per seeded direction
    of inputs.direction).  A random direction makes <grad, v> a sum of ~4e7
    terms of both signs that cancel to a small fraction of their magnitudes,
    so the error is stated relative to the sum of the terms' magnitudes,
    sum_i |g_i v_i| (rel_err, the dot product's own scale, as the
    element-wise error is relative to the largest gradient entry); the error
    relative to d_v L itself (rel_err_signed) and the ratio of the two
    scales (cancellation) are given beside it, and the loss against the
    mean of L(x +- eps v)."""
    out = []
    nb = study["dR0"].shape[0]
    for d in golden["directions"]:
        vn, vg, vR, vP = direction(study["dn0"].size, nb, d["seed"])
        terms = (study["dn0"] * vn, study["dg"] * vg, study["dR0"] * vR, study["dP0"] * vP)
        got = float(sum(t.sum() for t in terms))
        scale = float(sum(np.abs(t).sum() for t in terms))
        diff = abs(got - d["d_v_L"])
        out.append({"seed": d["seed"], "gpu": got, "oracle_fd": d["d_v_L"], "rel_err": diff / scale,
                    "rel_err_signed": diff / abs(d["d_v_L"]), "cancellation": scale / abs(d["d_v_L"]),
                    "loss_rel_err": abs(study["loss"] - d["L_mid"]) / abs(d["L_mid"])})
    return out
