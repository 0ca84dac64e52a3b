#!/usr/bin/env python3
"""Benchmark of the fluctuating D3Q19 hot path on one MI355X.

One step = the whole hot path on the 256^3 workload: bead half-drift, bond
forces, trilinear interpolation, Langevin momentum update and spreading for
64 chains x 32 beads into the force field and its site bitmap, then the fused
pull-stream + MRT collision with thermal noise and forcing (body force plus
the bead force at bitmap-marked sites) over all 16.8M sites, with fused FP64
mass/momentum totals, and the clear of the touched force rows.  Inputs are
synthetic (seeded), resident in HBM before the timed region.

Prints ONE JSON line with, beside the throughput:
  roofline      the dominant kernel (fused stream-collide, bead-force
                variant): algorithmic bytes per launch (19 reads + 19 writes
                of a 4-byte population per site, the read and write of the
                rest population's 4-byte rounding residual that keeps each
                site's mass exact, plus the 1-bit-per-site force bitmap)
                over its average duration, timed with events
                on the launch stream around each step's launch inside the
                timed region, against the 8 TB/s HBM peak, and beside it
                the rate of a plain device copy of one population buffer
                (the practical ceiling of a streaming kernel) and of the
                step's memory pattern alone (19 pulled planes and the
                residual plane, no arithmetic: the ceiling of its access
                pattern);
  cpu_baseline  the FP64 oracle on the host cores, timed on a bounded sample
                of the same workload (a few coupled steps of the full box);
  forms         the other throughputs the metric names: FP32 and BF16-storage
                MLUPS (nearest and stochastic rounding, kT > 0 and kT = 0)
                on the same box without beads and, per storage type, on the
                512^3 box of the precision workload, the batched form (512
                replica boxes, edges drawn from {24, 32, 40, 48, 64}, HIP
                graph replay; with and without the ensemble VACF reduced on
                the device) and the differentiation form (taped forward and
                adjoint of 500 coupled steps at 128^3 with 16 x 32 beads and
                the probe + drag loss, checkpoints every 50 steps, and with
                the whole tape resident in HBM; the gradient's error against
                stored FP64 oracle central differences), and the coupled
                step with Kremer-Grest chains (FENE bonds, WCA pairs with a
                cell list) in place of the harmonic ones.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "MLUPS + % of HBM peak, FP32 vs BF16-storage vs batched; backward MLUPS at 1e-6 err"
HBM_PEAK_GBS = 8000.0
KT = 1e-4
# Bond stiffness "k = 10" read in units of kT / b^2 (the paper quotes its bond
# constants in units of the thermal energy); k = 10 in plain lattice units makes
# the explicit bead-fluid scheme diverge within ten steps at zeta = 20, m = 1.
K_BOND = 10.0 * KT
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_coupled_step_256.json")
# FP64 oracle central differences of the differentiation workload's loss
C5_GOLDEN = os.path.join(ROOT, "tests", "golden", "c5_directional.json")
C5_ADJOINT = os.path.join(ROOT, "tests", "golden", "c5_adjoint.json")
# coupled steps of the workload over which the relative mass drift is reported
DRIFT_STEPS = 1000
# Friction of the Kremer-Grest chains: velocity relaxation time m/zeta = 5 steps
# (0.05 of the Lennard-Jones time sigma sqrt(m/eps) = 100 steps at eps = kT).
# With the harmonic chains' zeta = 20 the beads follow the lattice-scale fluid
# noise so closely that the WCA core (eps = kT) is breached within ~100 steps
# and a FENE bond overstretches, in the FP64 oracle as on the device.
KG_ZETA = 0.2


# everything the timed kernel (k_coupled_step) is built from
KERNEL_SOURCES = ("kernels.h", "collide.h", "rng.h", "aux_kernels.h", "pairs.h", "couple.h", "fused.h")


def source_hash() -> str:
    """Hash of the sources of the timed kernel; the committed PMC traffic
    figure is used only while it matches."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_0803_2826_amd", "csrc")
    for name in KERNEL_SOURCES:
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode())
            h.update(f.read())
    return h.hexdigest()[:16]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--L", type=int, default=256, help="box edge (default: the 256^3 workload)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=8)
    ap.add_argument("--block", type=int, default=-1,
                    help="threads per block of the timed loop's step launches: -1 (default) searches them on the "
                         "first step; a fixed value skips the search (profiling runs whose counters would "
                         "perturb the search's timings)")
    ap.add_argument("--chains", choices=("harmonic", "kg"), default="harmonic",
                    help="bead model of the timed loop: the harmonic chains of the workload (default) or "
                         "Kremer-Grest chains (FENE bonds + WCA pairs, eps = kT) for profiling that path")
    return ap.parse_args()


def cpu_baseline(L: int, n_chains: int, length: int, steps: int):
    """FP64 oracle on the host: `steps` coupled steps of the same workload after
    one untimed warm-up step."""
    import numpy as np

    import oracle
    from paper_0803_2826_amd.inputs import random_walk_chains

    oracle.build()
    pos, mom, bonds = random_walk_chains(n_chains, length, (L, L, L), seed=0)
    nb = pos.shape[0]
    p = oracle.Params(nx=L, ny=L, nz=L, kT=1e-4, seed=0)
    beads = oracle.Beads(pos, mom, np.ones(nb), np.full(nb, 20.0), bonds, K_BOND, 1.0)
    n = oracle.init_equilibrium(p)
    oracle.coupled_step(p, n, 0, beads)
    t0 = time.perf_counter()
    for t in range(steps):
        oracle.coupled_step(p, n, 1 + t, beads)
    dt = time.perf_counter() - t0
    del n
    return {
        "value": L ** 3 * steps / dt / 1e6,
        "unit": "MLUPS",
        "cores": oracle.num_threads(),
        "kind": "oracle",
        "sample": f"{steps} coupled steps (after 1 warm-up) of the full {L}^3 box with {n_chains}x{length} beads, "
                  f"FP64, OpenMP over sites; {dt:.1f} s",
    }


def run_forms(L: int) -> dict:
    """Throughputs of the precision, batched and differentiation forms (each
    after its own warm-up, timed with events on the context stream)."""
    import torch

    from paper_0803_2826_amd import forms, lattice
    from paper_0803_2826_amd.inputs import DIFF_WORKLOAD

    import numpy as np

    out = {}
    for kT in (KT, 0.0):
        out[f"f32_fluid_only_kT{kT:g}_mlups"] = round(forms.step_mlups("f32", L, kT, steps=100), 1)
    for st, rd in (("bf16", "nearest"), ("bf16", "stochastic")):
        out[f"{st}_{rd}_mlups"] = round(forms.step_mlups(st, L, KT, steps=100, rounding=rd), 1)
    out["bf16_nearest_kT0_mlups"] = round(forms.step_mlups("bf16", L, 0.0, steps=100), 1)
    # the precision workload's own box: 512^3, kT = 1e-4, per storage type and rounding
    out["precision_512_mlups"] = {
        f"{st}_{rd}": round(forms.step_mlups(st, 512, KT, steps=50, rounding=rd), 1)
        for st, rd in (("f32", "nearest"), ("bf16", "nearest"), ("bf16", "stochastic"), ("f16", "nearest"),
                       ("f16", "stochastic"))}
    # errors of each storage form against closed forms that the oracle pins:
    # the decay rate of the 512^3 workload's shear wave (k = 2 pi / 512, on a
    # 64 x 64 x 512 box: the same wave and per-site statistics) against
    # -ln lambda(k), beside the rate change round-to-nearest is predicted to
    # add; the stationary per-mode variances (32^3) against 3 kT w_k rho0
    errs = {}
    for st, rd in (("f32", "nearest"), ("bf16", "nearest"), ("bf16", "stochastic"), ("f16", "nearest"),
                   ("f16", "stochastic")):
        d = forms.decay_rate(st, 64, 64, 512, steps=2000, kT=KT, rounding=rd)
        v = forms.mode_variances(st, 32, KT, 300, rounding=rd)
        errs[f"{st}_{rd}"] = {
            "decay_rate_rel_err": round(float(d["rel_err"]), 5),
            "decay_rate_rel_err_predicted": round(forms.rounding_shrink(st) / d["rate_exact"], 5) if rd == "nearest"
            else 0.0,
            "mode_variance_max_rel_dev": round(float(np.abs(v - 1.0).max()), 6)}
    out["precision_errors"] = errs
    print("# forms: precision done", file=sys.stderr, flush=True)
    b = forms.batch_study(nbox=512, steps=200, kT=KT, lags=0, graph_steps=10)
    out["batched_mlups"] = round(b["mlups"], 1)
    out["batched_sites"] = b["sites"]
    # the batched workload as specified: 500 steps, the ensemble VACF of
    # every replica sampled and reduced on the device every step (persistent
    # launch), graph replay; C(tau)/C(0) per edge class against lambda(k)^tau
    bv = forms.batch_study(nbox=512, steps=500, kT=KT, lags=32, graph_steps=10)
    out["batched_vacf_mlups"] = round(bv["mlups"], 1)
    out["batched_vacf_launch"] = {"threads": bv["launch"][0], "blocks": bv["launch"][1],
                                  "tiles_per_block": bv["launch"][2]}
    out["batched_vacf_max_abs_dev"] = {str(k): round(v["max_abs_dev"], 4) for k, v in bv["vacf_by_edge"].items()}
    out["batched_vacf_edge_counts"] = {str(k): v["count"] for k, v in bv["vacf_by_edge"].items()}
    print("# forms: batch done", file=sys.stderr, flush=True)

    # the differentiation workload (128^3, 16 x 32 beads, 500 coupled steps,
    # probe + drag loss): checkpoints every 50 steps (the workload's own
    # interval; the reverse sweep recomputes all but the last segment), the
    # whole tape resident in HBM (84 GB, nothing recomputed), and a moments
    # tape (every step's rho - rho0 and j, 16.8 GB, nothing recomputed); the
    # error of the timed K = 50 gradient against the FP64 oracle's central
    # differences along seeded directions, stored by
    # tests/golden/make_c5_directional.py
    W = DIFF_WORKLOAD
    for K, tag in ((W["checkpoint_every"], ""), (W["steps"], "_tape_resident"), (0, "_moments_tape")):
        d = forms.differentiation_study(K)
        out["taped_forward_mlups" + tag] = round(d["sites"] * d["steps"] / (d["forward_ms"] * 1e-3) / 1e6, 1)
        out["backward_mlups" + tag] = round(d["sites"] * d["steps"] / (d["backward_ms"] * 1e-3) / 1e6, 1)
        if tag == "" and os.path.exists(C5_GOLDEN):
            with open(C5_GOLDEN) as f:
                golden = json.load(f)
            errs = forms.directional_errors(d, golden)
            out["backward_grad_rel_err"] = max(e["rel_err"] for e in errs)
            out["backward_grad_check"] = [{k: e[k] for k in ("seed", "gpu", "oracle_fd", "rel_err", "rel_err_signed",
                                                             "cancellation", "loss_rel_err")} for e in errs]
        if tag != "_tape_resident" and os.path.exists(C5_ADJOINT):
            with open(C5_ADJOINT) as f:
                ref = json.load(f)
            out["backward_grad_elementwise" + tag] = {k: float(f"{v:.3e}")
                                                      for k, v in forms.elementwise_errors(d, ref).items()}
        del d
    out["backward_config"] = (f"{W['L']}^3, {W['steps']} coupled steps from rest with {W['chains']} x "
                              f"{W['length']} beads (zeta {W['zeta']:g}, k 10 kT), probe + drag loss; "
                              f"checkpoints every {W['checkpoint_every']} steps (_tape_resident: all {W['steps']} "
                              f"step buffers kept, nothing recomputed; _moments_tape: every step's rho - rho0 and "
                              f"j kept, 16 B per site, nothing recomputed); FP32 fluid, FP64 beads; gradients w.r.t. "
                              f"n(0), g, R(0), P(0); grad error: directional derivatives along seeded random "
                              f"directions against FP64 oracle central differences (eps 3e-5), relative to "
                              f"sum |g_i v_i|; elementwise: against the FP64 oracle's adjoint of the same 500 "
                              f"steps, relative to each gradient's largest entry (dn0 at 20000 seeded indices); "
                              f"forward: fused coupled steps (lb_coupled_steps)")
    print("# forms: backward done", file=sys.stderr, flush=True)

    # Kremer-Grest chains: the same box and chain count with FENE bonds and
    # WCA pairs (cell list rebuilt every step), eps = kT, sigma = 1
    from paper_0803_2826_amd.inputs import kremer_grest_chains

    pk = lattice.FluidParams(nx=L, ny=L, nz=L, kT=KT, seed=0, track_totals=True, block=-1)
    lat = lattice.Lattice(pk)
    lat.init_equilibrium()
    pos, mom, bonds = kremer_grest_chains(64, 32, (L, L, L), seed=0)
    nb = pos.shape[0]
    kg = lattice.DeviceBeads(pos, mom, np.ones(nb), np.full(nb, KG_ZETA), bonds, 30 * KT, 1.5, bond="fene",
                             wca_epsilon=KT, wca_sigma=1.0)
    lat.step(1)
    lat.coupled_steps(kg, 20)
    Tk = 100
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    half = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(Tk)]
    torch.cuda.synchronize()
    # one launch per coupled step (the cell lists built by the launches)
    ev[0].record(lat.stream)
    lat.coupled_steps(kg, Tk)
    ev[1].record(lat.stream)
    # the separate launches, with the particle half timed on its own
    ev[2].record(lat.stream)
    for h0, h1 in half:
        h0.record(lat.stream)
        lat.couple(kg)
        h1.record(lat.stream)
        lat.step(1)
    ev[3].record(lat.stream)
    torch.cuda.synchronize()
    lat.sync()
    lat.close()
    ms = ev[0].elapsed_time(ev[1]) / Tk
    out["kg_coupled_mlups"] = round(L ** 3 / (ms * 1e-3) / 1e6, 1)
    out["kg_coupled_mlups_separate_launches"] = round(L ** 3 / (ev[2].elapsed_time(ev[3]) / Tk * 1e-3) / 1e6, 1)
    out["kg_particle_half_ms"] = round(sum(a.elapsed_time(b) for a, b in half) / Tk, 4)
    out["kg_config"] = (f"{L}^3 fluid as above, 64 x 32 Kremer-Grest chains: FENE k = 30 kT, R0 = 1.5, WCA "
                        f"eps = kT, sigma = 1 (cell list), zeta = {KG_ZETA}, m = 1")
    print("# forms: Kremer-Grest done", file=sys.stderr, flush=True)
    return out


def main() -> int:
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU path is "
              f"design-only in this build.", file=sys.stderr)
        return 2
    import numpy as np
    import torch

    from paper_0803_2826_amd import lattice
    from paper_0803_2826_amd.inputs import random_walk_chains

    torch.cuda.set_device(0)
    L = args.L
    n_chains, length = 64, 32
    N = L ** 3
    pd = lattice.FluidParams(nx=L, ny=L, nz=L, storage="f32", kT=KT, seed=0, track_totals=True, block=args.block)
    lat = lattice.Lattice(pd)
    lat.init_equilibrium()
    if args.chains == "kg":
        from paper_0803_2826_amd.inputs import kremer_grest_chains

        pos, mom, bonds = kremer_grest_chains(n_chains, length, (L, L, L), seed=0)
        nb = pos.shape[0]
        beads = lattice.DeviceBeads(pos, mom, np.ones(nb), np.full(nb, KG_ZETA), bonds, 30 * KT, 1.5, bond="fene",
                                    wca_epsilon=KT, wca_sigma=1.0)
        chain_desc = f"Kremer-Grest chains (FENE k=30 kT, R0=1.5; WCA eps=kT, sigma=1), zeta={KG_ZETA}, m=1"
    else:
        pos, mom, bonds = random_walk_chains(n_chains, length, (L, L, L), seed=0)
        nb = pos.shape[0]
        beads = lattice.DeviceBeads(pos, mom, np.ones(nb), np.full(nb, 20.0), bonds, K_BOND, 1.0)
        chain_desc = "(k=10 kT/b^2, r0=1, zeta=20, m=1)"
    tot0 = lat.totals(exact=True)
    stream = lat.stream

    # warm-up (the first steps with and without bead force search the launch
    # configuration of their kernel variant)
    lat.step(1)
    lat.coupled_steps(beads, args.warmup)
    torch.cuda.synchronize()
    print(f"# warmup done ({args.warmup} steps)", file=sys.stderr, flush=True)

    # the timed region: one lb_coupled_steps call, one launch per coupled
    # step (the particle half in the first blocks of the step's grid)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    ev0.record(stream)
    lat.coupled_steps(beads, args.steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    gpu_ms = ev0.elapsed_time(ev1)
    ms_per_step = max(gpu_ms, wall * 1e3) / args.steps
    mlups = N / (ms_per_step * 1e-3) / 1e6
    # the launches are back to back: their average duration is the events'
    # span per step (which also holds the call's prologue, the first step's
    # node bitmap and the bond table upload)
    kern_ms = gpu_ms / args.steps
    print(f"# timed {args.steps} steps: {ms_per_step:.4f} ms/step, {mlups:.0f} MLUPS; fused kernel {kern_ms:.4f} ms",
          file=sys.stderr, flush=True)
    # the separate launches (lb_couple, then lb_step) and the particle half
    # alone, after the timed region (reported, not part of the throughput)
    cev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True),
            torch.cuda.Event(enable_timing=True)) for _ in range(50)]
    for c0, c1, c2 in cev:
        c0.record(stream)
        lat.couple(beads)
        c1.record(stream)
        lat.step(1)
        c2.record(stream)
    torch.cuda.synchronize()
    half_ms = sum(c0.elapsed_time(c1) for c0, c1, _ in cev) / len(cev)
    sep_ms = sum(c0.elapsed_time(c2) for c0, _, c2 in cev) / len(cev)
    sep_kern_ms = sum(c1.elapsed_time(c2) for _, c1, c2 in cev) / len(cev)

    # conservation over at least 1000 coupled steps of the workload (after
    # the timed region, not part of the throughput)
    done = 1 + args.warmup + args.steps + len(cev)
    lat.coupled_steps(beads, max(0, DRIFT_STEPS - done))
    drift_steps = max(done, DRIFT_STEPS)
    tot1 = lat.totals()
    tot1x = lat.totals(exact=True)
    lat.sync()
    cfg = lat.launch_config(force=True)

    planes = 20  # FP32 storage: 19 populations + the rest population's rounding residual
    alg_bytes = 2 * planes * 4 * N + N // 8
    achieved = alg_bytes / (kern_ms * 1e-3) / 1e9
    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        with open(TRAFFIC_FILE) as f:
            tr = json.load(f)
        if tr.get("source_hash") == source_hash() and tr.get("L") == L:
            traffic = tr.get("traffic_bytes_per_launch")
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": "k_coupled_step<f32,thermal,totals,full relaxation,phi_2> (fluid step with the particle "
                          "half in its first blocks)", "kernel_ms": round(kern_ms, 5),
                "alg_bytes_per_launch": alg_bytes,
                "launch": {"threads": cfg[0], "blocks": cfg[1], "xcd_map": cfg[3]}}
    lat.close()
    del lat
    torch.cuda.empty_cache()
    from paper_0803_2826_amd.bw_ceilings import copy_ceiling, pull_ceiling
    ceiling, cblock = copy_ceiling(planes * 4 * N)
    roofline["copy_ceiling"] = {"achieved": round(ceiling, 1), "unit": "GB/s",
                                "kernel": f"streaming copy (16 B per thread, {cblock} threads per block) of one "
                                          f"{planes * 4 * N / 1e9:.2f} GB population buffer",
                                "frac_of_copy": round(achieved / ceiling, 4)}
    pull, pblock = pull_ceiling(L, planes)
    if pull:
        roofline["pull_pattern_ceiling"] = {"achieved": round(pull, 1), "unit": "GB/s",
                                            "kernel": f"the step's memory pattern without arithmetic: 19 planes "
                                                      f"pulled, the residual plane read, 20 stored "
                                                      f"({pblock} threads per block)",
                                            "frac_of_pattern": round(achieved / pull, 4)}

    forms = None if args.no_forms else run_forms(L)

    cpu = None
    if not args.no_cpu_baseline:
        print("# cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        cpu = cpu_baseline(L, n_chains, length, args.cpu_steps)

    line = {
        "metric": METRIC,
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"fluctuating D3Q19 MRT {L}^3 periodic, FP32 shifted storage, kT=1e-4, tau=1, "
                               f"{n_chains} chains x {length} beads {chain_desc}, "
                               f"trilinear interpolation + spreading every step",
                   "sites": N, "beads": nb, "parallelism": "single GPU"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "forms": forms,
        "separate_launches": {"ms_per_step": round(sep_ms, 5), "particle_half_ms": round(half_ms, 5),
                              "step_kernel_ms": round(sep_kern_ms, 5),
                              "note": "lb_couple (k_bead_half, k_bead_update) then lb_step (k_stream_collide with "
                                      "the bead force), 50 steps after the timed region"},
        "mass_drift_rel": (tot1x[0] - tot0[0]) / tot0[0],
        "mass_drift_steps": drift_steps,
        "fused_vs_exact_totals_abs": max(abs(a - b) for a, b in zip(tot1, tot1x)),
        "source_hash": source_hash(),
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
