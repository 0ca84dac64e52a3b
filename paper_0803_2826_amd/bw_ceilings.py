"""Bandwidth ceilings of the device for the LB step's memory pattern.

Times the kernels of libbwprobe.so (csrc/bw_probe.hip) with HIP events on the
current stream: plain copies in several shapes (vectors per thread,
non-temporal loads and stores, one chunk per block or a persistent grid),
read-only, write-only and in-place streams, the step's own pull pattern in
its z-major layout (19 planes, and 20 with the rest residual plane of FP32
storage) and the in-place AA pattern (one buffer; even and odd steps).
Bytes are counted as the kernel's algorithmic traffic: each byte read plus
each byte written once.

    python -m paper_0803_2826_amd.bw_ceilings [--L 256 512] [--json out.json]
    python -m paper_0803_2826_amd.bw_ceilings --best --L 256 [--reps 50]

prints one line per configuration and the best of each family (or, with
--best, runs only the best configuration of each family, for rocprofv3).  bench.py
uses copy_ceiling() and pull_ceiling() for the references in its line.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys

import torch

from paper_0803_2826_amd import build as hip_build

_P = None


def probe() -> ctypes.CDLL:
    global _P
    if _P is not None:
        return _P
    if not os.path.exists(hip_build.PROBE):
        raise RuntimeError(f"{hip_build.PROBE} is not built (run python -m paper_0803_2826_amd.build)")
    P = ctypes.CDLL(hip_build.PROBE)
    vp, i32, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint64
    P.bw_copy.argtypes = [vp, vp, u64, i32, vp]
    P.bw_copy_v.argtypes = [vp, vp, u64, i32, i32, i32, i32, i32, vp]
    P.bw_read.argtypes = [vp, u64, i32, vp, vp]
    P.bw_write.argtypes = [vp, u64, i32, vp]
    P.bw_inplace.argtypes = [vp, u64, i32, vp]
    P.bw_pull19.argtypes = [vp, vp, i32, i32, vp]
    P.bw_pull20.argtypes = [vp, vp, i32, i32, vp]
    P.bw_aa.argtypes = [vp, i32, i32, i32, vp]
    _P = P
    return P


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def time_ms(launch, reps: int = 20) -> float:
    """Mean duration of one launch (after one warm-up launch)."""
    if launch() != 0:
        raise RuntimeError("probe launch failed")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        launch()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def copy_ceiling(nbytes: int) -> tuple:
    """(GB/s, threads per block) of the plain streaming copy (bw_copy) of
    nbytes over 256 / 512 / 1024 threads per block."""
    P = probe()
    a = torch.zeros(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    s = _stream()
    best = (0.0, 0)
    for block in (256, 512, 1024):
        ms = time_ms(lambda: P.bw_copy(a.data_ptr(), b.data_ptr(), nbytes, block, s))
        best = max(best, (2 * nbytes / (ms * 1e-3) / 1e9, block))
    del a, b
    torch.cuda.empty_cache()
    return best


def pull_ceiling(L: int, planes: int = 20) -> tuple:
    """(GB/s, threads per block) of the step's pull pattern alone (P planes,
    z-major) over an L^3 box, or (None, None) if L is not a power of two."""
    lg = L.bit_length() - 1
    if (1 << lg) != L or not 4 <= lg <= 10:
        return None, None
    P = probe()
    fn = P.bw_pull20 if planes == 20 else P.bw_pull19
    N = L ** 3
    a = torch.zeros(planes * N, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    s = _stream()
    best = (0.0, 0)
    for block in (256, 512, 1024):
        ms = time_ms(lambda: fn(a.data_ptr(), b.data_ptr(), lg, block, s))
        best = max(best, (2 * planes * 4 * N / (ms * 1e-3) / 1e9, block))
    del a, b
    torch.cuda.empty_cache()
    return best


def sweep(L: int) -> list:
    """Every configuration at the state size of an L^3 FP32 box (20 planes)."""
    P = probe()
    s = _stream()
    lg = L.bit_length() - 1
    N = L ** 3
    nbytes = 20 * 4 * N
    rows = []

    def rec(family, cfg, ms, nb):
        rows.append({"L": L, "family": family, "config": cfg, "ms": round(ms, 5),
                     "gbs": round(nb / (ms * 1e-3) / 1e9, 1)})
        print(f"{L:4d}  {family:10s} {cfg:46s} {ms:9.4f} ms  {rows[-1]['gbs']:8.1f} GB/s", flush=True)

    a = torch.zeros(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.zeros_like(a)
    sink = torch.zeros(1, dtype=torch.float32, device="cuda")
    for block in (256, 512, 1024):
        rec("copy", f"16 B/thread, nt stores, block {block}",
            time_ms(lambda: P.bw_copy(a.data_ptr(), b.data_ptr(), nbytes, block, s)), 2 * nbytes)
    for vec in (1, 2, 4, 8):
        for ntl in (0, 1):
            for nts in (0, 1):
                for block in (256, 1024):
                    for grid in (0, 1024, 4096):
                        ms = time_ms(lambda: P.bw_copy_v(a.data_ptr(), b.data_ptr(), nbytes, block, vec, ntl, nts,
                                                         grid, s))
                        rec("copy_v", f"vec {vec} ntl {ntl} nts {nts} block {block} grid {grid or 'all'}", ms,
                            2 * nbytes)
    for block in (256, 512, 1024):
        rec("read", f"16 B/thread, block {block}",
            time_ms(lambda: P.bw_read(a.data_ptr(), nbytes, block, sink.data_ptr(), s)), nbytes)
        rec("write", f"16 B/thread, nt stores, block {block}",
            time_ms(lambda: P.bw_write(b.data_ptr(), nbytes, block, s)), nbytes)
        rec("inplace", f"16 B/thread, nt stores, block {block}",
            time_ms(lambda: P.bw_inplace(a.data_ptr(), nbytes, block, s)), 2 * nbytes)
    for block in (64, 128, 256, 512, 1024):
        rec("pull19", f"19 planes z-major, block {block}",
            time_ms(lambda: P.bw_pull19(a.data_ptr(), b.data_ptr(), lg, block, s)), 2 * 19 * 4 * N)
        rec("pull20", f"20 planes z-major, block {block}",
            time_ms(lambda: P.bw_pull20(a.data_ptr(), b.data_ptr(), lg, block, s)), 2 * 20 * 4 * N)

        def aa_pair():
            rc = P.bw_aa(a.data_ptr(), lg, 0, block, s)
            return rc or P.bw_aa(a.data_ptr(), lg, 1, block, s)
        rec("aa_pair", f"20 planes in place, even + odd, block {block}", time_ms(aa_pair) / 2, 2 * 20 * 4 * N)
        rec("aa_even", f"20 planes in place, block {block}",
            time_ms(lambda: P.bw_aa(a.data_ptr(), lg, 0, block, s)), 2 * 20 * 4 * N)
        rec("aa_odd", f"20 planes in place, block {block}",
            time_ms(lambda: P.bw_aa(a.data_ptr(), lg, 1, block, s)), 2 * 20 * 4 * N)
    del a, b
    torch.cuda.empty_cache()
    return rows


def best_only(L: int, reps: int) -> None:
    """The best configuration of each family from the sweep, `reps` launches
    each (for a profiler's per-kernel averages; kernel names differ per
    family: k_copy16, k_copy_v<1>, k_read16, k_write16, k_inplace16,
    k_pull<19>, k_pull<20>, k_aa<0>, k_aa<1>)."""
    P = probe()
    s = _stream()
    lg = L.bit_length() - 1
    N = L ** 3
    nbytes = 20 * 4 * N
    a = torch.zeros(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.zeros_like(a)
    sink = torch.zeros(1, dtype=torch.float32, device="cuda")
    runs = [
        ("copy", 2 * nbytes, lambda: P.bw_copy(a.data_ptr(), b.data_ptr(), nbytes, 256, s)),
        ("copy_v", 2 * nbytes, lambda: P.bw_copy_v(a.data_ptr(), b.data_ptr(), nbytes, 256, 1, 1, 0, 0, s)),
        ("read", nbytes, lambda: P.bw_read(a.data_ptr(), nbytes, 512, sink.data_ptr(), s)),
        ("write", nbytes, lambda: P.bw_write(b.data_ptr(), nbytes, 256, s)),
        ("inplace", 2 * nbytes, lambda: P.bw_inplace(a.data_ptr(), nbytes, 256, s)),
        ("pull19", 2 * 19 * 4 * N, lambda: P.bw_pull19(a.data_ptr(), b.data_ptr(), lg, 256, s)),
        ("pull20", 2 * 20 * 4 * N, lambda: P.bw_pull20(a.data_ptr(), b.data_ptr(), lg, 256, s)),
        ("aa_even", 2 * 20 * 4 * N, lambda: P.bw_aa(a.data_ptr(), lg, 0, 256, s)),
        ("aa_odd", 2 * 20 * 4 * N, lambda: P.bw_aa(a.data_ptr(), lg, 1, 256, s)),
    ]
    for name, nb, fn in runs:
        ms = time_ms(fn, reps)
        print(f"{L:4d}  {name:8s} {ms:9.4f} ms  {nb / (ms * 1e-3) / 1e9:8.1f} GB/s  ({nb} B per launch)", flush=True)
    del a, b
    torch.cuda.empty_cache()


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--L", type=int, nargs="+", default=[256, 512])
    ap.add_argument("--json", default=None)
    ap.add_argument("--best", action="store_true", help="only the best configuration of each family")
    ap.add_argument("--reps", type=int, default=50)
    args = ap.parse_args()
    torch.cuda.set_device(0)
    if args.best:
        for L in args.L:
            best_only(L, args.reps)
        return 0
    rows = []
    for L in args.L:
        rows += sweep(L)
    print("\nbest per family:")
    for L in args.L:
        for fam in sorted({r["family"] for r in rows if r["L"] == L}):
            best = max((r for r in rows if r["L"] == L and r["family"] == fam), key=lambda r: r["gbs"])
            print(f"{L:4d}  {fam:10s} {best['config']:46s} {best['gbs']:8.1f} GB/s ({best['gbs'] / 80:.1f} % of 8 TB/s)")
    if args.json:
        with open(args.json, "w") as f:
            json.dump(rows, f, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
