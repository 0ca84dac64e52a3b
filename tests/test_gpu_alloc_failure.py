"""A device allocation the library is refused leaves the context usable.

The HIP runtime keeps a refused hipMalloc as its last error, also across
later successful calls, and the library's launch checks read that error
after every launch: a refusal that was reported as LB_ENOMEM must not
resurface as a failed launch of a later call.  Two refusals, forced from the
host:
- lb_tape_begin's first checkpoint while PyTorch holds the free device
  memory (PyTorch clears its own refusals); no tape is left then;
- lb_backward's segment buffer on a checkpointed tape whose segment
  (checkpoint_every step buffers of 1.34 GB at 256^3) exceeds the device
  memory.
"""
import math

import pytest

from conftest import gpu_available

pytestmark = pytest.mark.gpu


def fill_device(torch):
    """Hold the free device memory in 1 GiB tensors (then 64 MiB ones)."""
    held = []
    for chunk in (1 << 30, 1 << 26):
        while True:
            try:
                held.append(torch.empty(chunk, dtype=torch.uint8, device="cuda"))
            except torch.cuda.OutOfMemoryError:
                break
    return held


def test_refused_allocation_leaves_the_context_usable():
    if not gpu_available():
        pytest.skip("no GPU")
    import torch
    from paper_0803_2826_amd import lattice
    from paper_0803_2826_amd._lib import LB_ENOMEM, LB_ESTATE, LBError
    L, K = 256, 250
    dev = lattice.Lattice(lattice.FluidParams(nx=L, ny=L, nz=L, kT=1e-4, seed=5, track_totals=True))
    w = torch.zeros(19 * L ** 3, dtype=torch.float32, device="cuda")
    try:
        total = torch.cuda.get_device_properties(0).total_memory
        assert K * 20 * 4 * L ** 3 > total, "the segment buffer must exceed the device memory"
        dev.init_equilibrium()
        # 1. the first checkpoint of a tape (no tape before it, so that none
        # of its memory is freed first)
        held = fill_device(torch)
        try:
            with pytest.raises(LBError) as ei:
                dev.tape_begin(4)
            assert ei.value.code == LB_ENOMEM, ei.value
        finally:
            del held
            torch.cuda.empty_cache()
        dev.step(1)
        assert all(math.isfinite(v) for v in dev.totals())
        with pytest.raises(LBError) as ei:
            dev.backward(w)
        assert ei.value.code == LB_ESTATE  # no tape was left
        # 2. the segment buffer of the reverse sweep
        dev.tape_begin(K)
        dev.step(K)
        with pytest.raises(LBError) as ei:
            dev.backward(w)
        assert ei.value.code == LB_ENOMEM, ei.value
        dev.step(1)
        assert all(math.isfinite(v) for v in dev.totals())
        # a tape that fits works
        dev.tape_begin(4)
        dev.step(8)
        dn0, dg = dev.backward(w)
        assert torch.isfinite(dn0).all() and float(dn0.abs().max()) == 0.0
        assert tuple(dg) == (0.0, 0.0, 0.0)
    finally:
        dev.close()
