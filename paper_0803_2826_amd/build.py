"""Build liblbmi.so (the LB library) and libbwprobe.so (the copy-bandwidth
reference of the benchmark), HIP for gfx950, in-tree with hipcc."""
from __future__ import annotations

import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblbmi.so")
PROBE = os.path.join(HERE, "libbwprobe.so")
ARCH = os.environ.get("LBMI_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared",
    f"--offload-arch={ARCH}",
    # no packed FP32 instructions: the kernels are written and checked for
    # scalar FP32 code generation
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-munsafe-fp-atomics",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
]
# the library's ROCTX ranges around the API calls
LDFLAGS = ["-L/opt/rocm/lib", "-Wl,-rpath,/opt/rocm/lib", "-lrocprofiler-sdk-roctx"]


def hipcc() -> str:
    return shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


def sources():
    return [os.path.join(CSRC, "lbmi.hip")]


def build(verbose: bool = False, extra: list[str] | None = None, out: str | None = None) -> str:
    """Compile every HIP source into liblbmi.so (always recompiles)."""
    target = out or LIB
    tmp = target + ".tmp%d" % os.getpid()
    cmd = [hipcc()] + FLAGS + (extra or []) + ["-o", tmp] + sources() + LDFLAGS
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True, cwd=CSRC)
    os.replace(tmp, target)
    return target


def build_probe(verbose: bool = False) -> str:
    """Compile the copy-bandwidth reference into libbwprobe.so (always recompiles)."""
    tmp = PROBE + ".tmp%d" % os.getpid()
    cmd = [hipcc()] + FLAGS + ["-o", tmp, os.path.join(CSRC, "bw_probe.hip")]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True, cwd=CSRC)
    os.replace(tmp, PROBE)
    return PROBE


if __name__ == "__main__":
    print(build(verbose=True))
    print(build_probe(verbose=True))
