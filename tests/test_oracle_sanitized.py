"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (host
code only): a copy of oracle/ is compiled with -fsanitize=address,undefined
and a small run of every oracle entry point family (fluid steps with noise
and walls, coupled steps with harmonic and Kremer-Grest beads and the wide
stencils, the fluid and coupled adjoints) executes in a child process with
the sanitizer runtime preloaded.  Any out-of-bounds access, use after free
or undefined behaviour aborts the child and fails the test."""
import os
import shutil
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = textwrap.dedent("""
    import sys
    import numpy as np
    sys.path.insert(0, sys.argv[1])
    import oracle as orc
    from paper_0803_2826_amd.inputs import kremer_grest_chains, random_walk_chains

    rng = np.random.default_rng(0)
    # fluid: noise, a body force, walls, general relaxation
    for walls in (0, 1):
        p = orc.Params(nx=6, ny=5, nz=7, kT=1e-4, seed=3, g=(1e-5, 0.0, -2e-5), gamma_shear=0.2, gamma_bulk=-0.1,
                       walls=walls)
        n = orc.init_equilibrium(p, u=rng.normal(scale=0.01, size=(3, 7, 5, 6)))
        orc.run(p, n, 3)
        orc.totals(p, n)
        orc.fields(p, n)
        lam, gbar = orc.backward(p, n, 2, rng.normal(size=n.shape))
    # coupled steps: harmonic chains with each stencil, Kremer-Grest chains with three-point noise
    L = 8
    p = orc.Params(nx=L, ny=L, nz=L, kT=1e-4, seed=5, g=(1e-5, 0.0, 0.0))
    for W in (2, 3, 4):
        pos, mom, bonds = random_walk_chains(2, 4, (L, L, L), seed=W)
        nb = pos.shape[0]
        b = orc.Beads(pos, mom, np.ones(nb), np.full(nb, 0.5), bonds, 1e-3, 1.0, stencil=W,
                      fext=rng.normal(scale=1e-5, size=(nb, 3)))
        n = orc.init_equilibrium(p)
        for t in range(2):
            orc.coupled_step(p, n, t, b)
        pos0 = b.pos.copy()
        b0 = b.copy()
        orc.backward_coupled(p, n, 2, b0, rng.normal(size=n.shape), rng.normal(size=(nb, 3)),
                             rng.normal(size=(nb, 3)))
    pos, _, bonds = kremer_grest_chains(2, 8, (L, L, L), seed=1)
    nb = pos.shape[0]
    kg = orc.Beads(pos, np.zeros((nb, 3)), np.ones(nb), np.full(nb, 0.5), bonds, 3e-3, 1.5, fene=True,
                   wca_eps=1e-4, wca_sigma=1.0, three_point=True)
    n = orc.init_equilibrium(p)
    for t in range(2):
        orc.coupled_step(p, n, t, kg)
    orc.backward_coupled(p, n, 2, kg.copy(), rng.normal(size=n.shape), rng.normal(size=(nb, 3)),
                         rng.normal(size=(nb, 3)))
    print("sanitized oracle run ok")
""")


def test_oracle_runs_clean_under_asan_and_ubsan(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    asan = subprocess.run([gcc, "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("the AddressSanitizer runtime is not installed")
    pkg = tmp_path / "oracle"
    shutil.copytree(os.path.join(ROOT, "oracle"), pkg, ignore=shutil.ignore_patterns("*.so", "__pycache__", "*.tmp*"))
    lib = pkg / "liblb_oracle.so"
    subprocess.run([gcc, "-O1", "-g", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
                    "-fPIC", "-shared", "-o", str(lib), str(pkg / "lb_oracle.c"), "-lm"], check=True)
    env = dict(os.environ)
    env["LD_PRELOAD"] = asan
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    env["OMP_NUM_THREADS"] = "2"
    env["PYTHONPATH"] = ROOT
    script = tmp_path / "run.py"
    script.write_text(SCRIPT)
    r = subprocess.run([sys.executable, str(script), str(tmp_path)], env=env, capture_output=True, text=True,
                       timeout=600)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "sanitized oracle run ok" in r.stdout
