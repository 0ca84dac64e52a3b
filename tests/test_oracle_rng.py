"""Pins of the oracle's random numbers.

- Philox4x32-10 (Salmon et al., SC'11) against rocRAND's independent engine,
  compiled for the host from its public header (no GPU needed).
- The Gaussian variates the collision uses (eq. stochupdaterule1 asks for
  independent zero-mean unit-variance Gaussians) pass distribution tests:
  moments, Kolmogorov-Smirnov against the normal CDF, and independence across
  modes, sites and steps.
"""
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rocrand_ref():
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available to build the rocRAND host reference")
    d = tempfile.mkdtemp()
    exe = os.path.join(d, "philox_ref")
    subprocess.run([hipcc, "-O1", "-o", exe, os.path.join(HERE, "rocrand_philox_ref.cpp")], check=True,
                   cwd=d, capture_output=True)
    yield exe
    shutil.rmtree(d, ignore_errors=True)


def test_philox_matches_rocrand(orc, rocrand_ref):
    rng = np.random.default_rng(0)
    cases = [[0, 0, 0, 0, 0, 0], [0xFFFFFFFF] * 6, [1, 2, 3, 4, 5, 6]]
    cases += rng.integers(0, 2 ** 32, size=(200, 6), dtype=np.uint64).tolist()
    text = "\n".join(" ".join(str(int(v)) for v in row) for row in cases) + "\n"
    out = subprocess.run([rocrand_ref], input=text, capture_output=True, text=True, check=True).stdout.split("\n")
    for row, line in zip(cases, out):
        ref = [int(v) for v in line.split()]
        got = orc.philox4x32_10(row[:4], row[4:]).tolist()
        assert got == ref, row


def test_fluid_normals_distribution(orc):
    from scipy import stats
    samples = np.array([orc.fluid_normals(42, s, t) for s in range(2000) for t in range(5)])
    assert samples.shape == (10000, 16)
    x = samples.reshape(-1)
    assert abs(x.mean()) < 4 / np.sqrt(x.size)
    assert x.var() == pytest.approx(1.0, abs=5 * np.sqrt(2 / x.size))
    assert stats.kurtosis(x, fisher=False) == pytest.approx(3.0, abs=0.1)
    assert stats.kstest(x, "norm").pvalue > 1e-3
    # each of the 16 slots separately is standard normal
    for k in range(16):
        assert stats.kstest(samples[:, k], "norm").pvalue > 1e-4
    # no correlation between slots (incl. the two outputs of one Box-Muller pair)
    C = np.corrcoef(samples.T)
    off = C - np.eye(16)
    assert np.abs(off).max() < 5 / np.sqrt(samples.shape[0])


def test_fluid_normals_depend_on_every_counter_word(orc):
    base = orc.fluid_normals(1, 10, 20, 0)
    for args in [(2, 10, 20, 0), (1, 11, 20, 0), (1, 10, 21, 0), (1, 10, 20, 1), (1 << 40, 10, 20, 0)]:
        other = orc.fluid_normals(*args)
        assert np.abs(other - base).min() > 0


def test_bead_normals_distribution(orc):
    from scipy import stats
    s = np.array([orc.bead_normals(9, b, t) for b in range(3000) for t in range(3)]).reshape(-1)
    assert stats.kstest(s, "norm").pvalue > 1e-3
    assert s.var() == pytest.approx(1.0, abs=0.05)
    # bead stream differs from the fluid stream at the same counter
    assert not np.allclose(orc.bead_normals(9, 5, 5)[:2], orc.fluid_normals(9, 5, 5)[:2])


def test_bead_three_point_follows_exact_thresholds(orc):
    """The three-point variate (Sec. "Force coupling", after eq.
    langevin_momentum_update) reads the first three words w of the bead
    stream's Philox call and maps w / 2^32 < 1/6 to -sqrt(3), >= 5/6 to
    +sqrt(3), anything else to 0; checked here with exact rational
    thresholds on the pinned Philox words, including words at the edges."""
    import math
    from fractions import Fraction
    seed = (7 << 32) | 3
    for bead, step, box in [(b, t, x) for b in range(60) for t in range(4) for x in (0, 5)]:
        w = orc.philox4x32_10([bead, step, 1 << 16, box], [seed & 0xFFFFFFFF, seed >> 32])
        got = orc.bead_three_point(seed, bead, step, box)
        for a in range(3):
            u = Fraction(int(w[a]), 2 ** 32)
            want = -math.sqrt(3.0) if u < Fraction(1, 6) else math.sqrt(3.0) if u >= Fraction(5, 6) else 0.0
            assert got[a] == want, (bead, step, box, a, int(w[a]))


def test_bead_three_point_moments(orc):
    """Probabilities 1/6, 2/3, 1/6 and the Gaussian moments the paper asks
    the distribution to reproduce: mean 0, variance 1, fourth moment 3."""
    s = np.array([orc.bead_three_point(11, b, t) for b in range(4000) for t in range(4)]).reshape(-1)
    r3 = np.sqrt(3.0)
    assert set(np.unique(s)) <= {-r3, 0.0, r3}
    n = s.size
    for value, prob in ((-r3, 1 / 6), (0.0, 2 / 3), (r3, 1 / 6)):
        frac = np.mean(s == value)
        assert abs(frac - prob) < 5 * np.sqrt(prob * (1 - prob) / n), value
    assert abs(s.mean()) < 5 / np.sqrt(n)
    assert (s ** 2).mean() == pytest.approx(1.0, abs=5 * np.sqrt(2 / n))
    assert (s ** 4).mean() == pytest.approx(3.0, abs=5 * np.sqrt(24 / n))
