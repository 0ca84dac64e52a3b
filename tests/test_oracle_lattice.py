"""Pins of the oracle's lattice tables, equilibrium and moment transforms.

Every expected value here is fixed by the paper (Table 1, the weights and
c_s^2 quoted after eq. original_equil_distrib, the moment conditions
eq. MBeq0-MBeq2 and eq. w0-w4, the weighted orthogonality eq. orthogonality)
or by exact linear algebra, never by the oracle itself.
"""
import os
from fractions import Fraction

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table1_d3q19.txt")


def load_table1():
    rows = []
    with open(GOLDEN) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            k, poly, w = [s.strip() for s in line.split("|")]
            rows.append((int(k), poly, Fraction(w)))
    return rows


def test_velocity_set(orc):
    c, a, e, w = orc.tables()
    # 1 rest, 6 speed-1, 12 speed-sqrt2 velocities, all distinct, closed under negation
    sp = (c ** 2).sum(1)
    assert sorted(sp.tolist()) == [0] + [1] * 6 + [2] * 12
    assert len({tuple(v) for v in c}) == 19
    for v in c:
        assert any((u == -v).all() for u in c)


def test_weights_and_isotropy(orc):
    """eq. w0-w4 with C2 = c_s^2 = 1/3, C4' = 0 and C4 = C2^2."""
    c, a, e, w = orc.tables()
    assert a[0] == pytest.approx(1 / 3, abs=1e-16)
    for i in range(19):
        s2 = int((c[i] ** 2).sum())
        assert a[i] == pytest.approx({0: 1 / 3, 1: 1 / 18, 2: 1 / 36}[s2], abs=1e-16)
    assert a.sum() == pytest.approx(1.0, abs=1e-15)
    cf = c.astype(float)
    np.testing.assert_allclose(np.einsum("i,ia->a", a, cf), 0, atol=1e-16)
    np.testing.assert_allclose(np.einsum("i,ia,ib->ab", a, cf, cf), np.eye(3) / 3, atol=1e-16)
    np.testing.assert_allclose(np.einsum("i,ia,ib,ic->abc", a, cf, cf, cf), 0, atol=1e-16)
    m4 = np.einsum("i,ia,ib,ic,id->abcd", a, cf, cf, cf, cf)
    d = np.eye(3)
    iso = (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d) + np.einsum("ad,bc->abcd", d, d))
    np.testing.assert_allclose(m4, iso / 9, atol=1e-16)


def test_basis_matches_table1(orc):
    """The oracle's e_ki equal the Table 1 polynomials (read from the golden
    fixture) and its w_k equal the printed normalisations."""
    c, a, e, w = orc.tables()
    rows = load_table1()
    assert [r[0] for r in rows] == list(range(19))
    for k, poly, wk in rows:
        for i in range(19):
            cx, cy, cz = (int(v) for v in c[i])
            c2 = cx * cx + cy * cy + cz * cz
            val = eval(poly, {"cx": cx, "cy": cy, "cz": cz, "c2": c2})
            assert e[k, i] == val, (k, i)
        assert w[k] == pytest.approx(float(wk), rel=1e-15)


def test_weighted_orthogonality(orc):
    """eq. orthogonality with q = a: sum_i a_i e_ki e_li = w_k delta_kl."""
    c, a, e, w = orc.tables()
    G = (e * a) @ e.T
    np.testing.assert_allclose(G, np.diag(w), atol=1e-15)
    assert np.linalg.matrix_rank(e) == 19


def test_forward_back_inverse(orc):
    """eq. back_transformation inverts eq. forward for any populations."""
    rng = np.random.default_rng(1)
    for _ in range(20):
        n = rng.normal(size=19)
        m = orc.moments_site(n)
        np.testing.assert_allclose(orc.back_site(m), n, atol=1e-14)
        mm = rng.normal(size=19)
        np.testing.assert_allclose(orc.moments_site(orc.back_site(mm)), mm, atol=1e-14)


def test_equilibrium_moments(orc):
    """eq. MBeq0-MBeq2: sum n^eq = rho, sum n^eq c = rho u,
    sum n^eq c c = rho c_s^2 delta + rho u u (Sec. D3Q19 model I)."""
    c, a, e, w = orc.tables()
    cf = c.astype(float)
    rng = np.random.default_rng(2)
    for _ in range(20):
        rho = 0.5 + rng.random()
        u = rng.normal(scale=0.05, size=3)
        neq = orc.equilibrium(rho, u)
        assert neq.sum() == pytest.approx(rho, rel=1e-14)
        np.testing.assert_allclose(neq @ cf, rho * u, atol=1e-15)
        pi = np.einsum("i,ia,ib->ab", neq, cf, cf)
        np.testing.assert_allclose(pi, rho / 3 * np.eye(3) + rho * np.outer(u, u), atol=1e-15)


def test_equilibrium_has_no_kinetic_projection(orc):
    """With q = a the kinetic moments m_10..m_18 of n^eq vanish (text after
    eq. back_transformation), and the stress moments follow eq. hmodes."""
    rng = np.random.default_rng(3)
    for _ in range(20):
        rho = 0.5 + rng.random()
        u = rng.normal(scale=0.05, size=3)
        m = orc.moments_site(orc.equilibrium(rho, u))
        np.testing.assert_allclose(m[10:], 0, atol=1e-15)
        j = rho * u
        pi = rho / 3 * np.eye(3) + rho * np.outer(u, u)
        # eq. hmodes_beg - hmodes_end
        assert m[0] == pytest.approx(rho, rel=1e-14)
        np.testing.assert_allclose(m[1:4], j, atol=1e-15)
        assert pi[0, 0] == pytest.approx((m[0] + m[4] + m[5]) / 3, abs=1e-14)
        assert pi[1, 1] == pytest.approx((2 * m[0] + 2 * m[4] - m[5] + 3 * m[6]) / 6, abs=1e-14)
        assert pi[2, 2] == pytest.approx((2 * m[0] + 2 * m[4] - m[5] - 3 * m[6]) / 6, abs=1e-14)
        assert pi[0, 1] == pytest.approx(m[7], abs=1e-15)
        assert pi[1, 2] == pytest.approx(m[8], abs=1e-15)
        assert pi[2, 0] == pytest.approx(m[9], abs=1e-15)
