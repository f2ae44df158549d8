"""Pins of the oracle's D3Q19 velocity set (Sec. 2.1): the isotropy moments
that make the equilibrium of eq. (5) reproduce mass, momentum and the
Navier-Stokes momentum flux with c_s^2 = 1/3."""
import itertools

import numpy as np

import oracle


def test_velocity_set_is_d3q19():
    c, w, qb = oracle.lattice()
    vecs = {tuple(v) for v in c}
    expect = {(0, 0, 0)}
    expect |= {tuple(s * e) for e in np.eye(3, dtype=int) for s in (1, -1)}
    expect |= {v for v in itertools.product((-1, 0, 1), repeat=3) if sum(map(abs, v)) == 2}
    assert vecs == expect and len(c) == 19
    # canonical order: rest, then +-x, +-y, +-z, then the 12 face diagonals in pairs
    assert tuple(c[0]) == (0, 0, 0)
    assert [tuple(v) for v in c[1:7]] == [(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)]


def test_inverse_directions():
    c, w, qb = oracle.lattice()
    for q in range(19):
        assert np.array_equal(c[qb[q]], -c[q])
        assert w[qb[q]] == w[q]
    # pairs are adjacent: q odd -> q+1
    for q in range(1, 19, 2):
        assert qb[q] == q + 1


def test_weight_moments():
    c, w, _ = oracle.lattice()
    c = c.astype(float)
    assert abs(w.sum() - 1.0) < 1e-15
    assert np.allclose(w @ c, 0.0, atol=1e-16)
    m2 = np.einsum("q,qa,qb->ab", w, c, c)
    assert np.allclose(m2, np.eye(3) / 3.0, atol=1e-15)
    m3 = np.einsum("q,qa,qb,qc->abc", w, c, c, c)
    assert np.allclose(m3, 0.0, atol=1e-16)
    m4 = np.einsum("q,qa,qb,qc,qd->abcd", w, c, c, c, c)
    d = np.eye(3)
    iso = (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d)
           + np.einsum("ad,bc->abcd", d, d)) / 9.0
    assert np.allclose(m4, iso, atol=1e-15)
