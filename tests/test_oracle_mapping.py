"""Pins of the oracle's solid-fraction mapping (Sec. 2.3.2, eqs. 25-27, and the
two-slot storage of Sec. 3.1.1) against quadrature, exact integer counts,
geometry and the stated slot rules."""
import math

import numpy as np
import pytest
from scipy import integrate

import oracle


@pytest.mark.parametrize("r", [1.0, 2.0, 3.0, 4.0, 5.0, 8.0, 10.0])
def test_Va_closed_form_matches_quadrature(r):
    # eq. (27): V_a is the integral of sqrt(r^2 - x^2 - y^2) over the unit square
    val, err = integrate.dblquad(lambda y, x: math.sqrt(r * r - x * x - y * y), -0.5, 0.5, -0.5, 0.5,
                                 epsabs=2e-13, epsrel=2e-13)
    assert abs(oracle.Va(r) - val) <= 1e-12 * max(1.0, val)


def _exact_axis_overlap(r, m):
    """Volume of {x^2+y^2+z^2 <= r^2} inside the cell [m-1/2, m+1/2] x [-1/2,1/2]^2."""
    def h(z, y):
        s = r * r - y * y - z * z
        top = math.sqrt(s) if s > 0 else 0.0
        return min(max(top - (m - 0.5), 0.0), 1.0)
    val, _ = integrate.dblquad(h, -0.5, 0.5, -0.5, 0.5, epsabs=1e-13, epsrel=1e-13)
    return val


@pytest.mark.parametrize("r", [3.3, 4.3, 6.2, 7.8, 10.2])
def test_linear_approximation_exact_on_axis_cells(r):
    # The approximation is derived from the case where the sphere surface crosses
    # an on-axis cell over its whole face (Fig. 2); there it equals the true volume.
    L = 40
    box = oracle.Box(L, L, L, tau=0.7)
    xc = np.array([[20.5, 20.5, 20.5]])  # sphere centred on the centre of cell (20,20,20)
    B, pid, ov = oracle.solid_map(box, xc, [r])
    Bf = B[0].reshape(L, L, L)  # [z][y][x]
    checked = 0
    for m in range(1, 12):
        # surface inside [m-1/2, m+1/2] over the whole face
        if math.sqrt(r * r - 0.5) >= m - 0.5 and r <= m + 0.5:
            exact = _exact_axis_overlap(r, m)
            for (dz, dy, dx) in [(0, 0, m), (0, 0, -m), (0, m, 0), (m, 0, 0), (-m, 0, 0)]:
                assert abs(Bf[20 + dz, 20 + dy, 20 + dx] - exact) < 1e-10
            checked += 1
    assert checked >= 1


@pytest.mark.parametrize("r,seed", [(3.0, 0), (4.0, 1), (8.0, 2), (10.0, 3)])
def test_linear_volume_close_to_sphere(r, seed):
    rng = np.random.default_rng(seed)
    L = int(2 * r + 12)
    box = oracle.Box(L, L, L, tau=0.7)
    for _ in range(3):
        x = rng.random((1, 3)) * L
        B, pid, ov = oracle.solid_map(box, x, [r])
        vol = 4.0 / 3.0 * math.pi * r ** 3
        # position-dependent discretisation error: a few 1e-3 for small spheres
        assert abs(B.sum() - vol) / vol < (5e-3 if r < 6 else 1e-3)
        assert ov == 0


def _integer_subsample(L, x8, r8, n=4):
    """Exact sub-sample counts with all coordinates scaled by 2n (integers).
    x8: centre * 2n (int), r8: r * 2n (int). Sample point of cell i, offset k:
    i + (k + 1/2)/n  -> scaled: 2n i + 2k + 1."""
    cnt = np.zeros((L, L, L), dtype=np.int64)
    s = 2 * n
    ks = 2 * np.arange(n) + 1
    for z in range(L):
        for y in range(L):
            for x in range(L):
                ds = []
                for ax, i in enumerate((x, y, z)):
                    d = s * i + ks - x8[ax]
                    # minimum image in scaled units: wrap the cell-centre offset
                    dc = s * i + n - x8[ax]
                    if dc >= s * L // 2:
                        d = d - s * L
                    elif dc < -(s * L // 2):
                        d = d + s * L
                    ds.append(d)
                d2 = (ds[0][:, None, None] ** 2 + ds[1][None, :, None] ** 2 + ds[2][None, None, :] ** 2)
                cnt[z, y, x] = int((d2 <= r8 * r8).sum())
    return cnt


@pytest.mark.parametrize("xc", [(6.0, 6.0, 6.0), (5.5, 6.25, 7.125), (0.375, 11.5, 6.625)])
def test_subsample_counts_exact(xc):
    # centres on multiples of 1/8 make every sample coordinate dyadic: exact
    L, r, n = 12, 4.0, 4
    box = oracle.Box(L, L, L, tau=0.7, mapping=oracle.MAP_SUBSAMPLE, nsub=n)
    B, pid, ov = oracle.solid_map(box, np.array([xc]), [r])
    x8 = [int(round(v * 2 * n)) for v in xc]
    cnt = _integer_subsample(L, x8, int(r * 2 * n), n)
    assert np.array_equal(B[0].reshape(L, L, L) * n ** 3, cnt.astype(float))
    assert np.all(pid[0][B[0] > 0] == 0)


@pytest.mark.parametrize("r", [4.0, 8.0])
def test_linear_vs_fine_subsampling(r):
    L = int(2 * r + 8)
    rng = np.random.default_rng(7)
    x = rng.random((1, 3)) * L
    bl = oracle.Box(L, L, L, tau=0.7)
    bs = oracle.Box(L, L, L, tau=0.7, mapping=oracle.MAP_SUBSAMPLE, nsub=16)
    Bl, _, _ = oracle.solid_map(bl, x, [r])
    Bs, _, _ = oracle.solid_map(bs, x, [r])
    assert np.max(np.abs(Bl[0] - Bs[0])) <= 0.05


def test_cube_symmetry_of_centred_sphere():
    L, r = 16, 4.6
    box = oracle.Box(L, L, L, tau=0.7)
    B, _, _ = oracle.solid_map(box, np.array([[8.5, 8.5, 8.5]]), [r])
    f = B[0].reshape(L, L, L)
    core = f[1:, 1:, 1:]  # centred on cell 8 -> symmetric about index 8 in [1, 15]
    for perm in [(0, 2, 1), (1, 0, 2), (2, 1, 0), (1, 2, 0)]:
        assert np.array_equal(core, core.transpose(perm))
    for ax in range(3):
        assert np.array_equal(core, np.flip(core, axis=ax))


def test_translation_invariance_of_map():
    L = 20
    box = oracle.Box(L, L, L, tau=0.7)
    rng = np.random.default_rng(3)
    x = rng.random((3, 3)) * L
    r = np.array([3.5, 4.0, 2.5])
    B0, p0, _ = oracle.solid_map(box, x, r)
    s = np.array([5, -3, 7])
    B1, p1, _ = oracle.solid_map(box, (x + s) % L, r)
    roll = lambda a: np.roll(a.reshape(2, L, L, L), shift=(s[2], s[1], s[0]), axis=(1, 2, 3)).reshape(2, -1)
    assert np.allclose(roll(B0), B1, atol=1e-13, rtol=0)
    assert np.array_equal(roll(p0), p1)


def test_slot_rules_against_single_particle_maps():
    """Three mutually overlapping spheres: each cell keeps the two largest
    fractions (ties -> smaller id), stores them in ascending id, renormalises
    when their sum exceeds 1, and counts every dropped overlap."""
    L = 16
    box = oracle.Box(L, L, L, tau=0.7)
    x = np.array([[7.3, 8.1, 8.0], [9.2, 7.6, 8.4], [8.1, 9.5, 7.2]])
    r = np.array([3.1, 2.9, 3.4])
    singles = np.stack([oracle.solid_map(box, x[p:p + 1], r[p:p + 1])[0][0] for p in range(3)])
    B, pid, ov = oracle.solid_map(box, x, r)
    dropped = 0
    for n in range(box.N):
        cand = [(singles[p, n], p) for p in range(3) if singles[p, n] > 0]
        cand.sort(key=lambda t: (-t[0], t[1]))
        dropped += max(0, len(cand) - 2)
        keep = sorted(cand[:2], key=lambda t: t[1])
        tot = sum(b for b, _ in keep)
        if tot > 1.0 and len(keep) == 2:
            keep = [(b / tot, p) for b, p in keep]
        exp_p = [p for _, p in keep] + [-1] * (2 - len(keep))
        exp_b = [b for b, _ in keep] + [0.0] * (2 - len(keep))
        assert [pid[0, n], pid[1, n]] == exp_p
        assert B[0, n] == exp_b[0] and B[1, n] == exp_b[1]
    assert ov == dropped and dropped > 0
    assert (B[0] + B[1]).max() <= 1.0 + 1e-15


def test_map_cell_bruteforce_equals_bounding_box_map():
    L = 18
    for mapping in (oracle.MAP_LINEAR, oracle.MAP_SUBSAMPLE):
        box = oracle.Box(L, L, L, tau=0.7, mapping=mapping, nsub=4)
        rng = np.random.default_rng(11)
        x = rng.random((4, 3)) * L
        r = rng.uniform(2.0, 4.0, 4)
        B, pid, _ = oracle.solid_map(box, x, r)
        for n in rng.integers(0, box.N, 300):
            i, j, k = n % L, (n // L) % L, n // (L * L)
            ns, p2, b2, _ = oracle.map_cell(box, i, j, k, x, r)
            assert list(p2) == [pid[0, n], pid[1, n]]
            assert list(b2) == [B[0, n], B[1, n]]
