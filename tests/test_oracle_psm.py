"""Pins of the oracle's PSM coupling (Sec. 2.3, eqs. 17-22) against closed
forms of the first step, exact balance laws and symmetries."""
import numpy as np
import pytest

import oracle
from paper_2303_11811_amd import inputs


def _cells(box):
    n = np.arange(box.N)
    i, j, k = n % box.nx, (n // box.nx) % box.ny, n // (box.nx * box.ny)
    return np.stack([i + 0.5, j + 0.5, k + 0.5], axis=1)


def _min_image(d, dims):
    L = np.asarray(dims, dtype=float)
    d = d.copy()
    d = np.where(d >= 0.5 * L, d - L, d)
    d = np.where(d < -0.5 * L, d + L, d)
    return d


def _first_step_setup(g=(0.0, 0.0, 0.0)):
    dims = (20, 18, 16)
    rng = np.random.default_rng(21)
    x, r = inputs.rsa_spheres(dims, np.array([3.2, 2.7, 3.9]), rng)
    U = inputs.uniform_velocities(rng, 3, 0.01)
    Om = inputs.uniform_velocities(rng, 3, 0.002)
    box = oracle.Box(*dims, tau=0.7, fext=g)
    U0 = np.array([0.011, -0.004, 0.007])
    f0 = oracle.equilibrium(box, np.repeat(U0[:, None], box.N, axis=1))
    return box, x, r, U, Om, U0, f0


@pytest.mark.parametrize("g", [(0.0, 0.0, 0.0), (3e-4, -2e-4, 1e-4)])
def test_first_step_force_and_torque_closed_form(g):
    """From f = E(1, U0): sum_q C^solid c_qbar = j - f/2 - U_p(x) per slot
    (first moments of eq. 19 with j = U0), so eqs. (21)-(22) give
    F = sum_x B (U0 - f/2 - U_p(x)),  T = sum_x B d x (U0 - f/2 - U_p(x))."""
    box, x, r, U, Om, U0, f0 = _first_step_setup(g)
    res = oracle.run(box, f0, 1, x, r, U, Om)
    cells = _cells(box)
    g = np.asarray(g)
    for p in range(len(r)):
        F = np.zeros(3)
        T = np.zeros(3)
        for s in range(2):
            m = res.pid[s] == p
            d = _min_image(cells[m] - x[p], (box.nx, box.ny, box.nz))
            Vp = U[p] + np.cross(Om[p], d)
            gvec = U0 - 0.5 * g - Vp
            F += (res.B[s][m][:, None] * gvec).sum(axis=0)
            T += (res.B[s][m][:, None] * np.cross(d, gvec)).sum(axis=0)
        assert np.allclose(res.F[p], F, rtol=1e-12, atol=1e-15)
        assert np.allclose(res.T[p], T, rtol=1e-12, atol=1e-14)


def test_comoving_particle_feels_no_force():
    box, x, r, U, Om, U0, f0 = _first_step_setup()
    Uc = np.repeat(U0[None, :], len(r), axis=0)
    res = oracle.run(box, f0, 1, x, r, Uc, np.zeros_like(Uc))
    # zero up to the round-off of the moments (force scale here is O(1))
    assert np.max(np.abs(res.F)) < 1e-14 and np.max(np.abs(res.T)) < 1e-13
    # and the fluid state is untouched
    assert np.max(np.abs(res.f - f0)) < 1e-16


def test_rotating_particle_in_resting_fluid():
    """Fluid at rest, particle spinning with Omega: U_p(x) = Omega x d, so
    T = -sum_x B d x (Omega x d) = -sum_x B (Omega |d|^2 - d (d . Omega)),
    a torque opposing the rotation."""
    dims = (24, 24, 24)
    box = oracle.Box(*dims, tau=0.8)
    f0 = oracle.equilibrium(box, np.zeros((3, box.N)))
    x = np.array([[12.3, 11.8, 12.1]])
    r = np.array([5.0])
    Om = np.array([[0.001, -0.0005, 0.002]])
    res = oracle.run(box, f0, 1, x, r, np.zeros((1, 3)), Om)
    m = res.pid[0] == 0
    d = _min_image(_cells(box)[m] - x[0], dims)
    B = res.B[0][m]
    Texp = -(B[:, None] * (Om[0][None, :] * (d * d).sum(1)[:, None] - d * (d @ Om[0])[:, None])).sum(0)
    assert np.allclose(res.T[0], Texp, rtol=1e-12, atol=0)
    assert np.dot(res.T[0], Om[0]) < 0


def test_particle_at_rest_in_resting_fluid():
    box = oracle.Box(16, 16, 16, tau=0.9)
    f0 = oracle.equilibrium(box, np.zeros((3, box.N)))
    res = oracle.run(box, f0, 3, np.array([[8.2, 7.9, 8.4]]), np.array([4.0]))
    assert np.max(np.abs(res.F)) < 1e-14 and np.max(np.abs(res.T)) < 1e-13
    assert np.max(np.abs(res.f - f0)) < 1e-16


@pytest.mark.parametrize("overlap", [False, True])
def test_momentum_balance_every_step(overlap):
    """sum_x j~ - sum_x j = f_ext sum_x (1 - B) - sum_p F_p exactly (eqs. 17-21):
    what the fluid loses to the particles is what eq. (21) hands them."""
    dims, g = (16, 14, 12), np.array([2e-4, -1e-4, 5e-5])
    spec = inputs.random_small(dims, 4, (2.0, 3.5), seed=31, tau=0.66, fext=tuple(g), vamp=0.02,
                               omamp=0.004, overlap=overlap)
    box = oracle.Box(*dims, tau=spec.tau, fext=tuple(g))
    f = oracle.equilibrium(box, spec.u0, spec.rho0)
    c, _, _ = oracle.lattice()
    for _ in range(3):
        P0 = (f.T @ c.astype(float)).sum(0)
        M0 = f.sum()
        res = oracle.run(box, f, 1, spec.x, spec.r, spec.U, spec.Om)
        P1 = (res.f.T @ c.astype(float)).sum(0)
        Btot = res.B[0] + res.B[1]
        expect = g * (1 - Btot).sum() - res.F.sum(0)
        scale = np.abs(res.F).sum() + np.abs(g).max() * box.N
        assert np.allclose(P1 - P0, expect, rtol=0, atol=1e-13 * scale)
        assert abs(res.f.sum() - M0) < 1e-13 * M0
        if overlap:
            assert res.overflow >= 0 and Btot.max() <= 1.0 + 1e-15
        f = res.f


def test_translation_invariance():
    dims = (16, 12, 14)
    spec = inputs.random_small(dims, 3, (2.0, 3.0), seed=41, tau=0.75, fext=(1e-4, 0, 0), omamp=0.003)
    box = oracle.Box(*dims, tau=spec.tau, fext=spec.fext)
    f0 = oracle.equilibrium(box, spec.u0, spec.rho0)
    a = oracle.run(box, f0, 3, spec.x, spec.r, spec.U, spec.Om)
    s = np.array([3, -5, 2])
    roll = lambda arr: np.roll(arr.reshape(-1, dims[2], dims[1], dims[0]), shift=(s[2], s[1], s[0]),
                               axis=(1, 2, 3)).reshape(arr.shape)
    # shifts chosen as multiples of 1/4 keep the particle coordinates exact
    xs = np.round(spec.x * 4) / 4
    a = oracle.run(box, f0, 3, xs, spec.r, spec.U, spec.Om)
    b = oracle.run(box, roll(f0), 3, (xs + s) % np.array(dims), spec.r, spec.U, spec.Om)
    assert np.max(np.abs(roll(a.f) - b.f)) < 1e-15
    assert np.allclose(a.F, b.F, rtol=1e-12, atol=1e-16)
    assert np.allclose(a.T, b.T, rtol=1e-12, atol=1e-15)


def test_mirror_symmetry():
    """Reflect the configuration in x: velocities and forces flip their x
    component, the angular velocity and torque (pseudo-vectors) flip y and z."""
    dims = (14, 12, 10)
    spec = inputs.random_small(dims, 3, (2.0, 3.0), seed=51, tau=0.7, fext=(1e-4, 2e-5, -3e-5),
                               omamp=0.003)
    c, _, _ = oracle.lattice()
    mirror_q = [int(np.where((c == c[q] * np.array([-1, 1, 1])).all(1))[0][0]) for q in range(19)]
    box = oracle.Box(*dims, tau=spec.tau, fext=spec.fext)
    boxm = oracle.Box(*dims, tau=spec.tau, fext=(-spec.fext[0], spec.fext[1], spec.fext[2]))
    f0 = oracle.equilibrium(box, spec.u0, spec.rho0)
    x = np.round(spec.x * 4) / 4
    a = oracle.run(box, f0, 2, x, spec.r, spec.U, spec.Om)

    def mirror_field(f):
        F = f.reshape(19, dims[2], dims[1], dims[0])[:, :, :, ::-1]
        return F[mirror_q].reshape(19, -1)

    M = np.array([-1.0, 1.0, 1.0])
    xm = x.copy()
    xm[:, 0] = dims[0] - x[:, 0]
    b = oracle.run(boxm, mirror_field(f0), 2, xm, spec.r, spec.U * M, -spec.Om * M)
    assert np.max(np.abs(mirror_field(a.f) - b.f)) < 1e-15
    assert np.allclose(a.F * M, b.F, rtol=1e-12, atol=1e-16)
    assert np.allclose(-a.T * M, b.T, rtol=1e-12, atol=1e-15)


def test_b_zero_cells_evolve_as_plain_lbm():
    """Cells whose whole pull neighbourhood has B = 0 update exactly like the
    particle-free step."""
    dims = (20, 16, 16)
    spec = inputs.random_small(dims, 2, (2.5, 3.0), seed=61, tau=0.7, fext=(1e-4, 0, 0))
    box = oracle.Box(*dims, tau=spec.tau, fext=spec.fext)
    f0 = oracle.equilibrium(box, spec.u0, spec.rho0)
    with_p = oracle.run(box, f0, 1, spec.x, spec.r, spec.U, spec.Om)
    without = oracle.run(box, f0, 1)
    solid = (with_p.B[0] + with_p.B[1]).reshape(dims[2], dims[1], dims[0]) > 0
    near = solid.copy()
    for ax in range(3):
        near |= np.roll(solid, 1, axis=ax) | np.roll(solid, -1, axis=ax)
    near2 = near.copy()
    for ax in range(3):
        near2 |= np.roll(near, 1, axis=ax) | np.roll(near, -1, axis=ax)
    far = ~near2.ravel()
    assert far.sum() > box.N // 4
    assert np.array_equal(with_p.f[:, far], without.f[:, far])
