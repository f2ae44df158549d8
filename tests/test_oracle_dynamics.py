"""Pins of the oracle's particle integrator (Sec. 2.2.2, eqs. 15-16, and the
explicit Euler update) against closed forms: the mass and moment of inertia
of a voxelised sphere, uniformly accelerated motion, the exact discrete
solution of velocity Verlet for a harmonic force, and periodic wrapping."""
import numpy as np
import pytest

import oracle


def _box(n=64):
    return oracle.Box(n, n, n, tau=0.6)


def _voxel_sphere(r, h=0.02):
    """Volume and z-axis second moment of a ball of radius r by midpoint
    quadrature on an h-grid (independent of any formula for m or I)."""
    g = np.arange(-r + h / 2, r, h)
    X, Y = np.meshgrid(g, g, indexing="ij")
    rho2 = X * X + Y * Y
    inside = rho2 <= r * r
    # exact integration along z through each column: chord length 2 sqrt(r^2 - rho^2)
    chord = np.where(inside, 2.0 * np.sqrt(np.maximum(r * r - rho2, 0.0)), 0.0)
    vol = chord.sum() * h * h
    # second moment about the z axis: int (x^2 + y^2) dV
    jz = (chord * rho2).sum() * h * h
    return vol, jz


@pytest.mark.parametrize("r,rho_p", [(4.0, 2.5), (8.0, 1.1), (10.0, 1.0)])
def test_mass_and_inertia_match_voxelised_sphere(r, rho_p):
    box = _box()
    dyn = oracle.Dynamics([[32.0, 32.0, 32.0]], [r], [[0, 0, 0]], [[0, 0, 0]])
    F = np.array([[1.0, -2.0, 0.5]])
    T = np.array([[0.0, 0.0, 3.0]])
    oracle.integrate(box, dyn, F, T, dt=1.0, scheme=oracle.EULER, rho_p=rho_p)
    m_eff = F[0, 0] / dyn.U[0, 0]
    I_eff = T[0, 2] / dyn.Om[0, 2]
    vol, jz = _voxel_sphere(r)
    assert abs(m_eff - rho_p * vol) <= 1e-4 * rho_p * vol
    assert abs(I_eff - rho_p * jz) <= 1e-4 * rho_p * jz
    # all three components see the same mass
    assert np.allclose(dyn.U[0] * m_eff, F[0], rtol=1e-14, atol=0)


def test_euler_uniform_acceleration_closed_form():
    box = _box()
    r, rho_p = 5.0, 2.0
    x0, U0 = np.array([[20.0, 30.0, 25.0]]), np.array([[0.01, -0.02, 0.005]])
    F = np.array([[3.0, 1.0, -2.0]])
    accel = np.array([0.0, 0.0, -1e-4])
    dyn = oracle.Dynamics(x0, [r], U0, [[0, 0, 0]])
    k, dt = 7, 0.5
    for _ in range(k):
        oracle.integrate(box, dyn, F, np.zeros((1, 3)), dt=dt, scheme=oracle.EULER, rho_p=rho_p, accel=accel)
    m = rho_p * 4.0 / 3.0 * np.pi * r ** 3
    a = F[0] / m + accel
    assert np.allclose(dyn.U[0], U0[0] + k * dt * a, rtol=1e-13, atol=1e-17)
    assert np.allclose(dyn.x[0], x0[0] + k * dt * U0[0] + dt * dt * a * k * (k - 1) / 2, rtol=1e-13, atol=1e-13)


def test_verlet_uniform_acceleration_is_exact():
    """Velocity Verlet integrates constant acceleration exactly:
    x_k = x_0 + k dt U_0 + (k dt)^2 a / 2; after k calls the velocity has
    been completed k - 1 times: U = U_0 + (k - 1) dt a. Same for rotation."""
    box = _box()
    r, rho_p = 6.0, 1.5
    x0, U0, Om0 = np.array([[10.0, 40.0, 33.0]]), np.array([[0.02, 0.0, -0.01]]), np.array([[0.0, 1e-3, 0.0]])
    F, T = np.array([[-2.0, 4.0, 1.0]]), np.array([[5.0, 0.0, -7.0]])
    dyn = oracle.Dynamics(x0, [r], U0, Om0)
    k, dt = 9, 0.25
    for _ in range(k):
        oracle.integrate(box, dyn, F, T, dt=dt, scheme=oracle.VERLET, rho_p=rho_p)
    m = rho_p * 4.0 / 3.0 * np.pi * r ** 3
    inertia = 0.4 * m * r * r
    a, alpha = F[0] / m, T[0] / inertia
    assert np.allclose(dyn.x[0], x0[0] + k * dt * U0[0] + (k * dt) ** 2 * a / 2, rtol=1e-13, atol=1e-13)
    assert np.allclose(dyn.U[0], U0[0] + (k - 1) * dt * a, rtol=1e-13, atol=1e-17)
    assert np.allclose(dyn.Om[0], Om0[0] + (k - 1) * dt * alpha, rtol=1e-13, atol=1e-17)


def test_verlet_harmonic_force_exact_discrete_solution():
    """For F = -K (x - c) velocity Verlet obeys x_{n+1} - 2 x_n + x_{n-1} =
    -(omega dt)^2 x_n, so from rest x_n - c = X cos(n theta) with
    cos(theta) = 1 - (omega dt)^2 / 2 exactly (the symplectic frequency shift)."""
    box = _box(64)
    r, rho_p = 3.0, 1.0
    m = rho_p * 4.0 / 3.0 * np.pi * r ** 3
    c = np.array([32.0, 32.0, 32.0])
    X = np.array([4.0, -3.0, 2.0])
    omega, dt = 0.3, 0.7
    K = m * omega * omega
    dyn = oracle.Dynamics([c + X], [r], [[0, 0, 0]], [[0, 0, 0]])
    theta = np.arccos(1.0 - (omega * dt) ** 2 / 2)
    for n in range(1, 60):
        F = -K * (dyn.x - c)
        oracle.integrate(box, dyn, F, np.zeros((1, 3)), dt=dt, scheme=oracle.VERLET, rho_p=rho_p)
        assert np.allclose(dyn.x[0] - c, X * np.cos(n * theta), rtol=0, atol=1e-11), n


def test_positions_wrap_into_the_box():
    box = oracle.Box(40, 30, 20, tau=0.6)
    dyn = oracle.Dynamics([[39.9, 0.1, 19.95], [0.0, 29.99, 10.0]], [2.0, 2.0],
                          [[0.3, -0.4, 0.1], [-0.5, 0.02, 0.0]], np.zeros((2, 3)))
    oracle.integrate(box, dyn, np.zeros((2, 3)), np.zeros((2, 3)), scheme=oracle.EULER)
    assert np.allclose(dyn.x, [[0.2, 29.7, 0.05], [39.5, 0.01, 10.0]], rtol=0, atol=1e-12)
    assert np.all(dyn.x >= 0) and np.all(dyn.x < np.array([40, 30, 20]))


def test_elastic_contact_with_walls():
    """Along an axis with walls a sphere keeps one cell of gap: a centre that
    passes r + 1 (or L - r - 1) is mirrored back and the normal velocity
    reverses; the other axes stay periodic."""
    box = oracle.Box(40, 30, 50, tau=0.6, walls_z=True, walls_x=True)
    r = 4.0
    dyn = oracle.Dynamics([[5.2, 29.5, 5.3], [34.7, 3.0, 44.6]], [r, r],
                          [[-0.5, 0.8, -0.6], [0.4, -0.1, 0.7]], np.zeros((2, 3)))
    oracle.integrate(box, dyn, np.zeros((2, 3)), np.zeros((2, 3)), scheme=oracle.EULER)
    # sphere 0: x 5.2 - 0.5 = 4.7 < 5 -> 5.3, y wraps (periodic), z 5.3 - 0.6 = 4.7 -> 5.3
    assert np.allclose(dyn.x[0], [5.3, 0.3, 5.3], rtol=0, atol=1e-12)
    assert np.allclose(dyn.U[0], [0.5, 0.8, 0.6])
    # sphere 1: x 35.1 > 35 -> 34.9, z 45.3 > 45 -> 44.7
    assert np.allclose(dyn.x[1], [34.9, 2.9, 44.7], rtol=0, atol=1e-12)
    assert np.allclose(dyn.U[1], [-0.4, -0.1, -0.7])
