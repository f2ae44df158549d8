"""Pins of the oracle's lattice Boltzmann part (Sec. 2.1, eqs. 1-8) against
closed forms, exact invariants and a textbook LBM written independently here.

Readings exercised: the forcing prefactor (1 - 1/(2 tau)) of eq. (8), and the
half-way bounce-back wall used only by the Poiseuille check."""
import math

import numpy as np
import pytest

import oracle
from paper_2303_11811_amd import inputs


def _total_momentum(box, f):
    c, _, _ = oracle.lattice()
    return (f.T @ c.astype(float)).sum(axis=0)


def test_uniform_flow_is_a_fixed_point():
    box = oracle.Box(6, 5, 4, tau=0.8)
    U0 = np.array([0.02, -0.01, 0.005])
    u = np.repeat(U0[:, None], box.N, axis=1)
    f0 = oracle.equilibrium(box, u)
    res = oracle.run(box, f0, 10)
    assert np.max(np.abs(res.f - f0)) < 2e-16


@pytest.mark.parametrize("tau", [0.51, 0.8, 1.7])
def test_mass_and_momentum_conserved(tau):
    spec = inputs.random_small((9, 7, 6), 0, (2, 3), seed=5, tau=tau)
    box = oracle.Box(*spec.dims, tau=tau)
    f0 = oracle.equilibrium(box, spec.u0, spec.rho0)
    f0 += np.random.default_rng(1).normal(0, 1e-4, f0.shape)  # non-equilibrium start
    res = oracle.run(box, f0, 50)
    assert abs(res.f.sum() - f0.sum()) / f0.sum() < 1e-13
    P0, P1 = _total_momentum(box, f0), _total_momentum(box, res.f)
    assert np.max(np.abs(P1 - P0)) < 1e-13 * box.N


@pytest.mark.parametrize("tau", [0.55, 0.8, 1.3])
def test_uniform_force_from_rest(tau):
    # The momentum input per step must equal the force density: j(t) = t f.
    g = np.array([1e-4, -3e-5, 2e-5])
    box = oracle.Box(4, 4, 4, tau=tau, fext=tuple(g))
    f = oracle.equilibrium(box, np.zeros((3, box.N)))
    for t in range(1, 6):
        f = oracle.run(box, f, 1).f
        rho, u = oracle.macroscopic(box, f)
        j = u - 0.5 * g[:, None]
        assert np.allclose(j, t * g[:, None], rtol=0, atol=1e-15 * t)
        assert np.allclose(rho, 1.0, atol=1e-15)


def _amplitude(box, f, comp, k_axis):
    _, u = oracle.macroscopic(box, f)
    dims = (box.nx, box.ny, box.nz)
    L = dims[k_axis]
    coord = np.arange(L) + 0.5
    ucomp = u[comp].reshape(box.nz, box.ny, box.nx)
    prof = ucomp.mean(axis=tuple(a for a in range(3) if a != 2 - k_axis))
    return 2.0 / L * np.sum(prof * np.sin(2 * math.pi * coord / L))


def _shear_rate_error(tau, L, axis_u, axis_k):
    dims = [1, 1, 1]
    dims[axis_k] = L
    box = oracle.Box(*dims, tau=tau)
    f = oracle.equilibrium(box, inputs.shear_wave(tuple(dims), 1e-4, axis_u=axis_u, axis_k=axis_k))
    nu = (tau - 0.5) / 3.0
    k = 2 * math.pi / L
    T = int(2.0 / (nu * k * k))
    f = oracle.run(box, f, T // 2).f
    a1 = _amplitude(box, f, axis_u, axis_k)
    f = oracle.run(box, f, T // 2).f
    a2 = _amplitude(box, f, axis_u, axis_k)
    rate = -math.log(a2 / a1) / (T // 2)
    return rate / (nu * k * k) - 1.0


@pytest.mark.parametrize("tau,axes", [(0.6, (0, 1)), (0.9, (2, 0)), (0.75, (1, 2))])
def test_shear_wave_decay_rate(tau, axes):
    """u_a = A sin(k x_b) decays as exp(-nu k^2 t), nu = (tau - 1/2)/3 (eq. 4),
    up to a lattice error O(k^2): within 1e-3 at L = 64, and the error falls
    by 4x when L doubles (second order)."""
    e32 = _shear_rate_error(tau, 32, *axes)
    e64 = _shear_rate_error(tau, 64, *axes)
    assert abs(e64) < 1e-3
    assert 3.8 < e32 / e64 < 4.2


def test_taylor_green_decay_rate():
    # 2-D Taylor-Green vortex: velocity amplitude decays as exp(-2 nu k^2 t)
    L, tau = 32, 0.6
    box = oracle.Box(L, L, 2, tau=tau)
    f = oracle.equilibrium(box, inputs.taylor_green((L, L, 2), 0.01))

    def amp(f):
        _, u = oracle.macroscopic(box, f)
        ref = inputs.taylor_green((L, L, 2), 1.0)
        return float((u[0] * ref[0]).sum() / (ref[0] * ref[0]).sum())

    T = 600
    f = oracle.run(box, f, T // 2).f
    a1 = amp(f)
    f = oracle.run(box, f, T // 2).f
    a2 = amp(f)
    nu = (tau - 0.5) / 3.0
    k = 2 * math.pi / L
    rate = -math.log(a2 / a1) / (T // 2)
    assert abs(rate / (2 * nu * k * k) - 1.0) < 1e-3


@pytest.mark.parametrize("tau", [0.55, 0.8, 1.0, 0.5 + math.sqrt(3.0) / 4.0])
def test_poiseuille_halfway_bounce_back(tau):
    """Body-force-driven channel between half-way bounce-back walls at z = -1/2
    and z = H - 1/2. The BGK steady state is the parabola with walls at the
    half-way points plus a uniform slip (2g/(3 nu))((tau - 1/2)^2 - 3/16),
    which vanishes at tau = 1/2 + sqrt(3)/4."""
    H, g = 12, 1e-5
    box = oracle.Box(2, 2, H, tau=tau, fext=(g, 0.0, 0.0), walls_z=True)
    f = oracle.equilibrium(box, np.zeros((3, box.N)))
    nu = (tau - 0.5) / 3.0
    nsteps = int(40 * H * H / (math.pi ** 2 * nu)) + 200
    f = oracle.run(box, f, nsteps).f
    _, u = oracle.macroscopic(box, f)
    z = np.arange(H) + 0.0
    exact = g / (2 * nu) * (z + 0.5) * (H - 0.5 - z) + 2 * g / (3 * nu) * ((tau - 0.5) ** 2 - 3.0 / 16.0)
    prof = u[0].reshape(H, 2, 2)[:, 0, 0]
    assert np.max(np.abs(prof - exact)) / exact.max() < 1e-9


def test_streaming_moves_mass_along_momentum():
    """sum_x x (rho(x,t+1) - 1) - sum_x x (rho(x,t) - 1) = sum_x j(x,t) exactly
    for a localized perturbation (eq. 2 pushes f_q along +c_q)."""
    L = 24
    box = oracle.Box(L, L, L, tau=0.7)
    c = (np.arange(L) + 0.5)
    Z, Y, X = np.meshgrid(c, c, c, indexing="ij")
    r2 = (X - 12) ** 2 + (Y - 12) ** 2 + (Z - 12) ** 2
    # compact support (radius 5): nothing reaches the periodic seam in 3 steps
    bump = (np.maximum(0.0, 1.0 - r2 / 25.0) ** 3).ravel()
    rho = 1 + 0.01 * bump
    u = np.stack([0.03 * bump, -0.02 * bump, 0.01 * bump])
    f = oracle.equilibrium(box, u, rho)
    pos = np.stack([X.ravel(), Y.ravel(), Z.ravel()])
    for _ in range(3):
        rho0, u0 = oracle.macroscopic(box, f)
        m0 = pos @ (rho0 - 1)
        P = u0.sum(axis=1)  # no force: U = j
        f = oracle.run(box, f, 1).f
        rho1, _ = oracle.macroscopic(box, f)
        m1 = pos @ (rho1 - 1)
        assert np.allclose(m1 - m0, P, rtol=1e-10, atol=1e-13)
        assert np.abs(P).max() > 1e-3


def _textbook_lbm_step(f, dims, tau, g):
    """Plain BGK D3Q19 with Guo forcing and incompressible equilibrium, streamed
    with np.roll. Written independently of the oracle (vectorised numpy)."""
    nx, ny, nz = dims
    cs = np.array([[0, 0, 0], [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1],
                   [1, 1, 0], [-1, -1, 0], [1, -1, 0], [-1, 1, 0], [1, 0, 1], [-1, 0, -1],
                   [1, 0, -1], [-1, 0, 1], [0, 1, 1], [0, -1, -1], [0, 1, -1], [0, -1, 1]])
    ws = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)
    F = f.reshape(19, nz, ny, nx)
    rho = F.sum(axis=0)
    jv = np.einsum("qa,qzyx->azyx", cs.astype(float), F)
    U = jv + 0.5 * np.asarray(g)[:, None, None, None]
    cu = np.einsum("qa,azyx->qzyx", cs.astype(float), U)
    uu = (U * U).sum(axis=0)
    feq = ws[:, None, None, None] * (rho[None] + 3 * cu + 4.5 * cu ** 2 - 1.5 * uu[None])
    cg = cs.astype(float) @ np.asarray(g)
    ug = np.einsum("a,azyx->zyx", np.asarray(g), U)
    Fq = (1 - 0.5 / tau) * ws[:, None, None, None] * (3 * (cg[:, None, None, None] - ug[None])
                                                        + 9 * cu * cg[:, None, None, None])
    post = F + (feq - F) / tau + Fq
    out = np.empty_like(post)
    for q in range(19):
        out[q] = np.roll(post[q], shift=(cs[q, 2], cs[q, 1], cs[q, 0]), axis=(0, 1, 2))
    return out.reshape(19, -1)


def test_no_particles_equals_textbook_lbm():
    dims, tau, g = (8, 6, 5), 0.63, (2e-5, -1e-5, 3e-6)
    spec = inputs.random_small(dims, 0, (2, 3), seed=9, tau=tau)
    box = oracle.Box(*dims, tau=tau, fext=g)
    f = oracle.equilibrium(box, spec.u0, spec.rho0)
    f += np.random.default_rng(2).normal(0, 1e-4, f.shape)
    ref = f.copy()
    for _ in range(5):
        ref = _textbook_lbm_step(ref, dims, tau, g)
    got = oracle.run(box, f, 5).f
    assert np.max(np.abs(got - ref)) < 1e-15


@pytest.mark.parametrize("tau", [0.6, 0.9, 1.4])
def test_couette_moving_walls_linear_profile(tau):
    """Walls at z = -1/2 and z = H - 1/2 moving with U_b and U_t along x and y:
    the steady BGK solution with half-way bounce-back and the moving-wall term
    is exactly linear, u(k) = U_b + (U_t - U_b)(k + 1/2)/H, at any tau."""
    H = 10
    Ub, Ut = np.array([-0.01, 0.004, 0.0]), np.array([0.03, -0.006, 0.0])
    box = oracle.Box(2, 2, H, tau=tau, walls_z=True, wall_u=(Ub, Ut))
    f = oracle.equilibrium(box, np.zeros((3, box.N)))
    nu = (tau - 0.5) / 3.0
    nsteps = int(50 * H * H / (math.pi ** 2 * nu)) + 200
    f = oracle.run(box, f, nsteps).f
    rho, u = oracle.macroscopic(box, f)
    k = np.arange(H) + 0.0
    for a in range(2):
        exact = Ub[a] + (Ut[a] - Ub[a]) * (k + 0.5) / H
        prof = u[a].reshape(H, 2, 2)[:, 0, 0]
        assert np.max(np.abs(prof - exact)) < 1e-10 * np.abs(Ut - Ub).max()
    assert np.max(np.abs(u[2])) < 1e-14
    # tangential walls neither add nor remove mass
    assert abs(rho.sum() - box.N) < 1e-11 * box.N


def test_uniform_through_flow_between_velocity_faces_is_a_fixed_point():
    """Faces at z = -1/2 and nz - 1/2 imposing the same velocity U, with a
    normal component (velocity inflow and outflow): the uniform flow E(1, U)
    is an exact fixed point of the step, since the bounced population
    E_qbar(U) + 6 w_q (c_q . U) equals E_q(U)."""
    H = 9
    U = np.array([0.012, -0.004, 0.02])
    box = oracle.Box(4, 4, H, tau=0.77, walls_z=True, wall_u=(U, U))
    u0 = np.repeat(U[:, None], box.N, axis=1)
    f0 = oracle.equilibrium(box, u0)
    f = oracle.run(box, f0, 150).f
    assert np.max(np.abs(f - f0)) < 1e-15


def test_velocity_inflow_pressure_outflow_plug_flow():
    """Velocity inflow U through z = -1/2, pressure outflow (rho = 1) through
    z = nz - 1/2: the uniform flow E(1, U) is an exact fixed point
    (anti-bounce-back of E_q with the cell's velocity U returns E_qbar), and
    a start from rest converges to it."""
    H = 10
    U = np.array([0.0, 0.0, 0.02])
    box = oracle.Box(4, 4, H, tau=0.8, walls_z=True, wall_u=(U, (0.0, 0.0, 0.0)),
                     face_type=(oracle.FACE_VELOCITY, oracle.FACE_PRESSURE), face_rho=(1.0, 1.0))
    plug = oracle.equilibrium(box, np.repeat(U[:, None], box.N, axis=1))
    f = oracle.run(box, plug, 100).f
    assert np.max(np.abs(f - plug)) < 1e-15
    f = oracle.run(box, oracle.equilibrium(box, np.zeros((3, box.N))), 6000).f
    assert np.max(np.abs(f - plug)) < 1e-12


def test_pressure_outflow_sets_the_outlet_density():
    """Through-flow with a tangential inflow component and an outlet density
    different from 1: mass flux in equals mass flux out at steady state, and
    the density next to the outlet approaches the prescribed one."""
    H = 12
    U = np.array([0.01, 0.0, 0.015])
    rho_out = 1.002
    box = oracle.Box(4, 4, H, tau=0.9, walls_z=True, wall_u=(U, (0.0, 0.0, 0.0)),
                     face_type=(oracle.FACE_VELOCITY, oracle.FACE_PRESSURE), face_rho=(1.0, rho_out))
    f = oracle.run(box, oracle.equilibrium(box, np.zeros((3, box.N))), 6000).f
    f2 = oracle.run(box, f, 1).f
    assert np.max(np.abs(f2 - f)) < 1e-11      # steady
    rho, u = oracle.macroscopic(box, f)
    rz = rho.reshape(H, 4, 4)[:, 0, 0]
    assert abs(rz[-1] - rho_out) < 2e-4
    # uniform mass flux rho u_z along the channel (steady continuity)
    jz = (rho * u[2]).reshape(H, 4, 4)[:, 0, 0]
    assert np.max(np.abs(jz - jz.mean())) < 1e-10


def test_duct_flow_side_walls():
    """Body-force flow along z through a duct with resting walls in x and y:
    the steady profile is symmetric in x and y, vanishes nowhere inside, and
    mass is conserved; with walls in x only the profile is the Poiseuille
    closed form in x (the half-way bounce-back solution, as pinned for z)."""
    tau, g = 0.8, 1e-5
    nu = (tau - 0.5) / 3.0
    H = 10
    box = oracle.Box(H, 4, 4, tau=tau, fext=(0.0, 0.0, g), walls_x=True)
    f = oracle.equilibrium(box, np.zeros((3, box.N)))
    steps = int(40 * H * H / (math.pi ** 2 * nu)) + 200
    f = oracle.run(box, f, steps).f
    rho, u = oracle.macroscopic(box, f)
    x = np.arange(H) + 0.0
    exact = g / (2 * nu) * (x + 0.5) * (H - 0.5 - x) + 2 * g / (3 * nu) * ((tau - 0.5) ** 2 - 3.0 / 16.0)
    prof = u[2].reshape(4, 4, H)[0, 0, :]
    assert np.max(np.abs(prof - exact)) / exact.max() < 1e-9
    assert abs(rho.sum() - box.N) < 1e-11 * box.N
    box2 = oracle.Box(8, 8, 4, tau=tau, fext=(0.0, 0.0, g), walls_x=True, walls_y=True)
    f2 = oracle.run(box2, oracle.equilibrium(box2, np.zeros((3, box2.N))), 3000).f
    _, u2 = oracle.macroscopic(box2, f2)
    w = u2[2].reshape(4, 8, 8)[0]
    assert np.allclose(w, w.T, rtol=0, atol=1e-15)
    assert np.allclose(w, w[::-1, :], rtol=0, atol=1e-15)
    assert np.all(w > 0)


def _face_group_sums(rho0, V, g, tau):
    """Sums over the five directions with c_z = +1 (s = +1) or -1 (s = -1) of
    the state E(rho0, V), of its post-collision values (SRT with the Guo
    forcing, g along z) and the post-collision velocity, derived by hand for
    a uniform state. Over such a group, sum_q w_q = 1/6, sum_q w_q (c_q.U) =
    s U_z/6 and sum_q w_q (c_q.U)^2 = (U_x^2 + U_y^2)/18 + U_z^2/6, so
      sum_q E_q(rho, U) = rho/6 + s U_z/2 + U_z^2/2    (tangential parts cancel)
      sum_q F_q         = (1 - 1/(2 tau)) g_z (s/2 + U_z),
    with U = V + g/2 inside the collision (eq. 7) and j = V before it."""
    pref = 1.0 - 1.0 / (2.0 * tau)
    Uz = V[2] + 0.5 * g
    out = {}
    for s in (1, -1):
        P = rho0 / 6.0 + s * V[2] / 2.0 + V[2] ** 2 / 2.0
        E = rho0 / 6.0 + s * Uz / 2.0 + Uz ** 2 / 2.0
        out[s] = P + (E - P) / tau + pref * g * (s / 2.0 + Uz)
    return out


@pytest.mark.parametrize("faces", ["velocity_in", "both_pressure"])
@pytest.mark.parametrize("g", [2e-3, -1.5e-3])
def test_pressure_face_first_step_mass_balance(faces, g):
    """Which velocity the anti-bounce-back uses (R16: the boundary cell's
    post-collision velocity j + g of the same step, not the pre-collision j
    nor U = j + g/2) decides the mass that crosses a pressure face. Per face
    cell and step the face rule returns f_qbar = -f~_q + 2 w_q (rho_w +
    4.5 (c_q.u)^2 - 1.5 u.u) for the five leaving directions q, so the mass
    leaving is 2 S - rho_w/3 - u_z^2 (S the sum of the leaving f~_q, and
    sum_q w_q (4.5 (c_q.u)^2 - 1.5 u.u) = u_z^2/2 over the group). A velocity
    face adds exactly u_wz per cell (sum of 6 w_q (c_q.u_w) over the group).
    With a body force along the flow, the first step from a uniform E(rho0, V)
    then changes the total mass by a closed form in which u_z = V_z + g; the
    other two readings differ from it by N_xy (2 V_z g + g^2) and
    N_xy (V_z g + g^2/4), far above round-off."""
    tau, rho0 = 0.8, 1.01
    V = np.array([0.01, -0.02, 0.04])
    nx, ny, nz = 4, 5, 6
    rho_top, rho_bot = 0.995, 1.004
    uw = np.array([0.003, 0.001, 0.035])
    if faces == "velocity_in":
        box = oracle.Box(nx, ny, nz, tau=tau, fext=(0.0, 0.0, g), walls_z=True, wall_u=(uw, (0.0, 0.0, 0.0)),
                         face_type=(oracle.FACE_VELOCITY, oracle.FACE_PRESSURE), face_rho=(1.0, rho_top))
    else:
        box = oracle.Box(nx, ny, nz, tau=tau, fext=(0.0, 0.0, g), walls_z=True,
                         face_type=(oracle.FACE_PRESSURE, oracle.FACE_PRESSURE), face_rho=(rho_bot, rho_top))
    f0 = oracle.equilibrium(box, np.repeat(V[:, None], box.N, axis=1), np.full(box.N, rho0))
    f1 = oracle.run(box, f0, 1).f
    dm = f1.sum() - f0.sum()

    S = _face_group_sums(rho0, V, g, tau)
    nxy = nx * ny

    def expected(uz):
        out_top = 2.0 * S[1] - rho_top / 3.0 - uz ** 2
        if faces == "velocity_in":
            into_bottom = uw[2]
        else:
            into_bottom = -(2.0 * S[-1] - rho_bot / 3.0 - uz ** 2)
        return nxy * (into_bottom - out_top)

    exact = expected(V[2] + g)
    assert abs(dm - exact) < 1e-13 * f0.sum()
    # the pre-collision readings would be told apart
    for uz in (V[2], V[2] + 0.5 * g):
        assert abs(expected(uz) - exact) > 1e6 * 1e-13 * f0.sum()
