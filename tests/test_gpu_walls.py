"""No-slip walls at z = 0 and z = nz (half-way bounce-back with the
moving-wall term) on the GPU, through the C ABI: parity with the oracle's
walls (FP64 1e-12, deviation forms within the precision bounds), state I/O
round trips, FP64 stats, and the closed-form Couette and Poiseuille profiles."""
import math

import numpy as np
import pytest

import oracle
import paper_2303_11811_amd as psm
from paper_2303_11811_amd import inputs
from psm_cases import assert_forces_close, assert_pdfs_close, initial_f, make_engine, run_engine, run_oracle

pytestmark = pytest.mark.gpu


def _channel(dims, n, seed, tau=0.7, fext=(2e-5, -1e-5, 0.0), wall_u=((0.01, 0.0, 0.0), (-0.005, 0.008, 0.0))):
    """Spheres kept r + 1 away from the walls, a random start flow."""
    rng = np.random.default_rng(seed)
    r = rng.uniform(2.5, 4.0, n)
    L = np.asarray(dims, dtype=float)
    x = rng.random((n, 3)) * L
    x[:, 2] = r + 1.0 + rng.random(n) * (L[2] - 2.0 * (r + 1.0))
    base = inputs.random_small(dims, 0, (2, 3), seed=seed, tau=tau)
    return inputs.BoxSpec(dims=dims, tau=tau, fext=fext, x=x, r=r, U=inputs.uniform_velocities(rng, n, 0.01),
                          Om=inputs.uniform_velocities(rng, n, 0.002), u0=base.u0, walls_z=True, wall_u=wall_u)


@pytest.mark.parametrize("dims,launch", [((40, 30, 22), (64, 4, 4, 0)), ((36, 28, 26), (32, 8, 8, 3)),
                                         ((33, 20, 18), (16, 16, 1, 2))])
def test_walls_parity_fp64(dims, launch):
    spec = _channel(dims, 5, seed=sum(dims))
    print(f"[case] walls fp64 dims={dims} launch={launch}", flush=True)
    steps = 15
    ref = run_oracle(spec, steps)
    f, F, T, B, pid, eng = run_engine(spec, steps, launch=launch)
    assert_pdfs_close(f, ref.f, 1e-12)
    assert np.array_equal(pid, ref.pid)
    assert_forces_close(F, ref.F, ref.A)
    assert_forces_close(T, ref.T, ref.A, lever=spec.r.max() + 1)
    # FP64 stats from the canonical state
    mass, mom, _ = eng.get_stats(0)
    c, _, _ = oracle.lattice()
    assert abs(mass - ref.f.sum()) <= 1e-12 * ref.f.sum()
    mref = np.array([(ref.f * c[:, a:a + 1]).sum() for a in range(3)])
    assert np.all(np.abs(mom - mref) <= 1e-12 * ref.f.sum())
    eng.close()


@pytest.mark.parametrize("storage,tol_u", [(psm.PSM_FP32DEV, 2e-5), (psm.PSM_FP16DEV, 3e-3)])
def test_walls_deviation_forms(storage, tol_u):
    spec = _channel((32, 24, 20), 3, seed=4)
    steps = 40
    ref = run_oracle(spec, steps)
    f, F, T, B, pid, eng = run_engine(spec, steps, storage=storage)
    eng.close()
    box = oracle.Box(*spec.dims, tau=spec.tau)
    _, u_ref = oracle.macroscopic(box, ref.f)
    _, u = oracle.macroscopic(box, f)
    err = np.linalg.norm(u - u_ref) / np.linalg.norm(u_ref)
    assert err < tol_u, err


@pytest.mark.parametrize("storage", [psm.PSM_FP64, psm.PSM_FP32DEV])
def test_walls_state_roundtrip(storage):
    """set_pdfs then get_pdfs returns f (to the rounding of (f - t) + t for a
    wall term t in FP64, to the FP32 rounding of the deviation otherwise): the
    wall slots invert the bounce-back read."""
    spec = _channel((20, 12, 10), 0, seed=2)
    f0 = initial_f(spec) + 1e-3 * np.random.default_rng(0).standard_normal((19, spec.N))
    eng = make_engine([spec], storage=storage)
    eng.set_pdfs(0, f0)
    f1 = eng.get_pdfs(0).cpu().numpy()
    sel = np.random.default_rng(1).integers(0, spec.N, 50)
    fa = eng.get_pdfs_at(0, sel).cpu().numpy()
    eng.close()
    tol = 1e-16 if storage == psm.PSM_FP64 else 1e-7   # (f - wall term) + wall term
    assert np.max(np.abs(f1 - f0)) <= tol
    assert np.max(np.abs(fa - f0[:, sel])) <= tol


def test_couette_profile_on_gpu():
    """Exact linear profile between moving walls (as pinned for the oracle)."""
    H, tau = 12, 0.9
    Ub, Ut = (-0.01, 0.004, 0.0), (0.03, -0.006, 0.0)
    spec = inputs.BoxSpec(dims=(4, 4, H), tau=tau, walls_z=True, wall_u=(Ub, Ut))
    nu = (tau - 0.5) / 3.0
    steps = int(50 * H * H / (math.pi ** 2 * nu)) + 200
    f, *_ , eng = run_engine(spec, steps, launch=(16, 16, 4, 0))
    rho, u = eng.get_macroscopic(0)
    u = u.cpu().numpy()
    eng.close()
    k = np.arange(H) + 0.5
    for a in range(2):
        exact = Ub[a] + (Ut[a] - Ub[a]) * k / H
        prof = u[a].reshape(H, 4, 4)[:, 0, 0]
        assert np.max(np.abs(prof - exact)) < 1e-10 * 0.04
    assert abs(rho.sum().item() - spec.N) < 1e-11 * spec.N


def test_poiseuille_profile_on_gpu():
    """Body-force channel between resting walls: the BGK half-way bounce-back
    steady state (parabola plus the tau-dependent uniform slip)."""
    H, tau, g = 12, 0.8, 1e-5
    spec = inputs.BoxSpec(dims=(4, 4, H), tau=tau, fext=(g, 0.0, 0.0), walls_z=True)
    nu = (tau - 0.5) / 3.0
    steps = int(40 * H * H / (math.pi ** 2 * nu)) + 200
    f, *_, eng = run_engine(spec, steps, launch=(16, 16, 4, 0))
    _, u = eng.get_macroscopic(0)
    u = u.cpu().numpy()
    eng.close()
    z = np.arange(H) + 0.0
    exact = g / (2 * nu) * (z + 0.5) * (H - 0.5 - z) + 2 * g / (3 * nu) * ((tau - 0.5) ** 2 - 3.0 / 16.0)
    prof = u[0].reshape(H, 4, 4)[:, 0, 0]
    assert np.max(np.abs(prof - exact)) / exact.max() < 1e-9


def test_wall_particle_placement_is_checked():
    spec = _channel((30, 30, 20), 1, seed=9)
    eng = make_engine([spec])
    x = spec.x.copy()
    x[0, 2] = spec.r[0] + 0.5
    with pytest.raises(psm.PsmError) as ei:
        eng.set_particles(0, x, spec.r, spec.U)
    eng.close()
    assert ei.value.code == psm.PSM_EINVAL


def test_through_flow_faces_parity_and_fixed_point():
    """Velocity faces with a normal component (inflow at z = 0, outflow at
    z = nz at the same velocity): parity with the oracle with spheres in the
    stream, and the uniform flow as an exact fixed point without them."""
    Uf = (0.004, 0.0, 0.015)
    spec = _channel((30, 26, 24), 3, seed=31, fext=(0.0, 0.0, 0.0), wall_u=(Uf, Uf))
    ref = run_oracle(spec, 12)
    f, F, T, B, pid, eng = run_engine(spec, 12, launch=(32, 8, 4, 0))
    eng.close()
    assert_pdfs_close(f, ref.f, 1e-12)
    assert_forces_close(F, ref.F, ref.A)
    plug = inputs.BoxSpec(dims=(16, 12, 10), tau=0.8, walls_z=True, wall_u=(Uf, Uf),
                          u0=np.repeat(np.array(Uf)[:, None], 16 * 12 * 10, axis=1))
    f0 = initial_f(plug)
    f1, *_, eng = run_engine(plug, 100)
    eng.close()
    assert np.max(np.abs(f1 - f0)) < 1e-15


def _outflow(dims, n, seed, storage_rho=1.0, U=(0.003, 0.0, 0.012)):
    """Velocity inflow through z = 0, pressure outflow through z = nz."""
    spec = _channel(dims, n, seed, fext=(0.0, 0.0, 0.0), wall_u=(U, (0.0, 0.0, 0.0)))
    spec.face_type = (psm.PSM_FACE_VELOCITY, psm.PSM_FACE_PRESSURE)
    spec.face_rho = (1.0, storage_rho)
    return spec


@pytest.mark.parametrize("dims,launch,rho_out", [((36, 30, 24), (64, 4, 4, 0), 1.0),
                                                 ((33, 26, 21), (32, 8, 8, 3), 1.003)])
def test_pressure_outflow_parity_fp64(dims, launch, rho_out):
    spec = _outflow(dims, 4, seed=sum(dims), storage_rho=rho_out)
    print(f"[case] outflow fp64 dims={dims} launch={launch}", flush=True)
    ref = run_oracle(spec, 15)
    f, F, T, B, pid, eng = run_engine(spec, 15, launch=launch)
    mass, mom, _ = eng.get_stats(0)
    eng.close()
    assert_pdfs_close(f, ref.f, 1e-12)
    assert_forces_close(F, ref.F, ref.A)
    assert_forces_close(T, ref.T, ref.A, lever=spec.r.max() + 1)
    c, _, _ = oracle.lattice()
    assert abs(mass - ref.f.sum()) <= 1e-12 * ref.f.sum()
    mref = np.array([(ref.f * c[:, a:a + 1]).sum() for a in range(3)])
    assert np.all(np.abs(mom - mref) <= 1e-12 * ref.f.sum())


@pytest.mark.parametrize("storage,tol_u", [(psm.PSM_FP32DEV, 2e-5), (psm.PSM_FP16DEV, 3e-3)])
def test_pressure_outflow_deviation_forms(storage, tol_u):
    spec = _outflow((28, 20, 18), 2, seed=8, storage_rho=1.002)
    ref = run_oracle(spec, 40)
    f, *_, eng = run_engine(spec, 40, storage=storage)
    eng.close()
    box = oracle.Box(*spec.dims, tau=spec.tau)
    _, u_ref = oracle.macroscopic(box, ref.f)
    _, u = oracle.macroscopic(box, f)
    assert np.linalg.norm(u - u_ref) / np.linalg.norm(u_ref) < tol_u


def test_pressure_outflow_state_roundtrip_and_plug_flow():
    """set_pdfs inverts the anti-bounce-back read (fixed-point solve of the
    boundary slots), and the uniform inflow velocity is an exact fixed point
    that a start from rest converges to."""
    spec = _outflow((12, 8, 10), 0, seed=3)
    f0 = initial_f(spec) + 1e-3 * np.random.default_rng(4).standard_normal((19, spec.N))
    eng = make_engine([spec])
    eng.set_pdfs(0, f0)
    f1 = eng.get_pdfs(0).cpu().numpy()
    eng.close()
    assert np.max(np.abs(f1 - f0)) <= 1e-15
    U = np.array(spec.wall_u[0])
    plug = inputs.BoxSpec(dims=(4, 4, 10), tau=0.8, walls_z=True, wall_u=(tuple(U), (0.0, 0.0, 0.0)),
                          face_type=(0, 1), u0=np.repeat(U[:, None], 160, axis=1))
    fp = initial_f(plug)
    f2, *_, eng = run_engine(plug, 100)
    eng.close()
    assert np.max(np.abs(f2 - fp)) < 1e-15
    rest = inputs.BoxSpec(dims=(4, 4, 10), tau=0.8, walls_z=True, wall_u=(tuple(U), (0.0, 0.0, 0.0)),
                          face_type=(0, 1))
    f3, *_, eng = run_engine(rest, 7000, launch=(16, 16, 2, 0))
    eng.close()
    assert np.max(np.abs(f3 - fp)) < 1e-12


def _bed(dims, n, seed, tau=0.7, U=(0.0, 0.0, 0.01), rho_out=1.0):
    """A small fluidized-bed-like box: resting side walls in x and y, a
    velocity inflow at z = 0, a pressure outflow at z = nz, spheres at least
    r + 1 from every wall."""
    rng = np.random.default_rng(seed)
    r = rng.uniform(2.5, 4.0, n)
    L = np.asarray(dims, dtype=float)
    x = (r + 1.0)[:, None] + rng.random((n, 3)) * (L[None, :] - 2.0 * (r + 1.0)[:, None])
    base = inputs.random_small(dims, 0, (2, 3), seed=seed, tau=tau)
    return inputs.BoxSpec(dims=dims, tau=tau, fext=(0.0, 0.0, -2e-6), x=x, r=r,
                          U=inputs.uniform_velocities(rng, n, 0.01), Om=inputs.uniform_velocities(rng, n, 0.002),
                          u0=0.5 * base.u0, walls_z=True, wall_u=(U, (0.0, 0.0, 0.0)), face_type=(0, 1),
                          face_rho=(1.0, rho_out), walls_x=True, walls_y=True)


@pytest.mark.parametrize("dims,launch", [((30, 22, 26), (32, 8, 4, 0)), ((41, 27, 19), (64, 4, 8, 3)),
                                         ((20, 36, 24), (16, 16, 2, 2)),
                                         # rows padded to a 64-cell block (pitch 64 for nx 59)
                                         ((59, 18, 22), (64, 4, 4, 2))])
def test_side_walls_bed_parity_fp64(dims, launch):
    spec = _bed(dims, 4, seed=sum(dims), rho_out=1.001)
    print(f"[case] bed fp64 dims={dims} launch={launch}", flush=True)
    ref = run_oracle(spec, 15)
    f, F, T, B, pid, eng = run_engine(spec, 15, launch=launch)
    mass, mom, _ = eng.get_stats(0)
    eng.close()
    assert_pdfs_close(f, ref.f, 1e-12)
    assert_forces_close(F, ref.F, ref.A)
    assert_forces_close(T, ref.T, ref.A, lever=spec.r.max() + 1)
    c, _, _ = oracle.lattice()
    assert abs(mass - ref.f.sum()) <= 1e-12 * ref.f.sum()
    mref = np.array([(ref.f * c[:, a:a + 1]).sum() for a in range(3)])
    assert np.all(np.abs(mom - mref) <= 1e-12 * ref.f.sum())


@pytest.mark.parametrize("storage,tol_u", [(psm.PSM_FP32DEV, 2e-5), (psm.PSM_FP16DEV, 3e-3)])
def test_side_walls_bed_deviation_forms(storage, tol_u):
    spec = _bed((24, 20, 18), 2, seed=12)
    ref = run_oracle(spec, 40)
    f, *_, eng = run_engine(spec, 40, storage=storage)
    eng.close()
    box = oracle.Box(*spec.dims, tau=spec.tau)
    _, u_ref = oracle.macroscopic(box, ref.f)
    _, u = oracle.macroscopic(box, f)
    assert np.linalg.norm(u - u_ref) / np.linalg.norm(u_ref) < tol_u


def test_side_walls_roundtrip_and_duct_profile():
    spec = _bed((14, 10, 8), 0, seed=6)
    f0 = initial_f(spec) + 1e-3 * np.random.default_rng(7).standard_normal((19, spec.N))
    eng = make_engine([spec])
    eng.set_pdfs(0, f0)
    f1 = eng.get_pdfs(0).cpu().numpy()
    eng.close()
    assert np.max(np.abs(f1 - f0)) <= 1e-15
    # body-force flow along z between x walls: the half-way bounce-back closed form
    H, tau, g = 10, 0.8, 1e-5
    nu = (tau - 0.5) / 3.0
    duct = inputs.BoxSpec(dims=(H, 4, 4), tau=tau, fext=(0.0, 0.0, g), walls_x=True)
    steps = int(40 * H * H / (math.pi ** 2 * nu)) + 200
    f, *_, eng = run_engine(duct, steps, launch=(16, 16, 4, 0))
    _, u = eng.get_macroscopic(0)
    u = u.cpu().numpy()
    eng.close()
    x = np.arange(H) + 0.0
    exact = g / (2 * nu) * (x + 0.5) * (H - 0.5 - x) + 2 * g / (3 * nu) * ((tau - 0.5) ** 2 - 3.0 / 16.0)
    prof = u[2].reshape(4, 4, H)[0, 0, :]
    assert np.max(np.abs(prof - exact)) / exact.max() < 1e-9


def test_mixed_boxes_in_one_launch():
    """A periodic box, a channel with moving walls and a closed bed with
    sub-sampled spheres in one context (one launch per step) each match the
    oracle run alone, also under device-side sphere updates with different
    dynamics per box."""
    specs = [inputs.random_small((30, 28, 26), 4, (2.5, 4.0), seed=51, tau=0.66, fext=(1e-5, 0, 0),
                                 vamp=0.05, omamp=0.002),
             _channel((34, 24, 22), 3, seed=52),
             _bed((26, 30, 28), 3, seed=53, rho_out=1.002)]
    specs[2].mapping = psm.PSM_MAP_SUBSAMPLE
    dyn_par = [(1.2, (0.0, 0.0, 0.0)), (1.8, (0.0, 0.0, -2e-4)), (2.5, (1e-4, 0.0, -1e-4))]
    steps = 8
    print("[case] mixed boxes", flush=True)
    refs = []
    for s, (rho_p, acc) in zip(specs, dyn_par):
        box = oracle_box_of(s)
        f = initial_f(s)
        dyn = oracle.Dynamics(s.x, s.r, s.U, s.Om)
        for _ in range(steps):
            ref = oracle.run(box, f, 1, dyn.x, dyn.r, dyn.U, dyn.Om)
            f = ref.f
            oracle.integrate(box, dyn, ref.F, ref.T, dt=1.0, scheme=psm.PSM_VERLET, rho_p=rho_p, accel=acc)
        refs.append((f, ref, dyn))
    eng = make_engine(specs)
    eng.set_launch(32, 8, 4, psm.PSM_LAUNCH_FILTER)
    for b, (s, (rho_p, acc)) in enumerate(zip(specs, dyn_par)):
        eng.set_pdfs(b, initial_f(s))
        eng.set_particles(b, s.x, s.r, s.U, s.Om)
        eng.set_dynamics(b, rho_p, acc)
    eng.run(steps, 1.0, psm.PSM_VERLET)
    for b, (f, ref, dyn) in enumerate(refs):
        assert_pdfs_close(eng.get_pdfs(b).cpu().numpy(), f, 1e-12)
        F, T = eng.get_forces(b)
        assert_forces_close(F, ref.F, ref.A)
        x, U, _ = eng.get_particles(b)
        assert np.allclose(x, dyn.x, rtol=1e-12, atol=1e-12)
        assert np.allclose(U, dyn.U, rtol=1e-12, atol=1e-15)
    eng.close()


def oracle_box_of(spec):
    from psm_cases import oracle_box
    return oracle_box(spec)


@pytest.mark.parametrize("storage,tol_u", [(psm.PSM_FP32DEV, 2e-5), (psm.PSM_FP16DEV, 3e-3)])
def test_mixed_boxes_deviation_forms_with_graphs(storage, tol_u):
    """Mixed boxes (periodic, wall channel, closed bed with sampled spheres)
    in a deviation form, persistent grid with the filter, graph replays; then
    fewer spheres in one box and no spheres in another, and more steps: each
    box stays within the form's velocity bound of the oracle."""
    specs = [inputs.random_small((28, 26, 24), 4, (2.5, 4.0), seed=61, tau=0.7, fext=(1e-5, 0, 0)),
             _channel((30, 22, 20), 3, seed=62),
             _bed((24, 26, 26), 3, seed=63)]
    specs[2].mapping = psm.PSM_MAP_SUBSAMPLE
    print(f"[case] mixed boxes storage={storage}", flush=True)
    eng = make_engine(specs, storage=storage)
    eng.set_launch(64, 4, 4, psm.PSM_LAUNCH_PERSISTENT | psm.PSM_LAUNCH_FILTER)
    eng.set_graph(True)
    for b, s in enumerate(specs):
        eng.set_pdfs(b, initial_f(s))
        eng.set_particles(b, s.x, s.r, s.U, s.Om)
    eng.step(20)
    # second phase: box 0 keeps two spheres, box 1 none
    s0, s1 = specs[0], specs[1]
    eng.set_particles(0, s0.x[:2], s0.r[:2], s0.U[:2], s0.Om[:2])
    eng.set_particles(1, np.zeros((0, 3)), np.zeros(0), np.zeros((0, 3)))
    eng.step(10)
    got = [eng.get_pdfs(b).cpu().numpy() for b in range(3)]
    eng.close()
    phase2 = [dict(x=s0.x[:2], r=s0.r[:2], U=s0.U[:2], Om=s0.Om[:2]),
              dict(x=np.zeros((0, 3)), r=np.zeros(0), U=np.zeros((0, 3)), Om=np.zeros((0, 3))),
              dict(x=specs[2].x, r=specs[2].r, U=specs[2].U, Om=specs[2].Om)]
    for b, s in enumerate(specs):
        box = oracle_box_of(s)
        f = oracle.run(box, initial_f(s), 20, s.x, s.r, s.U, s.Om).f
        p2 = phase2[b]
        f = oracle.run(box, f, 10, p2["x"], p2["r"], p2["U"], p2["Om"]).f
        ob = oracle.Box(*s.dims, tau=s.tau)
        _, u_ref = oracle.macroscopic(ob, f)
        _, u = oracle.macroscopic(ob, got[b])
        assert np.linalg.norm(u - u_ref) / np.linalg.norm(u_ref) < tol_u, b


@pytest.mark.parametrize("storage", [psm.PSM_FP32DEV, psm.PSM_FP16DEV])
@pytest.mark.parametrize("case", ["moving_walls", "bed"])
def test_deviation_forms_one_step_every_value_with_boundaries(storage, case):
    """Every value of the box after one step from the engine's own state
    agrees with the FP64 oracle's step from that state to the one-step bound
    of the deviation forms (psm_cases.one_step_bound: the storage rounding of
    the stored post-collision value each canonical value comes from, which
    for a population entering through a wall or face is the cell's own
    opposite value, plus the FP32 collision): moving no-slip walls with a
    body force, and the bed box (resting side walls, velocity inflow, pressure
    outflow at a raised density), two launches each."""
    from psm_cases import one_step_bound, oracle_box, post_collision_field

    spec = (_channel((34, 22, 20), 3, seed=31) if case == "moving_walls"
            else _bed((30, 22, 24), 3, seed=32, rho_out=1.002))
    box = oracle_box(spec)
    for launch in ((64, 4, 4, 0), (32, 8, 2, 0)):
        print(f"[case] one step {case} storage={storage} launch={launch}", flush=True)
        eng = make_engine([spec], storage=storage)
        eng.set_launch(*launch)
        eng.set_pdfs(0, initial_f(spec))
        eng.set_particles(0, spec.x, spec.r, spec.U, spec.Om)
        eng.step(3)
        f_t = eng.get_pdfs(0).cpu().numpy()
        eng.step(1)
        got = eng.get_pdfs(0).cpu().numpy()
        eng.close()
        ref = oracle.run(box, f_t, 1, spec.x, spec.r, spec.U, spec.Om).f
        bound = one_step_bound(spec, storage, f_t, post_collision_field(box, f_t, spec.x, spec.r, spec.U, spec.Om))
        ratio = float(np.max(np.abs(got - ref) / bound))
        print(f"[ratio] max |err|/bound = {ratio:.3g}", flush=True)
        assert ratio <= 1.0
