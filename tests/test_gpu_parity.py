"""GPU-vs-oracle parity of the fused PSM-LBM step (FP64 storage), called
through the C ABI. Tolerance for FP64: 1e-12 relative on PDFs, density and
velocity; forces and torques to 1e-12 relative plus 1e-14 of the force's
term magnitude (the two sides sum the same terms in different orders);
solid-fraction slots: particle ids exact, fractions exact for sub-sampling
and to 1e-15 for the linear approximation."""
import numpy as np
import pytest

import oracle
import paper_2303_11811_amd as psm
from paper_2303_11811_amd import inputs
from psm_cases import (assert_forces_close, assert_pdfs_close, initial_f, make_engine, run_engine,
                       run_oracle)

pytestmark = pytest.mark.gpu


def _print_case(name, **kw):
    print(f"[case] {name} {kw}", flush=True)


@pytest.mark.parametrize("launch", [None, (32, 8, 4, psm.PSM_LAUNCH_FILTER)])
def test_parity_32_subsample_100_steps(launch):
    """32^3, tau 0.6, Taylor-Green start, 8 spheres r=4 with 4^3 sampling."""
    spec = inputs.parity_32(seed=0)
    _print_case("parity_32", steps=100, launch=launch)
    ref = run_oracle(spec, 100)
    f, F, T, B, pid, eng = run_engine(spec, 100, launch=launch)
    assert_pdfs_close(f, ref.f, 1e-12)
    assert np.array_equal(pid, ref.pid)
    assert np.array_equal(B, ref.B)
    assert_forces_close(F, ref.F, ref.A)
    assert_forces_close(T, ref.T, ref.A, lever=spec.r.max() + 1)
    rho, u = eng.get_macroscopic(0)
    rho_ref, u_ref = oracle.macroscopic(oracle.Box(*spec.dims, tau=spec.tau), ref.f)
    assert np.allclose(rho.cpu().numpy(), rho_ref, rtol=1e-12, atol=0)
    assert np.allclose(u.cpu().numpy(), u_ref, rtol=0, atol=1e-14)


RAGGED = [
    # dims, tiles (tx, ty, tz), particles, overlap
    ((40, 36, 20), (64, 4, 4), 4, False),
    ((37, 29, 23), (32, 8, 16), 5, False),
    ((70, 21, 18), (16, 16, 2), 3, True),
    ((33, 40, 27), (128, 2, 8), 6, True),
    ((24, 24, 24), (256, 1, 32), 2, False),
    ((45, 38, 31), (64, 4, 8, 1), 5, False),
    ((52, 33, 29), (32, 8, 2, 1), 4, True),
    # with the per-wave candidate filter (flag 2), also combined with the persistent grid
    ((40, 36, 20), (64, 4, 4, 2), 4, False),
    ((70, 21, 18), (16, 16, 2, 2), 3, True),
    ((33, 40, 27), (128, 2, 8, 3), 6, True),
    ((24, 24, 24), (256, 1, 32, 2), 2, False),
    # row pitch padded to whole 64-cell blocks (nx 60 -> 64, nx 121 -> 128)
    ((60, 22, 18), (64, 4, 4), 4, True),
    ((121, 14, 12), (128, 2, 8, 3), 5, False),
    ((60, 22, 18), (32, 8, 2, 2), 4, True),
]


@pytest.mark.parametrize("dims,tiles,npart,overlap", RAGGED)
def test_parity_ragged_linear(dims, tiles, npart, overlap, radii=(2.5, 4.0)):
    """Boxes that are not multiples of the tile, several tiles per axis,
    body force, rotating spheres, overlapping spheres (renormalised slots)."""
    spec = inputs.random_small(dims, npart, radii, seed=sum(dims), tau=0.67,
                               fext=(2e-5, -1e-5, 5e-6), vamp=0.01, omamp=0.002, overlap=overlap)
    _print_case("ragged", dims=dims, tiles=tiles, n=len(spec.r))
    steps = 12
    ref = run_oracle(spec, steps)
    f, F, T, B, pid, eng = run_engine(spec, steps, launch=tiles)
    assert_pdfs_close(f, ref.f, 1e-12)
    assert np.array_equal(pid, ref.pid)
    assert np.max(np.abs(B - ref.B)) <= 1e-15
    assert_forces_close(F, ref.F, ref.A)
    assert_forces_close(T, ref.T, ref.A, lever=spec.r.max() + 1)
    _, _, ov = eng.get_stats(0)
    # overflow count of the current mapping equals the oracle's
    assert ov == ref.overflow


@pytest.mark.parametrize("dims,tiles,npart,radii", [
    # the smallest spheres allowed (r = 1: f(r) needs r^2 > 1/2), many per tile
    ((24, 20, 16), (64, 4, 4, 0), 12, (1.0, 1.5)),
    ((24, 20, 16), (16, 16, 2, 3), 12, (1.0, 1.5)),
    # one sphere nearly as large as the box allows (L >= 2 (r + 1) + 2): its
    # bounding box wraps in every axis and covers most tiles
    ((24, 24, 22), (32, 8, 4, 2), 1, (9.0, 9.0)),
])
def test_parity_extreme_radii(dims, tiles, npart, radii):
    """The radius limits of the linear mapping, checked like the ragged cases."""
    test_parity_ragged_linear(dims, tiles, npart, npart > 1, radii=radii)


@pytest.mark.parametrize("launch", [(16, 16, 1, 0), (16, 16, 2, 2), (32, 8, 4, 1)])
def test_parity_spheres_wrapping_through_short_last_tiles(launch):
    """Periodic axes whose last tile is short (33 = 16 + 16 + 1 and
    41 = 16 + 16 + 9 cells at 16-cell tiles), with spheres whose cell range
    wraps through that tile and so touches one tile more than a range of the
    same length that does not wrap: each sphere's force partials, one per
    tile it touches, must stay inside its own slots."""
    x = np.array([[32.3, 20.0, 13.0], [32.3, 3.5, 15.5], [0.4, 0.6, 24.0], [10.0, 10.0, 25.5],
                  [31.6, 39.7, 9.0]])
    r = np.array([4.0, 4.0, 3.2, 2.5, 3.9])
    rng = np.random.default_rng(7)
    spec = inputs.BoxSpec(dims=(33, 41, 26), tau=0.7, fext=(2e-5, -1e-5, 5e-6), x=x, r=r,
                          U=rng.uniform(-0.01, 0.01, (5, 3)), Om=rng.uniform(-0.002, 0.002, (5, 3)))
    _print_case("short last tiles", launch=launch)
    steps = 10
    ref = run_oracle(spec, steps)
    f, F, T, B, pid, eng = run_engine(spec, steps, launch=launch)
    eng.close()
    assert_pdfs_close(f, ref.f, 1e-12)
    assert np.array_equal(pid, ref.pid)
    assert_forces_close(F, ref.F, ref.A)
    assert_forces_close(T, ref.T, ref.A, lever=r.max() + 1)


def test_parity_no_particles_with_force():
    spec = inputs.random_small((48, 20, 12), 0, (2, 3), seed=3, tau=0.83, fext=(1e-5, 2e-6, -3e-6))
    ref = run_oracle(spec, 30)
    f, *_ = run_engine(spec, 30)
    assert_pdfs_close(f, ref.f, 1e-12)


def test_set_equilibrium_matches_oracle():
    spec = inputs.random_small((20, 12, 9), 0, (2, 3), seed=8, tau=0.7, fext=(1e-4, 0, 0))
    eng = make_engine([spec])
    eng.set_equilibrium(0, spec.u0, spec.rho0)
    f = eng.get_pdfs(0).cpu().numpy()
    ref = initial_f(spec)
    assert np.max(np.abs(f - ref)) <= 1e-16


def test_batched_boxes_match_single_runs():
    """Three boxes of different sizes, relaxation times, forces and particles
    in one context advance exactly as the oracle advances each alone."""
    specs = [inputs.random_small((32, 32, 32), 4, (3.0, 4.0), seed=11, tau=0.55),
             inputs.random_small((48, 40, 36), 6, (3.0, 5.0), seed=12, tau=0.93, fext=(0, 3e-6, 0)),
             inputs.random_small((20, 20, 20), 0, (2, 3), seed=13, tau=0.71)]
    eng = make_engine(specs)
    for b, s in enumerate(specs):
        eng.set_pdfs(b, initial_f(s))
        if s.n_particles:
            eng.set_particles(b, s.x, s.r, s.U, s.Om)
    eng.step(9)
    forces = {}
    for b, s in enumerate(specs):
        ref = run_oracle(s, 9)
        assert_pdfs_close(eng.get_pdfs(b).cpu().numpy(), ref.f, 1e-12)
        if s.n_particles:
            F, T = eng.get_forces(b)
            forces[b] = (F, T)
            assert_forces_close(F, ref.F, ref.A)
            assert_forces_close(T, ref.T, ref.A, lever=s.r.max() + 1)
    eng.close()
    # the same run with the force read-back: each box's forces from the one
    # copy of all boxes' sums that the step makes, bit for bit
    eng = make_engine(specs)
    eng.set_force_readback(True)
    for b, s in enumerate(specs):
        eng.set_pdfs(b, initial_f(s))
        if s.n_particles:
            eng.set_particles(b, s.x, s.r, s.U, s.Om)
    eng.step(9)
    for b, (F, T) in forces.items():
        Fr, Tr = eng.get_forces(b)
        assert np.array_equal(F, Fr) and np.array_equal(T, Tr)
    eng.close()


def test_graph_replay_equals_eager_bitwise():
    spec = inputs.random_small((40, 36, 28), 5, (3.0, 4.5), seed=21, tau=0.6, fext=(1e-5, 0, 0),
                               omamp=0.002)
    f_e, F_e, T_e, *_ = run_engine(spec, 20, graph=False)
    f_g, F_g, T_g, *_ = run_engine(spec, 20, graph=True)
    assert np.array_equal(f_e, f_g)
    assert np.array_equal(F_e, F_g) and np.array_equal(T_e, T_g)
    # replays interleaved with eager steps and syncs
    f_m, F_m, _, _, _, eng = run_engine(spec, 13, graph=True)
    eng.step(7)
    f2 = eng.get_pdfs(0).cpu().numpy()
    assert np.array_equal(f2, f_e)
    eng.close()
    # every replay checked against the eager engine, with synchronising reads
    # and eager steps of the graph engine (odd counts switch the captured
    # graph's starting parity) between the replays
    engines = []
    for graph in (False, True):
        e = make_engine([spec])
        e.set_graph(graph)
        e.set_pdfs(0, initial_f(spec))
        e.set_particles(0, spec.x, spec.r, spec.U, spec.Om)
        engines.append(e)
    eager, graphed = engines
    for n in (10, 10, 3, 10, 10, 1, 20):
        eager.step(n)
        graphed.step(n)
        assert np.array_equal(eager.get_pdfs(0).cpu().numpy(), graphed.get_pdfs(0).cpu().numpy()), n
        Fa, Ta = eager.get_forces(0)
        Fb, Tb = graphed.get_forces(0)
        assert np.array_equal(Fa, Fb) and np.array_equal(Ta, Tb), n
    for e in engines:
        e.close()


def test_deterministic_repeat():
    spec = inputs.random_small((36, 36, 36), 6, (3.0, 5.0), seed=31, tau=0.7, omamp=0.003)
    a = run_engine(spec, 10)
    b = run_engine(spec, 10)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])


def test_stats_mass_and_momentum():
    spec = inputs.random_small((30, 26, 22), 3, (2.5, 3.5), seed=41, tau=0.8, fext=(3e-5, 0, 1e-5))
    ref = run_oracle(spec, 5)
    f, F, T, B, pid, eng = run_engine(spec, 5)
    mass, mom, ov = eng.get_stats(0)
    c, _, _ = oracle.lattice()
    assert abs(mass - ref.f.sum()) <= 1e-12 * ref.f.sum()
    assert np.allclose(mom, (ref.f.T @ c.astype(float)).sum(0), rtol=1e-10, atol=1e-13)


def test_tile_capacity_error_is_reported():
    """More sphere candidates in one tile than the kernel stages: the lists
    are built on the device without waiting, the list of that tile is cut (a
    step still runs in bounds), the next synchronising call reports
    PSM_ECAPACITY, the context refuses to step, and a valid set makes it
    usable again."""
    dims = (64, 64, 64)
    rng = np.random.default_rng(5)
    n = 80
    x = np.column_stack([rng.uniform(20, 44, n), rng.uniform(20, 24, n), rng.uniform(30, 34, n)])
    r = np.full(n, 1.5)
    eng = psm.Engine([psm.make_desc(*dims, 0.7, max_particles=n, max_radius=2.0)])
    eng.set_equilibrium(0, np.zeros((3, dims[0] * dims[1] * dims[2])))
    eng.set_launch(256, 1, 32)
    eng.set_particles(0, x, r, np.zeros((n, 3)))
    eng.step(1)
    with pytest.raises(psm.PsmError) as e:
        eng.get_forces(0)
    assert e.value.code == psm.PSM_ECAPACITY
    with pytest.raises(psm.PsmError) as e:
        eng.step(1)
    assert e.value.code == psm.PSM_ESTATE
    eng.set_particles(0, x[:4], r[:4], np.zeros((4, 3)))
    eng.set_equilibrium(0, np.zeros((3, dims[0] * dims[1] * dims[2])))
    eng.step(1)
    F, _ = eng.get_forces(0)
    assert np.all(np.isfinite(F))
    eng.close()


def test_velocity_only_update_keeps_lists_and_uses_new_velocities():
    """Re-setting the spheres with the same positions and radii but new
    velocities skips the re-binning; the next step must use the new U, Omega."""
    spec = inputs.random_small((40, 32, 30), 5, (3.0, 4.5), seed=71, tau=0.66, omamp=0.002)
    f0 = initial_f(spec)
    eng = make_engine([spec])
    eng.set_pdfs(0, f0)
    eng.set_particles(0, spec.x, spec.r, spec.U, spec.Om)
    eng.step(3)
    f_mid = eng.get_pdfs(0).cpu().numpy()
    rng = np.random.default_rng(3)
    U2 = inputs.uniform_velocities(rng, len(spec.r), 0.02)
    Om2 = inputs.uniform_velocities(rng, len(spec.r), 0.003)
    eng.set_particles(0, spec.x, spec.r, U2, Om2)
    eng.step(4)
    f = eng.get_pdfs(0).cpu().numpy()
    F, T = eng.get_forces(0)
    spec2 = inputs.BoxSpec(dims=spec.dims, tau=spec.tau, fext=spec.fext, x=spec.x, r=spec.r, U=U2, Om=Om2)
    ref = run_oracle(spec2, 4, f0=f_mid)
    assert_pdfs_close(f, ref.f, 1e-12)
    assert_forces_close(F, ref.F, ref.A)
    assert_forces_close(T, ref.T, ref.A, lever=spec.r.max() + 1)


def test_many_tiles_multi_chunk_scan():
    """A box with more than ten thousand tiles (tile 16 x 16 x 1): the tile
    scan runs over many chunks."""
    spec = inputs.random_small((200, 160, 40), 12, (3.0, 6.0), seed=81, tau=0.75, fext=(0, 0, 2e-6))
    steps = 3
    ref = run_oracle(spec, steps)
    f, F, T, B, pid, eng = run_engine(spec, steps, launch=(16, 16, 1, 0))
    assert_pdfs_close(f, ref.f, 1e-12)
    assert np.array_equal(pid, ref.pid)
    assert_forces_close(F, ref.F, ref.A)


def test_checkpoint_resume_bitwise():
    """State = canonical PDFs + spheres: step(2n) equals step(n) -> save ->
    new context -> restore -> step(n), bit for bit (forces too: the force
    reduction has a fixed order)."""
    spec = inputs.random_small((44, 36, 30), 5, (3.0, 4.5), seed=91, tau=0.61, fext=(1e-5, 0, 0), omamp=0.002)
    f_full, F_full, T_full, *_ = run_engine(spec, 16, launch=(64, 4, 2, 0))
    f_half, *_ = run_engine(spec, 8, launch=(64, 4, 2, 0))
    f_res, F_res, T_res, *_ = run_engine(spec, 8, launch=(64, 4, 2, 0), f0=f_half)
    assert np.array_equal(f_full, f_res)
    assert np.array_equal(F_full, F_res) and np.array_equal(T_full, T_res)


@pytest.mark.parametrize("storage", [psm.PSM_FP64, psm.PSM_FP16DEV])
def test_persistent_grid_matches_one_workgroup_per_tile(storage):
    """The persistent grid hands tiles out through per-die counters that a
    kernel zeroes before every step, also inside captured graphs: its PDFs,
    forces and torques are bit for bit those of one workgroup per tile at the
    same tile shape, over eager steps and over several graph replays."""
    specs = [inputs.random_small((44, 36, 30), 5, (3.0, 4.5), seed=93, tau=0.62, fext=(1e-5, 0, 0)),
             inputs.random_small((21, 50, 17), 3, (2.5, 3.5), seed=94, tau=0.8)]
    out = {}
    for flags in (0, psm.PSM_LAUNCH_PERSISTENT):
        eng = make_engine(specs, storage=storage, max_radius=4.5)
        eng.set_launch(64, 4, 2, flags)
        for b, sp in enumerate(specs):
            eng.set_pdfs(b, initial_f(sp))
            eng.set_particles(b, sp.x, sp.r, sp.U, sp.Om)
        res = []
        for graph, n in ((False, 3), (True, 10), (True, 10), (False, 1), (True, 10)):
            eng.set_graph(graph)
            eng.step(n)
            res.append([(eng.get_pdfs(b).cpu().numpy(), *eng.get_forces(b)) for b in range(len(specs))])
        out[flags] = res
        eng.close()
    for r0, r1 in zip(out[0], out[psm.PSM_LAUNCH_PERSISTENT]):
        for a, b in zip(r0, r1):
            assert all(np.array_equal(x, y) for x, y in zip(a, b))


def test_kernel_timing_counts_every_eager_launch():
    """Timing events come from a fixed pool that is folded into the totals
    when full: 300 steps (more than the pool's 128 pairs) count 300 launches
    with a positive total; with timing on, steps run eagerly even where graphs
    are enabled, so they are counted too; reset clears."""
    spec = inputs.random_small((40, 36, 28), 3, (3.0, 4.0), seed=95, tau=0.7)
    eng = make_engine([spec])
    eng.set_pdfs(0, initial_f(spec))
    eng.set_particles(0, spec.x, spec.r, spec.U, spec.Om)
    eng.set_timing(True)
    eng.step(300)
    n, ms = eng.get_timing()
    assert n == 300 and ms > 0.0
    eng.set_graph(True)
    eng.step(20)
    assert eng.get_timing()[0] == 320
    eng.set_graph(False)
    eng.reset_timing()
    eng.step(5)
    n, ms5 = eng.get_timing()
    assert n == 5 and 0.0 < ms5 < ms
    eng.close()


@pytest.mark.parametrize("storage", [psm.PSM_FP64, psm.PSM_FP16DEV])
def test_pattern_copy_leaves_the_state(storage):
    """The access-pattern bandwidth reference writes only the grid the next
    step overwrites: the state, and the steps after it, are bit for bit those
    of a context that never ran it."""
    spec = inputs.random_small((44, 36, 30), 5, (3.0, 4.5), seed=92, tau=0.62, fext=(1e-5, 0, 0))
    f_ref, F_ref, T_ref, *_ = run_engine(spec, 4, storage=storage, launch=(64, 4, 2, 0))
    eng = make_engine([spec], storage=storage)
    eng.set_launch(64, 4, 2, 0)
    eng.set_pdfs(0, initial_f(spec))
    eng.set_particles(0, spec.x, spec.r, spec.U, spec.Om)
    eng.step(2)
    f_mid = eng.get_pdfs(0).cpu().numpy()
    for shifted in (1, 0):
        ms = eng.pattern_copy(shifted, 2)
        assert ms > 0.0
    assert np.array_equal(eng.get_pdfs(0).cpu().numpy(), f_mid)
    eng.step(2)
    F, T = eng.get_forces(0)
    assert np.array_equal(eng.get_pdfs(0).cpu().numpy(), f_ref)
    assert np.array_equal(F, F_ref) and np.array_equal(T, T_ref)
    with pytest.raises(psm.PsmError):
        eng.pattern_copy(2, 1)
    eng.close()


def test_nonfinite_state_is_reported():
    spec = inputs.random_small((24, 20, 16), 2, (2.5, 3.0), seed=5, tau=0.7)
    f0 = initial_f(spec)
    f0[3, 777] = np.nan
    eng = make_engine([spec])
    eng.set_pdfs(0, f0)
    eng.set_particles(0, spec.x, spec.r, spec.U, spec.Om)
    eng.step(2)
    with pytest.raises(psm.PsmError) as e:
        eng.get_stats(0)
    assert e.value.code == psm.PSM_ENONFINITE


@pytest.mark.parametrize("storage", [psm.PSM_FP64, psm.PSM_FP32DEV, psm.PSM_FP16DEV])
def test_candidate_filter_is_exact(storage):
    """The per-wave candidate filter only skips spheres that give zero
    fraction, so every storage form produces bitwise the same PDFs, forces and
    slots with and without it, here on a dense packing (many candidates per
    tile, overlapping spheres, ragged tiles, both mappings)."""
    for mapping, dims in ((psm.PSM_MAP_LINEAR, (72, 50, 36)), (psm.PSM_MAP_SUBSAMPLE, (40, 34, 30))):
        spec = inputs.random_small(dims, 40, (2.0, 5.0), seed=11, tau=0.7, fext=(1e-5, 0, -2e-6),
                                   vamp=0.01, omamp=0.003, overlap=True, mapping=mapping)
        _print_case("filter", storage=storage, mapping=mapping, dims=dims, n=len(spec.r))
        out = []
        for launch in ((32, 8, 4, 0), (32, 8, 4, psm.PSM_LAUNCH_FILTER)):
            f, F, T, B, pid, eng = run_engine(spec, 6, storage=storage, launch=launch)
            eng.close()
            out.append((f, F, T, B, pid))
        for a, b in zip(*out):
            assert np.array_equal(a, b)


def test_autotune_picks_an_allowed_launch_and_keeps_parity():
    """The tuner's pick is one of the documented shapes, is the launch the
    context keeps, and the step under it still matches the oracle."""
    spec = inputs.random_small((60, 22, 18), 4, (2.5, 4.0), seed=81, tau=0.7, fext=(1e-5, 0, 0), overlap=True)
    print("[case] autotune", flush=True)
    eng = make_engine([spec])
    eng.set_pdfs(0, initial_f(spec))
    eng.set_particles(0, spec.x, spec.r, spec.U, spec.Om)
    shape, ms = eng.autotune(trial_steps=2)
    tx, ty, tz, flags = shape
    assert tx in (16, 32, 64, 128, 256) and tx * ty == 256 and tz in (1, 2, 4, 8, 16, 32)
    assert flags in (0, 1, 2, 3) and ms > 0.0
    assert tuple(eng.get_launch()) == tuple(shape)
    ref = run_oracle(spec, 10)
    f, F, T, B, pid, eng = run_engine(spec, 10, eng=eng)
    assert_pdfs_close(f, ref.f, 1e-12)
    assert np.array_equal(pid, ref.pid)
    assert_forces_close(F, ref.F, ref.A)
    eng.close()


def test_autotune_cache(tmp_path, monkeypatch):
    """A second context of the same class (same box, storage, walls and
    sphere volume fraction) gets the cached pick without trials (its PDF
    state is left as set); the pick is appended to the file PSM_TUNE_CACHE
    names; psm_clear_tune_cache forgets it (and does not read the file
    again), so the next context is timed again."""
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("PSM_TUNE_CACHE", str(cache))
    psm.psm_clear_tune_cache()
    spec = inputs.random_small((50, 20, 16), 3, (2.5, 3.5), seed=83, tau=0.7)
    f0 = initial_f(spec)

    def tuned():
        eng = make_engine([spec])
        eng.set_pdfs(0, f0)
        eng.set_particles(0, spec.x, spec.r, spec.U, spec.Om)
        shape, ms = eng.autotune(trial_steps=2)
        advanced = not np.array_equal(eng.get_pdfs(0).cpu().numpy(), f0)
        eng.close()
        return shape, ms, advanced

    s1, ms1, adv1 = tuned()
    s2, ms2, adv2 = tuned()
    assert adv1 and not adv2 and s1 == s2 and ms1 == ms2
    lines = cache.read_text().split("\n")
    assert len([l for l in lines if l.strip()]) == 1 and "|s0|" in lines[0]
    psm.psm_clear_tune_cache()
    s3, _, adv3 = tuned()
    assert adv3
    monkeypatch.delenv("PSM_TUNE_CACHE")
    psm.psm_clear_tune_cache()


def test_state_and_argument_errors_on_a_live_context():
    """The documented codes on a live context, each leaving it usable: more
    spheres than max_particles (PSM_ECAPACITY), radius out of range, box out
    of range, NULL buffers, bad time step, scheme, density ratio, launch or
    trial count (PSM_EINVAL); a context with no spheres set steps as plain
    LBM; forces read before any step of a sphere set are zeros; afterwards
    the context still matches the oracle."""
    import ctypes

    spec = inputs.random_small((30, 20, 16), 3, (2.5, 3.5), seed=97, tau=0.75, fext=(1e-5, 0, 0), vamp=0.01)
    print("[case] state and argument errors", flush=True)
    eng = make_engine([spec], max_particles=3, max_radius=4.0)
    L = psm.lib()
    assert L.psm_step(eng.ctx, 1) == psm.PSM_OK
    x4 = np.vstack([spec.x, spec.x[:1]])
    with pytest.raises(psm.PsmError) as e:
        eng.set_particles(0, x4, np.full(4, 3.0), np.zeros((4, 3)))
    assert e.value.code == psm.PSM_ECAPACITY
    for bad_r in (0.5, 4.5):
        with pytest.raises(psm.PsmError) as e:
            eng.set_particles(0, spec.x, np.array([3.0, bad_r, 3.0]), spec.U)
        assert e.value.code == psm.PSM_EINVAL and "radius" in str(e.value)
    with pytest.raises(psm.PsmError) as e:
        eng.set_particles(1, spec.x, spec.r, spec.U)
    assert e.value.code == psm.PSM_EINVAL and "out of range" in str(e.value)
    eng.set_particles(0, spec.x, spec.r, spec.U, spec.Om)
    F, T = eng.get_forces(0)
    assert not F.any() and not T.any()
    assert L.psm_get_pdfs(eng.ctx, 0, None) == psm.PSM_EINVAL
    assert L.psm_get_forces(eng.ctx, 0, None, None) == psm.PSM_EINVAL
    assert L.psm_integrate(eng.ctx, 0.0, psm.PSM_EULER) == psm.PSM_EINVAL
    assert L.psm_integrate(eng.ctx, 1.0, 7) == psm.PSM_EINVAL
    assert L.psm_run(eng.ctx, -1, 1.0, psm.PSM_EULER) == psm.PSM_EINVAL
    assert L.psm_set_dynamics(eng.ctx, 0, 0.0, None) == psm.PSM_EINVAL
    assert L.psm_set_dynamics(eng.ctx, 0, float("nan"), None) == psm.PSM_EINVAL
    acc = (ctypes.c_double * 3)(0.0, float("inf"), 0.0)
    assert L.psm_set_dynamics(eng.ctx, 0, 2.0, acc) == psm.PSM_EINVAL
    assert L.psm_set_launch(eng.ctx, 64, 8, 4, 0) == psm.PSM_EINVAL
    assert L.psm_set_launch(eng.ctx, 64, 4, 3, 0) == psm.PSM_EINVAL
    assert L.psm_set_launch(eng.ctx, 64, 4, 4, 8) == psm.PSM_EINVAL
    assert L.psm_autotune(eng.ctx, 0, None, None, None, None, None) == psm.PSM_EINVAL
    # still usable, and still right
    ref = run_oracle(spec, 8)
    f, F, T, B, pid, eng = run_engine(spec, 8, eng=eng)
    assert_pdfs_close(f, ref.f, 1e-12)
    assert_forces_close(F, ref.F, ref.A)
    eng.close()
