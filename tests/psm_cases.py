"""Shared drivers for the GPU parity tests: run a seeded box on the oracle and
on the engine (through the C ABI) and compare with stated tolerances."""
from __future__ import annotations

import numpy as np

import oracle
import paper_2303_11811_amd as psm


def oracle_box(spec):
    return oracle.Box(*spec.dims, tau=spec.tau, fext=spec.fext, mapping=spec.mapping, nsub=spec.nsub,
                      walls_z=spec.walls_z, wall_u=spec.wall_u, face_type=spec.face_type, face_rho=spec.face_rho,
                      walls_x=spec.walls_x, walls_y=spec.walls_y)


def initial_f(spec):
    """Oracle equilibrium start f = E(rho0, u0) (eq. 5)."""
    box = oracle_box(spec)
    u0 = np.zeros((3, spec.N)) if spec.u0 is None else spec.u0
    return oracle.equilibrium(box, u0, spec.rho0)


def run_oracle(spec, steps, f0=None):
    box = oracle_box(spec)
    f0 = initial_f(spec) if f0 is None else f0
    return oracle.run(box, f0, steps, spec.x, spec.r, spec.U, spec.Om)


def make_engine(specs, storage=psm.PSM_FP64, fp16_scale=0.0, max_particles=None, max_radius=None):
    descs = [psm.desc_from_spec(s, max_particles=max_particles, max_radius=max_radius) for s in specs]
    return psm.Engine(descs, storage=storage, fp16_scale=fp16_scale)


def run_engine(spec, steps, storage=psm.PSM_FP64, launch=None, graph=False, f0=None, eng=None,
               fp16_scale=0.0):
    """Run one box on the GPU from the oracle's initial PDFs. Returns the
    canonical PDFs, forces, torques, slots and the engine."""
    if eng is None:
        eng = make_engine([spec], storage=storage, fp16_scale=fp16_scale)
    if launch is not None:
        eng.set_launch(*launch)
    eng.set_graph(graph)
    f0 = initial_f(spec) if f0 is None else f0
    eng.set_pdfs(0, f0)
    if spec.n_particles:
        eng.set_particles(0, spec.x, spec.r, spec.U, spec.Om)
    eng.step(steps)
    f = eng.get_pdfs(0).cpu().numpy()
    F, T = eng.get_forces(0)
    B, pid = eng.get_solid_fraction(0)
    eng.synchronize()
    return f, F, T, B.cpu().numpy(), pid.cpu().numpy(), eng


def assert_pdfs_close(f_gpu, f_ref, rtol):
    err = np.abs(f_gpu - f_ref)
    bound = rtol * np.abs(f_ref) + rtol * 1e-3
    bad = err > bound
    assert not bad.any(), (f"{int(bad.sum())} PDFs off; max abs err {err.max():.3e}, "
                           f"max rel {(err / np.maximum(np.abs(f_ref), 1e-300)).max():.3e}")


def assert_forces_close(F_gpu, F_ref, A, lever=1.0, rtol=1e-12, atol_scale=1e-14):
    """|dF_p| <= rtol |F_p| + atol_scale * A_p (A_p: sum over the sphere's cells
    of B |g|, the magnitude the terms of the sum carry)."""
    d = np.linalg.norm(F_gpu - F_ref, axis=1)
    bound = rtol * np.linalg.norm(F_ref, axis=1) + atol_scale * A * lever + 1e-300
    assert np.all(d <= bound), f"max excess {np.max(d / bound):.3g}"


CX = np.array([0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0])
CY = np.array([0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1])
CZ = np.array([0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1])
W = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)


def sample_cells(spec, x, r, rng, n_surface=32, n_random=32):
    """Cells near sphere surfaces (where the PSM terms act) plus random cells."""
    dims = np.asarray(spec.dims)
    cells = []
    if len(r):
        for p in rng.integers(0, len(r), n_surface):
            d = rng.normal(size=3)
            d *= (r[p] + rng.uniform(-1.5, 0.8)) / np.linalg.norm(d)
            cells.append(tuple((np.floor(x[p] + d).astype(int)) % dims))
    cells += [tuple(v) for v in rng.integers(0, dims, (n_random, 3))]
    return cells


def _idx(c, dims):
    return int(c[0] % dims[0] + dims[0] * ((c[1] % dims[1]) + dims[1] * (c[2] % dims[2])))


def gather_sources(eng, box, spec, cells):
    """The engine's f(t) at the 19 source cells x - c_q of every sampled cell."""
    dims = spec.dims
    flat = [(i - CX[q], j - CY[q], k - CZ[q]) for (i, j, k) in cells for q in range(19)]
    f_t = eng.get_pdfs_at(box, [_idx(t, dims) for t in flat]).cpu().numpy()
    return flat, f_t


def oracle_after(eng, box, spec, cells, flat, f_t, x, r, U, Om):
    """After one engine step: the engine's f(x, t+1) at the sampled cells and
    the oracle's value computed in FP64 from the engine's f(t) at the sources
    (map_cell over all spheres, collide_cell): arrays (ncells, 19) each."""
    dims = spec.dims
    got = eng.get_pdfs_at(box, [_idx(c, dims) for c in cells]).cpu().numpy().T.copy()
    ob = oracle.Box(*dims, tau=spec.tau, fext=spec.fext, mapping=spec.mapping, nsub=spec.nsub)
    frv = oracle.fr(r) if len(r) else np.zeros(0)
    ref = np.zeros((len(cells), 19))
    for a in range(len(cells)):
        for q in range(19):
            t = flat[a * 19 + q]
            si, sj, sk = t[0] % dims[0], t[1] % dims[1], t[2] % dims[2]
            ns, pid, B, _ = oracle.map_cell(ob, si, sj, sk, x, r, frv)
            ft, _ = oracle.collide_cell(ob, si, sj, sk, f_t[:, a * 19 + q], pid[:ns], B[:ns], x, U, Om)
            ref[a, q] = ft[q]
    return got, ref


def one_step_sampled(eng, box, spec, cells, x, r, U, Om):
    """gather_sources, one engine step, oracle_after."""
    flat, f_t = gather_sources(eng, box, spec, cells)
    eng.step(1)
    return oracle_after(eng, box, spec, cells, flat, f_t, x, r, U, Om)


def deviation_bound(ref, storage):
    """Per-value bound for one step computed in FP32 from the same state:
    the rounding of the stored output (FP32: 2^-24 relative; FP16 keeps
    2^10 d: 2^-11 relative, 2^-35 absolute below the normal range) plus
    sixteen FP32 roundings at the largest deviation of the cell
    (16 x 2^-24 < 1e-6)."""
    d = np.abs(ref - W[None, :])
    cell_max = d.max(axis=1, keepdims=True)
    if storage == psm.PSM_FP16DEV:
        out = 2.0 ** -11 * d + 2.0 ** -35
    else:
        out = 2.0 ** -24 * d
    return out + 1e-6 * cell_max


def bench_launch(storage):
    """The launch bench.py times the 512^3 workload at in this storage form:
    that of the committed counter run while it matches the kernel source,
    else None (bench.py then runs the autotuner)."""
    import os
    import sys

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if root not in sys.path:
        sys.path.insert(0, root)
    import bench

    _, launch = bench.measured_traffic(storage)
    return tuple(launch) if launch else None


def post_collision_field(box, f, x, r, U, Om):
    """The oracle's post-collision values f~ [19][N] of every cell of state f
    (its own slots and collision, cell by cell)."""
    B, pid, _ = oracle.solid_map(box, x, r) if len(r) else (np.zeros((2, box.N)), -np.ones((2, box.N), int), 0)
    ft = np.empty_like(f)
    nx, ny = box.nx, box.ny
    for n in range(box.N):
        i, j, k = n % nx, (n // nx) % ny, n // (nx * ny)
        ns = int((pid[:, n] >= 0).sum())
        ft[:, n], _ = oracle.collide_cell(box, i, j, k, f[:, n], pid[:ns, n], B[:ns, n], x, U, Om)
    return ft


def one_step_bound(spec, storage, f_t, ft):
    """Per-value bound [19][N] for one step of a deviation form from the
    canonical state f_t, with ft the oracle's post-collision field of f_t.
    Each canonical value after the step comes from one stored post-collision
    value: f~_q(x - c_q) for a plain pull, f~_qbar(x) for a population that
    enters through a wall or face (the wall or face term is added exactly on
    read-out). The bound is the storage rounding of that stored value (FP32:
    2^-24 relative; FP16 keeps 2^10 d: 2^-11 relative, 2^-35 absolute below
    the normal range) plus sixteen FP32 roundings at the largest deviation
    of the computing cell before or after its collision (16 x 2^-24 < 1e-6)."""
    nx, ny, nz = spec.dims
    n = np.arange(nx * ny * nz)
    i, j, k = n % nx, (n // nx) % ny, n // (nx * ny)
    dt = np.abs(ft - W[:, None])
    scale = np.maximum(dt.max(axis=0), np.abs(f_t - W[:, None]).max(axis=0))
    walled = (getattr(spec, "walls_x", False), getattr(spec, "walls_y", False), getattr(spec, "walls_z", False))
    out = np.empty_like(ft)
    opp = np.array([0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17])
    for q in range(19):
        si, sj, sk = i - CX[q], j - CY[q], k - CZ[q]
        through = np.zeros(len(n), bool)
        for a, (sv, L) in enumerate(((si, nx), (sj, ny), (sk, nz))):
            if walled[a]:
                through |= (sv < 0) | (sv >= L)
        src = (si % nx) + nx * ((sj % ny) + ny * (sk % nz))
        d_src = np.where(through, dt[opp[q], n], dt[q, src])
        c_src = np.where(through, scale[n], scale[src])
        rel, ab = (2.0 ** -11, 2.0 ** -35) if storage == psm.PSM_FP16DEV else (2.0 ** -24, 0.0)
        out[q] = rel * d_src + ab + 1e-6 * c_src
    return out

