"""Seeded synthetic inputs shared by the engine's tests/benchmark and the oracle.

This module holds no arithmetic of the method itself (no equilibrium, no
solid fraction, no collision). It only draws what a simulation is started
from: sphere centres, radii and velocities, and initial velocity fields.

The paper's fluidized-bed geometry and particle data are not available
(Sec. 4.1 describes them; the data set is external), so every workload is
synthetic with the paper's shapes: spheres of 20 cells diameter resolved in
FP64 on ~10^8-cell blocks (Sec. 4, 4.1), solid fractions between the paper's
dilute and dense cases.

Generator: ``numpy.random.default_rng(seed)`` (PCG64). Sphere placement is
random sequential addition (RSA) in a periodic box with a minimum-image
centre distance >= r_i + r_j (non-overlapping spheres).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


def _rsa_equal(L, n, r, rng, gap, batch=512, max_candidates=None):
    """Random sequential addition of n spheres of one radius r: candidates are
    drawn in batches and taken in draw order, each accepted iff it keeps the
    distance 2r + gap (minimum image) to every sphere accepted before it."""
    dmin = 2.0 * r + gap
    ng = np.maximum((L // dmin).astype(int), 1)
    csz = L / ng
    cap = int(np.prod(np.floor(csz / max(2.0 * r, 1.0)) + 1))
    grid = -np.ones((ng[0], ng[1], ng[2], cap), dtype=np.int64)
    fill = np.zeros((ng[0], ng[1], ng[2]), dtype=np.int64)
    xs = np.zeros((n, 3))
    offs = np.array([(a, b, c) for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1)])
    count = 0
    drawn = 0
    max_candidates = max_candidates or 200 * n + 100000
    while count < n and drawn < max_candidates:
        cand = rng.random((batch, 3)) * L
        drawn += batch
        gc = np.minimum((cand // csz).astype(int), ng - 1)
        # conflicts with spheres accepted in earlier batches
        nb = (gc[:, None, :] + offs[None, :, :]) % ng
        idx = grid[nb[..., 0], nb[..., 1], nb[..., 2]].reshape(batch, -1)
        d = cand[:, None, :] - xs[np.maximum(idx, 0)]
        d -= L * np.round(d / L)
        close = ((d * d).sum(-1) < dmin * dmin) & (idx >= 0)
        ok = ~close.any(axis=1)
        # conflicts among the candidates of this batch, resolved in draw order
        dd = cand[:, None, :] - cand[None, :, :]
        dd -= L * np.round(dd / L)
        pair = (dd * dd).sum(-1) < dmin * dmin
        taken = []
        for j in np.nonzero(ok)[0]:
            if count >= n:
                break
            if taken and pair[j, taken].any():
                continue
            k = fill[gc[j, 0], gc[j, 1], gc[j, 2]]
            if k >= cap:
                continue
            grid[gc[j, 0], gc[j, 1], gc[j, 2], k] = count
            fill[gc[j, 0], gc[j, 1], gc[j, 2]] += 1
            xs[count] = cand[j]
            taken.append(j)
            count += 1
    return xs[:count].copy(), np.full(count, r)


def rsa_spheres(dims, radii, rng, max_attempts_per_sphere=20000, gap=0.0):
    """Place spheres of the given radii one after another at uniform random
    centres in [0,L)^3, rejecting any candidate closer than r_i + r_j + gap
    (minimum image) to an accepted sphere. A sphere that finds no place within
    ``max_attempts_per_sphere`` candidates is dropped. Equal radii take the
    batched path (same acceptance rule, candidates drawn 512 at a time).
    Returns (x (n,3), r (n,))."""
    L = np.asarray(dims, dtype=np.float64)
    radii = np.asarray(radii, dtype=np.float64)
    if len(radii) == 0:
        return np.zeros((0, 3)), np.zeros(0)
    if len(radii) > 64 and np.all(radii == radii[0]):
        return _rsa_equal(L, len(radii), float(radii[0]), rng, gap)
    rmax = float(radii.max())
    cell = 2.0 * rmax + gap
    ng = np.maximum((L // cell).astype(int), 1)
    csz = L / ng
    # centres at pairwise distance >= 2 r_min: at most this many per grid cell
    cap = int(np.prod(np.floor(csz / (2.0 * max(radii.min(), 0.5))) + 1))
    grid = -np.ones((ng[0], ng[1], ng[2], cap), dtype=np.int64)
    fill = np.zeros((ng[0], ng[1], ng[2]), dtype=np.int64)
    xs = np.zeros((len(radii), 3))
    rs = np.zeros(len(radii))
    n = 0
    offs = np.array([(a, b, c) for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1)])
    for ri in radii:
        placed = False
        # candidates are drawn in batches; the first acceptable one is taken
        tries = 0
        while tries < max_attempts_per_sphere and not placed:
            batch = min(64, max_attempts_per_sphere - tries)
            cand = rng.random((batch, 3)) * L
            tries += batch
            for c in cand:
                gc = np.minimum((c // csz).astype(int), ng - 1)
                cells = (gc[None, :] + offs) % ng
                idx = grid[cells[:, 0], cells[:, 1], cells[:, 2]].ravel()
                idx = np.unique(idx[idx >= 0])
                if len(idx):
                    d = c[None, :] - xs[idx]
                    d -= L * np.round(d / L)
                    dist2 = (d * d).sum(axis=1)
                    lim = rs[idx] + ri + gap
                    if np.any(dist2 < lim * lim):
                        continue
                k = fill[gc[0], gc[1], gc[2]]
                if k >= cap:
                    continue
                grid[gc[0], gc[1], gc[2], k] = n
                fill[gc[0], gc[1], gc[2]] += 1
                xs[n] = c
                rs[n] = ri
                n += 1
                placed = True
                break
    return xs[:n].copy(), rs[:n].copy()


def jittered_lattice_spheres(dims, n, r, rng):
    """n non-overlapping spheres of radius r for dense packings (where random
    sequential addition slows down near jamming): the coarsest near-cubic
    lattice with at least n sites (else the finest with spacing >= 2r along
    every axis), a seeded choice of n sites, each centre jittered uniformly
    by up to half the gap between neighbouring spheres per axis."""
    L = np.asarray(dims, dtype=np.float64)
    m = int(math.ceil((n * L.min() ** 3 / np.prod(L)) ** (1.0 / 3.0)))
    counts = np.maximum((m * L / L.min()).astype(int), 1)
    while np.prod(counts) < n:
        counts[np.argmin(L / counts)] += 1
    a = L / counts
    if np.any(a < 2.0 * r):
        # the near-cubic lattice is too fine along some axis: take the most
        # sites that keep a spacing of 2r along every axis
        counts = np.floor(L / (2.0 * r)).astype(int)
        if np.prod(counts) < n:
            raise ValueError("solid fraction too high for a jittered lattice")
        a = L / counts
    sites = np.stack(np.meshgrid(*[np.arange(c) for c in counts], indexing="ij"), -1).reshape(-1, 3)
    pick = rng.choice(len(sites), n, replace=False)
    jit = (rng.random((n, 3)) * 2.0 - 1.0) * (a - 2.0 * r) / 2.0
    x = np.mod((sites[pick] + 0.5) * a + jit, L)
    return x, np.full(n, float(r))


def uniform_velocities(rng, n, amp):
    """Each component uniform in [-amp, amp]."""
    return (rng.random((n, 3)) * 2.0 - 1.0) * amp


def taylor_green(dims, amp):
    """2-D Taylor-Green vortex extruded along z, sampled at cell centres
    (i+1/2, j+1/2): u = A sin(kx x) cos(ky y), v = -A (kx/ky) cos(kx x) sin(ky y),
    w = 0, with k = 2 pi / L per axis (divergence free). Returns u [3][N]
    with cell index n = x + nx (y + ny z)."""
    nx, ny, nz = dims
    kx, ky = 2 * math.pi / nx, 2 * math.pi / ny
    x = (np.arange(nx) + 0.5)[None, None, :]
    y = (np.arange(ny) + 0.5)[None, :, None]
    u = np.zeros((3, nz, ny, nx))
    u[0] = amp * np.sin(kx * x) * np.cos(ky * y)
    u[1] = -amp * (kx / ky) * np.cos(kx * x) * np.sin(ky * y)
    return u.reshape(3, -1)


def shear_wave(dims, amp, axis_u=0, axis_k=1):
    """u_axis_u = A sin(2 pi (coord_axis_k + 1/2) / L) (a decaying shear wave)."""
    nx, ny, nz = dims
    L = dims[axis_k]
    coord = np.arange(L) + 0.5
    prof = amp * np.sin(2 * math.pi * coord / L)
    u = np.zeros((3, nz, ny, nx))
    shape = [1, 1, 1]
    shape[2 - axis_k] = L
    u[axis_u] = prof.reshape(shape)
    return u.reshape(3, -1)


@dataclass
class BoxSpec:
    """One box (periodic, or with walls in z) and its particles."""
    dims: tuple
    tau: float
    fext: tuple = (0.0, 0.0, 0.0)
    mapping: int = 0          # 0 linear approximation, 1 sub-division sampling
    nsub: int = 4
    x: np.ndarray = field(default_factory=lambda: np.zeros((0, 3)))
    r: np.ndarray = field(default_factory=lambda: np.zeros(0))
    U: np.ndarray = field(default_factory=lambda: np.zeros((0, 3)))
    Om: np.ndarray = field(default_factory=lambda: np.zeros((0, 3)))
    u0: np.ndarray | None = None   # initial velocity [3][N]; None = rest
    rho0: np.ndarray | None = None
    walls_z: bool = False          # faces at z = 0 and z = nz instead of periodicity
    wall_u: tuple = ((0.0, 0.0, 0.0), (0.0, 0.0, 0.0))   # bottom and top velocity-face velocities
    face_type: tuple = (0, 0)      # 0 velocity face (bounce-back), 1 pressure face (anti-bounce-back)
    face_rho: tuple = (1.0, 1.0)   # pressure-face densities
    walls_x: bool = False          # resting no-slip walls at x = 0 and x = nx
    walls_y: bool = False          # resting no-slip walls at y = 0 and y = ny

    @property
    def N(self):
        return int(self.dims[0]) * int(self.dims[1]) * int(self.dims[2])

    @property
    def n_particles(self):
        return int(len(self.r))


def n_spheres_for_fraction(dims, phi, r):
    vol = float(dims[0]) * dims[1] * dims[2]
    return int(round(phi * vol / (4.0 / 3.0 * math.pi * r ** 3)))


# ---------------------------------------------------------------------------
# Workload recipes: sizes, seeds and distributions of each benchmark and test workload

def parity_32(seed=0):
    """32^3 periodic box, tau 0.6, Taylor-Green amplitude 0.01, 8 spheres of
    radius 4 at seeded positions with velocities in [-0.01, 0.01]^3, fixed,
    4^3 sub-division sampling, FP64. Run 100 steps."""
    rng = np.random.default_rng(seed)
    dims = (32, 32, 32)
    x, r = rsa_spheres(dims, np.full(8, 4.0), rng)
    U = uniform_velocities(rng, len(r), 0.01)
    return BoxSpec(dims=dims, tau=0.6, mapping=1, nsub=4, x=x, r=r, U=U,
                   Om=np.zeros_like(U), u0=taylor_green(dims, 0.01))


def paper_scale(n=512, seed=1, phi=0.10, radius=10.0, tau=0.55, g=1e-6, vamp=0.005):
    """n^3 periodic box (512 at full size), tau 0.55, body force g along +x,
    fluid at rest, spheres of diameter 20 at 10 % solid volume fraction
    (3204 at 512^3) with velocities in [-0.005, 0.005]^3, linear mapping."""
    rng = np.random.default_rng(seed)
    dims = (n, n, n)
    np_ = n_spheres_for_fraction(dims, phi, radius)
    x, r = rsa_spheres(dims, np.full(np_, radius), rng)
    U = uniform_velocities(rng, len(r), vamp)
    return BoxSpec(dims=dims, tau=tau, fext=(g, 0.0, 0.0), mapping=0, x=x, r=r, U=U,
                   Om=np.zeros_like(U), u0=None)


def batched_boxes(nbox=64, seed=3):
    """64 independent periodic cubic boxes: edge in {32,48,64,96,128}, tau in
    [0.55, 1.0], 0-30 spheres of radius 3-8 (RSA drops spheres that do not
    fit), velocities in [-0.01, 0.01]^3, Taylor-Green amplitude 0.01 start,
    no body force, linear mapping."""
    rng = np.random.default_rng(seed)
    edges = np.array([32, 48, 64, 96, 128])
    out = []
    for _ in range(nbox):
        L = int(edges[rng.integers(0, len(edges))])
        tau = float(rng.uniform(0.55, 1.0))
        nb = int(rng.integers(0, 31))
        radii = rng.uniform(3.0, 8.0, size=nb)
        dims = (L, L, L)
        x, r = rsa_spheres(dims, radii, rng, max_attempts_per_sphere=2000)
        U = uniform_velocities(rng, len(r), 0.01)
        out.append(BoxSpec(dims=dims, tau=tau, mapping=0, x=x, r=r, U=U, Om=np.zeros_like(U),
                           u0=taylor_green(dims, 0.01)))
    return out


def dense_moving(n=768, seed=4, phi=0.30, radius=8.0, vamp=0.005):
    """n^3 periodic box (768 at full size), fluid at rest, spheres of
    diameter 16 at 30 % solid volume fraction (63,365 at 768^3) on a seeded
    jittered lattice, velocities in [-0.005, 0.005]^3, tau 0.6, linear mapping."""
    rng = np.random.default_rng(seed)
    dims = (n, n, n)
    np_ = n_spheres_for_fraction(dims, phi, radius)
    x, r = jittered_lattice_spheres(dims, np_, radius, rng)
    U = uniform_velocities(rng, len(r), vamp)
    return BoxSpec(dims=dims, tau=0.6, mapping=0, x=x, r=r, U=U, Om=np.zeros_like(U), u0=None)


def random_small(dims, nparticles, radius_range, seed, tau=0.7, fext=(0.0, 0.0, 0.0),
                 vamp=0.01, omamp=0.0, mapping=0, amp_u=0.01, overlap=False):
    """Small seeded box for parity tests: random velocity field plus a
    Taylor-Green component, random spheres (optionally allowed to overlap),
    random translational and angular velocities."""
    rng = np.random.default_rng(seed)
    radii = rng.uniform(radius_range[0], radius_range[1], size=nparticles)
    if overlap:
        x = rng.random((nparticles, 3)) * np.asarray(dims, dtype=np.float64)
        r = radii
    else:
        x, r = rsa_spheres(dims, radii, rng, max_attempts_per_sphere=4000)
    U = uniform_velocities(rng, len(r), vamp)
    Om = uniform_velocities(rng, len(r), omamp)
    N = int(np.prod(dims))
    u0 = taylor_green(dims, amp_u) + (rng.random((3, N)) * 2 - 1) * (0.2 * amp_u)
    rho0 = 1.0 + (rng.random(N) * 2 - 1) * 1e-3
    return BoxSpec(dims=tuple(int(d) for d in dims), tau=tau, fext=tuple(fext), mapping=mapping,
                   x=x, r=r, U=U, Om=Om, u0=u0, rho0=rho0)


def fluidized_bed(case="dilute", seed=5, tau=0.65, rho_p=1.1, galileo=8.9, re_p=1.0):
    """Synthetic stand-in for the paper's fluidized bed (Sec. 4.1): a
    500 x 200 x 800 box (z vertical) with resting no-slip walls in x and y,
    a velocity inflow at z = 0 and a pressure outflow (density 1) at z = 800,
    FP64, spheres of diameter 20 and density ratio 1.1: 627 (dilute, about
    3.3 % solid) placed by random sequential addition, or 8073 (dense, about
    42 %) on a jittered lattice, every centre at least r + 1 from the walls,
    at rest. The inflow speed follows from the particle Reynolds number
    U d / nu = re_p and the sphere's gravity-minus-buoyancy acceleration from
    the Galileo number sqrt((rho_p - 1) g d^3) / nu = galileo, with
    nu = (tau - 1/2)/3. Returns (spec, density ratio, external acceleration)."""
    rng = np.random.default_rng(seed)
    dims = (500, 200, 800)
    r = 10.0
    L = np.asarray(dims, dtype=np.float64)
    if case == "dilute":
        inner = L - 2.0 * (r + 1.0)
        x, rr = rsa_spheres(tuple(inner), np.full(627, r), rng)
        x = x + (r + 1.0)
    elif case == "dense":
        # lattice centres 1 + (k + 1/2) a with a >= 2r stay r + 1 from the walls
        x, rr = jittered_lattice_spheres(tuple(L - 2.0), 8073, r, rng)
        x = x + 1.0
    else:
        raise ValueError(case)
    nu = (tau - 0.5) / 3.0
    d = 2.0 * r
    u_in = re_p * nu / d
    g = (galileo * nu) ** 2 / ((rho_p - 1.0) * d ** 3)
    accel = (0.0, 0.0, -g * (1.0 - 1.0 / rho_p))
    N = int(np.prod(dims))
    u0 = np.zeros((3, N))
    u0[2] = u_in
    spec = BoxSpec(dims=dims, tau=tau, fext=(0.0, 0.0, 0.0), mapping=0, x=x, r=rr, U=np.zeros_like(x),
                   Om=np.zeros_like(x), u0=u0, walls_z=True, wall_u=((0.0, 0.0, u_in), (0.0, 0.0, 0.0)),
                   face_type=(0, 1), face_rho=(1.0, 1.0), walls_x=True, walls_y=True)
    return spec, rho_p, accel
