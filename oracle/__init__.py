"""Plain FP64 CPU oracle of the PSM-LBM step (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package. The GPU engine never calls it, and the
two share no code: the oracle is ``psm_oracle.c`` plus this thin ctypes
wrapper, written from arXiv 2303.11811:

* Sec. 2.1, eqs. (1)-(8): D3Q19 SRT lattice Boltzmann step with forcing;
* Sec. 2.3, eqs. (17)-(22): partially saturated cells collision, particle
  velocity at the cell centre, hydrodynamic force and torque;
* Sec. 2.3.2, eqs. (25)-(27): linear-approximation solid fraction (and the
  sub-division sampling it is compared with);
* Sec. 2.2.2, eqs. (15)-(16): velocity-Verlet update of the spheres (and the
  explicit Euler update of the moving-particle workload).

The C header comment of ``psm_oracle.c`` lists every reading taken where the
paper is silent. Everything here is FP64.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "psm_oracle.c")
_LIB = os.path.join(_HERE, "libpsm_oracle.so")
# timing build of the same source with OpenMP (the CPU baseline's all-core
# figure); every test uses the plain build
_LIB_OMP = os.path.join(_HERE, "libpsm_oracle_omp.so")

NQ = 19
MAP_LINEAR = 0
MAP_SUBSAMPLE = 1


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no fused multiply-add, plain -O2), and the
    OpenMP timing build of the same source."""
    for lib, extra in ((_LIB, []), (_LIB_OMP, ["-fopenmp"])):
        if force or not os.path.exists(lib) or os.path.getmtime(lib) < os.path.getmtime(_SRC):
            tmp = lib + ".tmp"
            subprocess.check_call(["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fPIC", "-shared", *extra,
                                   "-o", tmp, _SRC, "-lm"])
            os.replace(tmp, lib)
    return _LIB


class _Box(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
                ("tau", ctypes.c_double), ("fext", ctypes.c_double * 3),
                ("mapping", ctypes.c_int), ("nsub", ctypes.c_int), ("walls_z", ctypes.c_int),
                ("uwall", (ctypes.c_double * 3) * 2), ("face_type", ctypes.c_int * 2),
                ("face_rho", ctypes.c_double * 2), ("walls_x", ctypes.c_int), ("walls_y", ctypes.c_int)]


_libs = {}
_D = ctypes.POINTER(ctypes.c_double)
_I = ctypes.POINTER(ctypes.c_int)


def _load(timing_build=False):
    path = _LIB_OMP if timing_build else _LIB
    if path not in _libs:
        if not os.path.exists(path):
            build(force=False)
        lib = ctypes.CDLL(path)
        lib.psmo_threads.argtypes = [ctypes.c_int]
        lib.psmo_threads.restype = ctypes.c_int
        lib.psmo_lattice.argtypes = [_I, _D, _I]
        lib.psmo_Va.argtypes = [ctypes.c_double]
        lib.psmo_Va.restype = ctypes.c_double
        lib.psmo_fr.argtypes = [ctypes.c_double]
        lib.psmo_fr.restype = ctypes.c_double
        bp = ctypes.POINTER(_Box)
        lib.psmo_equilibrium_field.argtypes = [bp, _D, _D, _D]
        lib.psmo_macroscopic.argtypes = [bp, _D, _D, _D]
        lib.psmo_map.argtypes = [bp, ctypes.c_int, _D, _D, _D, _D, _I]
        lib.psmo_map.restype = ctypes.c_longlong
        lib.psmo_map_cell.argtypes = [bp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                      _D, _D, _D, _I, _D, ctypes.POINTER(ctypes.c_longlong)]
        lib.psmo_map_cell.restype = ctypes.c_int
        lib.psmo_collide_cell.argtypes = [bp, ctypes.c_int, ctypes.c_int, ctypes.c_int, _D,
                                          ctypes.c_int, _I, _D, ctypes.c_int, _D, _D, _D, _D, _D]
        lib.psmo_run.argtypes = [bp, ctypes.c_int, ctypes.c_int, _D, _D, _D, _D, _D, _D,
                                 _D, _D, _D, _D, _I]
        lib.psmo_run.restype = ctypes.c_longlong
        lib.psmo_integrate.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double, _D, _D,
                                       _I, _D, _D, _D, _D, _D, _D, _D, _D, ctypes.c_int]
        _libs[path] = lib
    return _libs[path]


def threads(n=0, timing_build=True) -> int:
    """Set (n > 0) and return the thread count of the collide-and-stream loop
    of the timing build; the plain build always reports 1."""
    return int(_load(timing_build).psmo_threads(int(n)))


def _dp(a):
    return None if a is None else a.ctypes.data_as(_D)


def _ip(a):
    return None if a is None else a.ctypes.data_as(_I)


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


FACE_VELOCITY = 0
FACE_PRESSURE = 1


class Box:
    """A box, periodic in x and y unless walls_x / walls_y put resting
    no-slip walls at -1/2 and n - 1/2 (cell-index coordinates); in z
    periodic, or bounded by faces at z = -1/2 and z = nz - 1/2: velocity
    faces (half-way bounce-back moving with wall_u) or pressure faces
    (anti-bounce-back to density face_rho), bottom first."""

    def __init__(self, nx, ny, nz, tau, fext=(0.0, 0.0, 0.0), mapping=MAP_LINEAR, nsub=4,
                 walls_z=False, wall_u=((0.0, 0.0, 0.0), (0.0, 0.0, 0.0)),
                 face_type=(FACE_VELOCITY, FACE_VELOCITY), face_rho=(1.0, 1.0), walls_x=False, walls_y=False):
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self.tau = float(tau)
        self.fext = tuple(float(v) for v in fext)
        self.mapping = int(mapping)
        self.nsub = int(nsub)
        self.walls_z = bool(walls_z)
        self.wall_u = tuple(tuple(float(v) for v in w) for w in wall_u)
        self.face_type = tuple(int(t) for t in face_type)
        self.face_rho = tuple(float(v) for v in face_rho)
        self.walls_x, self.walls_y = bool(walls_x), bool(walls_y)

    @property
    def N(self):
        return self.nx * self.ny * self.nz

    def _c(self):
        b = _Box()
        b.nx, b.ny, b.nz = self.nx, self.ny, self.nz
        b.tau = self.tau
        for a in range(3):
            b.fext[a] = self.fext[a]
        b.mapping, b.nsub, b.walls_z = self.mapping, self.nsub, int(self.walls_z)
        for w in range(2):
            for a in range(3):
                b.uwall[w][a] = self.wall_u[w][a]
            b.face_type[w] = self.face_type[w]
            b.face_rho[w] = self.face_rho[w]
        b.walls_x, b.walls_y = int(self.walls_x), int(self.walls_y)
        return b


def lattice():
    """(c [19,3] int, w [19] float, qbar [19] int) as the oracle defines them."""
    lib = _load()
    c = np.zeros(57, dtype=np.int32)
    w = np.zeros(19)
    qb = np.zeros(19, dtype=np.int32)
    lib.psmo_lattice(_ip(c), _dp(w), _ip(qb))
    return c.reshape(19, 3), w, qb


def Va(r: float) -> float:
    return _load().psmo_Va(float(r))


def fr(r) -> np.ndarray:
    lib = _load()
    r = np.atleast_1d(np.asarray(r, dtype=np.float64))
    return np.array([lib.psmo_fr(float(v)) for v in r])


def equilibrium(box: Box, u, rho=None) -> np.ndarray:
    """f_q = E_q(rho, u) on the whole box. u: [3][N] (or (3,nz,ny,nx))."""
    u = _f64(u, (3, box.N))
    rho = None if rho is None else _f64(rho, (box.N,))
    f = np.empty((NQ, box.N))
    bc = box._c()
    _load().psmo_equilibrium_field(ctypes.byref(bc), _dp(rho), _dp(u), _dp(f))
    return f


def macroscopic(box: Box, f):
    f = _f64(f, (NQ, box.N))
    rho = np.empty(box.N)
    u = np.empty((3, box.N))
    bc = box._c()
    _load().psmo_macroscopic(ctypes.byref(bc), _dp(f), _dp(rho), _dp(u))
    return rho, u


def solid_map(box: Box, x, r, frv=None):
    """Two-slot solid fractions: B [2][N], pid [2][N] (-1 empty), overflow count."""
    x = _f64(x, (-1, 3))
    r = _f64(r, (-1,))
    frv = fr(r) if frv is None else _f64(frv, (-1,))
    B = np.zeros((2, box.N))
    pid = np.zeros((2, box.N), dtype=np.int32)
    bc = box._c()
    ov = _load().psmo_map(ctypes.byref(bc), len(r), _dp(x), _dp(r), _dp(frv), _dp(B), _ip(pid))
    return B, pid, int(ov)


def map_cell(box: Box, i, j, k, x, r, frv=None):
    """Slots of one cell by brute force over all particles."""
    x = _f64(x, (-1, 3))
    r = _f64(r, (-1,))
    frv = fr(r) if frv is None else _f64(frv, (-1,))
    pid = np.zeros(2, dtype=np.int32)
    B = np.zeros(2)
    ov = ctypes.c_longlong(0)
    bc = box._c()
    ns = _load().psmo_map_cell(ctypes.byref(bc), int(i), int(j), int(k), len(r), _dp(x), _dp(r),
                               _dp(frv), _ip(pid), _dp(B), ctypes.byref(ov))
    return int(ns), pid, B, int(ov.value)


def collide_cell(box: Box, i, j, k, f19, pid, B, x, U, Om):
    """Post-collision PDFs of one cell and per-slot sum_q C^solid c_qbar."""
    f19 = _f64(f19, (NQ,))
    pid = np.ascontiguousarray(pid, dtype=np.int32)
    B = _f64(B)
    ns = int(len(pid))
    x = _f64(x, (-1, 3))
    U = _f64(U, (-1, 3))
    Om = _f64(Om, (-1, 3))
    ft = np.empty(NQ)
    g = np.zeros((max(ns, 1), 3))
    bc = box._c()
    _load().psmo_collide_cell(ctypes.byref(bc), int(i), int(j), int(k), _dp(f19), ns, _ip(pid),
                              _dp(B), len(x), _dp(x), _dp(U), _dp(Om), _dp(ft), _dp(g))
    return ft, g[:ns]


class Result:
    __slots__ = ("f", "F", "T", "A", "B", "pid", "overflow")


def run(box: Box, f0, nsteps, x=None, r=None, U=None, Om=None, frv=None, timing_build=False) -> Result:
    """Advance f0 ([19][N], pre-collision) by nsteps. Returns the new field and
    the last step's force, torque, force scale, slots and overflow count.
    timing_build: run the OpenMP build (same arithmetic per cell; force and
    torque summed per thread, then over threads in order)."""
    f = _f64(f0, (NQ, box.N)).copy()
    if x is None or len(np.atleast_1d(r)) == 0:
        x = np.zeros((0, 3)); r = np.zeros(0); U = np.zeros((0, 3)); Om = np.zeros((0, 3))
    x = _f64(x, (-1, 3))
    r = _f64(r, (-1,))
    np_ = len(r)
    U = np.zeros((np_, 3)) if U is None else _f64(U, (-1, 3))
    Om = np.zeros((np_, 3)) if Om is None else _f64(Om, (-1, 3))
    frv = fr(r) if (frv is None and np_) else (np.zeros(0) if frv is None else _f64(frv, (-1,)))
    res = Result()
    res.F = np.zeros((np_, 3))
    res.T = np.zeros((np_, 3))
    res.A = np.zeros(np_)
    res.B = np.zeros((2, box.N))
    res.pid = np.zeros((2, box.N), dtype=np.int32)
    bc = box._c()
    res.overflow = int(_load(timing_build).psmo_run(ctypes.byref(bc), int(nsteps), np_, _dp(x), _dp(r),
                                        _dp(frv), _dp(U), _dp(Om), _dp(f), _dp(res.F),
                                        _dp(res.T), _dp(res.A), _dp(res.B), _ip(res.pid)))
    res.f = f
    return res


EULER = 0
VERLET = 1


class Dynamics:
    """Particle state of the integrator: positions x, velocities U, angular
    velocities Om (n,3) and, for velocity Verlet, the previous total force
    and torque."""

    def __init__(self, x, r, U, Om):
        self.x = _f64(x, (-1, 3)).copy()
        self.r = _f64(r, (-1,)).copy()
        self.U = _f64(U, (-1, 3)).copy()
        self.Om = _f64(Om, (-1, 3)).copy()
        self.Fprev = np.zeros_like(self.x)
        self.Tprev = np.zeros_like(self.x)
        self.have_prev = False


def integrate(box: Box, dyn: Dynamics, F, T, dt=1.0, scheme=VERLET, rho_p=1.0, accel=(0.0, 0.0, 0.0)):
    """One particle update of dyn in place from the hydrodynamic force and
    torque F, T (n,3) of the fluid step just done (psmo_integrate)."""
    F = _f64(F, (-1, 3))
    T = _f64(T, (-1, 3))
    L = np.array([box.nx, box.ny, box.nz], dtype=np.float64)
    walls = np.array([box.walls_x, box.walls_y, box.walls_z], dtype=np.int32)
    a = _f64(accel, (3,))
    _load().psmo_integrate(len(dyn.r), int(scheme), float(dt), float(rho_p), _dp(a), _dp(L), _ip(walls), _dp(dyn.r),
                           _dp(dyn.x), _dp(dyn.U), _dp(dyn.Om), _dp(F), _dp(T), _dp(dyn.Fprev),
                           _dp(dyn.Tprev), int(dyn.have_prev))
    if scheme == VERLET:
        dyn.have_prev = True
