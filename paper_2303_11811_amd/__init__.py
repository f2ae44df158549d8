"""MI355X (gfx950) engine for the PSM-LBM hot path of arXiv 2303.11811.

Thin ctypes binding of ``libpsm.so`` (C ABI in ``include/psm.h``): every
function below has the name of the C call it marshals, and all computation
happens in the library's HIP kernels. PyTorch is used only by :class:`Engine`
for device memory (the workspace and I/O tensors) and the HIP stream.

Importing this package does not need a GPU; the library is loaded on first
use and a missing library raises ``RuntimeError`` (there is no fallback).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpsm.so")

PSM_OK, PSM_EINVAL, PSM_EHIP, PSM_ECAPACITY, PSM_ENONFINITE, PSM_EDRIFT, PSM_ESTATE = 0, -1, -2, -3, -4, -5, -6
PSM_FP64, PSM_FP32DEV, PSM_FP16DEV = 0, 1, 2
PSM_MAP_LINEAR, PSM_MAP_SUBSAMPLE = 0, 1
PSM_LAUNCH_PERSISTENT, PSM_LAUNCH_FILTER = 1, 2
PSM_EULER, PSM_VERLET = 0, 1
PSM_FACE_VELOCITY, PSM_FACE_PRESSURE = 0, 1
STORAGE = {"f64": PSM_FP64, "f32dev": PSM_FP32DEV, "f16dev": PSM_FP16DEV}


class PsmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"psm error {code}: {msg}")
        self.code = code


class psm_box_desc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
                ("tau", ctypes.c_double), ("fext", ctypes.c_double * 3),
                ("max_particles", ctypes.c_int), ("max_radius", ctypes.c_double),
                ("mapping", ctypes.c_int), ("subsample_n", ctypes.c_int),
                ("walls_z", ctypes.c_int), ("wall_u", (ctypes.c_double * 3) * 2),
                ("face_type", ctypes.c_int * 2), ("face_rho", ctypes.c_double * 2),
                ("walls_x", ctypes.c_int), ("walls_y", ctypes.c_int)]


_lib = None
_P = ctypes.c_void_p
_D = ctypes.POINTER(ctypes.c_double)
_SIGS = {
    "psm_workspace_size": ([ctypes.POINTER(psm_box_desc), ctypes.c_int, ctypes.c_int,
                            ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "psm_create": ([ctypes.POINTER(psm_box_desc), ctypes.c_int, ctypes.c_int, ctypes.c_double, _P, _P,
                    ctypes.c_size_t, ctypes.POINTER(_P)], ctypes.c_int),
    "psm_destroy": ([_P], ctypes.c_int),
    "psm_set_equilibrium": ([_P, ctypes.c_int, _P, _P], ctypes.c_int),
    "psm_set_pdfs": ([_P, ctypes.c_int, _P], ctypes.c_int),
    "psm_get_pdfs": ([_P, ctypes.c_int, _P], ctypes.c_int),
    "psm_get_pdfs_at": ([_P, ctypes.c_int, ctypes.c_int, _P, _P], ctypes.c_int),
    "psm_get_macroscopic": ([_P, ctypes.c_int, _P, _P], ctypes.c_int),
    "psm_set_particles": ([_P, ctypes.c_int, ctypes.c_int, _D, _D, _D, _D], ctypes.c_int),
    "psm_set_particle_positions": ([_P, ctypes.c_int, ctypes.c_int, _D], ctypes.c_int),
    "psm_set_particle_velocities": ([_P, ctypes.c_int, ctypes.c_int, _D, _D], ctypes.c_int),
    "psm_step": ([_P, ctypes.c_int], ctypes.c_int),
    "psm_get_forces": ([_P, ctypes.c_int, _D, _D], ctypes.c_int),
    "psm_get_solid_fraction": ([_P, ctypes.c_int, _P, _P], ctypes.c_int),
    "psm_get_stats": ([_P, ctypes.c_int, _D, _D, ctypes.POINTER(ctypes.c_longlong)], ctypes.c_int),
    "psm_set_drift_check": ([_P, ctypes.c_int, ctypes.c_double], ctypes.c_int),
    "psm_set_strict_slots": ([_P, ctypes.c_int], ctypes.c_int),
    "psm_set_force_readback": ([_P, ctypes.c_int], ctypes.c_int),
    "psm_set_launch": ([_P, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int], ctypes.c_int),
    "psm_get_launch": ([_P, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                        ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)], ctypes.c_int),
    "psm_autotune": ([_P, ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                      ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int), _D], ctypes.c_int),
    "psm_clear_tune_cache": ([], ctypes.c_int),
    "psm_set_graph": ([_P, ctypes.c_int], ctypes.c_int),
    "psm_set_timing": ([_P, ctypes.c_int], ctypes.c_int),
    "psm_get_timing": ([_P, ctypes.POINTER(ctypes.c_longlong), _D], ctypes.c_int),
    "psm_reset_timing": ([_P], ctypes.c_int),
    "psm_pattern_copy": ([_P, ctypes.c_int, ctypes.c_int, _D], ctypes.c_int),
    "psm_set_dynamics": ([_P, ctypes.c_int, ctypes.c_double, _D], ctypes.c_int),
    "psm_integrate": ([_P, ctypes.c_double, ctypes.c_int], ctypes.c_int),
    "psm_get_particles": ([_P, ctypes.c_int, _D, _D, _D], ctypes.c_int),
    "psm_run": ([_P, ctypes.c_int, ctypes.c_double, ctypes.c_int], ctypes.c_int),
    "psm_stream_copy": ([_P, _P, ctypes.c_size_t, _P], ctypes.c_int),
    "psm_field_stats_noalloc": ([_P, ctypes.c_longlong, _P, _P], ctypes.c_int),
    "psm_last_error": ([], ctypes.c_char_p),
}


def lib():
    """The loaded ``libpsm.so`` (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2303_11811_amd.build` (no fallback path exists)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def psm_last_error() -> str:
    return lib().psm_last_error().decode()


def _check(rc):
    if rc != PSM_OK:
        raise PsmError(rc, psm_last_error())
    return rc


def _dptr(a):
    return None if a is None else a.ctypes.data_as(_D)


def make_desc(nx, ny, nz, tau, fext=(0.0, 0.0, 0.0), max_particles=0, max_radius=1.0,
              mapping=PSM_MAP_LINEAR, subsample_n=4, walls_z=False,
              wall_u=((0.0, 0.0, 0.0), (0.0, 0.0, 0.0)), face_type=(PSM_FACE_VELOCITY, PSM_FACE_VELOCITY),
              face_rho=(1.0, 1.0), walls_x=False, walls_y=False) -> psm_box_desc:
    d = psm_box_desc()
    d.nx, d.ny, d.nz = int(nx), int(ny), int(nz)
    d.tau = float(tau)
    for a in range(3):
        d.fext[a] = float(fext[a])
    d.max_particles = int(max_particles)
    d.max_radius = float(max_radius)
    d.mapping = int(mapping)
    d.subsample_n = int(subsample_n)
    d.walls_z = int(bool(walls_z))
    for w in range(2):
        for a in range(3):
            d.wall_u[w][a] = float(wall_u[w][a])
        d.face_type[w] = int(face_type[w])
        d.face_rho[w] = float(face_rho[w])
    d.walls_x, d.walls_y = int(bool(walls_x)), int(bool(walls_y))
    return d


def _desc_array(descs):
    arr = (psm_box_desc * len(descs))()
    for i, d in enumerate(descs):
        arr[i] = d
    return arr


# --- same-name wrappers of the C ABI (argument marshalling only) -----------

def psm_workspace_size(descs, storage) -> int:
    arr = _desc_array(descs)
    out = ctypes.c_size_t(0)
    _check(lib().psm_workspace_size(arr, len(descs), int(storage), ctypes.byref(out)))
    return int(out.value)


def psm_create(descs, storage, fp16_scale, stream, workspace_ptr, workspace_bytes):
    arr = _desc_array(descs)
    ctx = _P()
    _check(lib().psm_create(arr, len(descs), int(storage), float(fp16_scale), _P(stream),
                            _P(workspace_ptr), ctypes.c_size_t(workspace_bytes), ctypes.byref(ctx)))
    return ctx


def psm_destroy(ctx):
    return _check(lib().psm_destroy(ctx))


def psm_set_equilibrium(ctx, box, rho_ptr, u_ptr):
    return _check(lib().psm_set_equilibrium(ctx, box, _P(rho_ptr), _P(u_ptr)))


def psm_set_pdfs(ctx, box, f_ptr):
    return _check(lib().psm_set_pdfs(ctx, box, _P(f_ptr)))


def psm_get_pdfs(ctx, box, f_ptr):
    return _check(lib().psm_get_pdfs(ctx, box, _P(f_ptr)))


def psm_get_pdfs_at(ctx, box, ncells, cells_ptr, out_ptr):
    return _check(lib().psm_get_pdfs_at(ctx, box, int(ncells), _P(cells_ptr), _P(out_ptr)))


def psm_get_macroscopic(ctx, box, rho_ptr, u_ptr):
    return _check(lib().psm_get_macroscopic(ctx, box, _P(rho_ptr), _P(u_ptr)))


def psm_set_particles(ctx, box, x, r, U, omega=None):
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, 3)
    r = np.ascontiguousarray(r, dtype=np.float64).reshape(-1)
    U = np.ascontiguousarray(U, dtype=np.float64).reshape(-1, 3)
    om = None if omega is None else np.ascontiguousarray(omega, dtype=np.float64).reshape(-1, 3)
    return _check(lib().psm_set_particles(ctx, box, len(r), _dptr(x), _dptr(r), _dptr(U), _dptr(om)))


def psm_set_particle_positions(ctx, box, x):
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, 3)
    return _check(lib().psm_set_particle_positions(ctx, box, len(x), _dptr(x)))


def psm_set_particle_velocities(ctx, box, U, omega=None):
    U = np.ascontiguousarray(U, dtype=np.float64).reshape(-1, 3)
    om = None if omega is None else np.ascontiguousarray(omega, dtype=np.float64).reshape(-1, 3)
    return _check(lib().psm_set_particle_velocities(ctx, box, len(U), _dptr(U), _dptr(om)))


def psm_step(ctx, nsteps):
    return _check(lib().psm_step(ctx, int(nsteps)))


def psm_get_forces(ctx, box, n, F=None, T=None):
    """F, T (n, 3) FP64; caller arrays of that shape (C-contiguous FP64) are
    filled in place when given."""
    F = np.empty((n, 3)) if F is None else F
    T = np.empty((n, 3)) if T is None else T
    for a in (F, T):
        if a.shape != (n, 3) or a.dtype != np.float64 or not a.flags.c_contiguous:
            raise ValueError(f"force arrays must be C-contiguous float64 of shape ({n}, 3)")
    _check(lib().psm_get_forces(ctx, box, _dptr(F), _dptr(T)))
    return F, T


def psm_set_dynamics(ctx, box, density_ratio, accel=None):
    a = None if accel is None else np.ascontiguousarray(accel, dtype=np.float64).reshape(3)
    return _check(lib().psm_set_dynamics(ctx, box, float(density_ratio), _dptr(a)))


def psm_integrate(ctx, dt, scheme):
    return _check(lib().psm_integrate(ctx, float(dt), int(scheme)))


def psm_run(ctx, nsteps, dt, scheme):
    return _check(lib().psm_run(ctx, int(nsteps), float(dt), int(scheme)))


def psm_get_particles(ctx, box, n):
    x, U, Om = np.zeros((n, 3)), np.zeros((n, 3)), np.zeros((n, 3))
    _check(lib().psm_get_particles(ctx, box, _dptr(x), _dptr(U), _dptr(Om)))
    return x, U, Om


def psm_get_solid_fraction(ctx, box, B_ptr, pid_ptr):
    return _check(lib().psm_get_solid_fraction(ctx, box, _P(B_ptr), _P(pid_ptr)))


def psm_get_stats(ctx, box):
    mass = ctypes.c_double(0)
    mom = np.zeros(3)
    ov = ctypes.c_longlong(0)
    _check(lib().psm_get_stats(ctx, box, ctypes.byref(mass), _dptr(mom), ctypes.byref(ov)))
    return mass.value, mom, int(ov.value)


def psm_set_drift_check(ctx, box, rel_tol):
    return _check(lib().psm_set_drift_check(ctx, box, float(rel_tol)))


def psm_set_strict_slots(ctx, enable):
    return _check(lib().psm_set_strict_slots(ctx, int(bool(enable))))


def psm_set_force_readback(ctx, enable):
    return _check(lib().psm_set_force_readback(ctx, int(bool(enable))))


def psm_set_launch(ctx, tx, ty, tz, flags=0):
    return _check(lib().psm_set_launch(ctx, int(tx), int(ty), int(tz), int(flags)))


def psm_get_launch(ctx):
    a, b, c, d = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    _check(lib().psm_get_launch(ctx, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c), ctypes.byref(d)))
    return a.value, b.value, c.value, d.value


def psm_autotune(ctx, trial_steps):
    a, b, c, d = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    ms = ctypes.c_double()
    _check(lib().psm_autotune(ctx, int(trial_steps), ctypes.byref(a), ctypes.byref(b), ctypes.byref(c),
                              ctypes.byref(d), ctypes.byref(ms)))
    return (a.value, b.value, c.value, d.value), ms.value


def psm_clear_tune_cache():
    return _check(lib().psm_clear_tune_cache())


def psm_set_graph(ctx, enable):
    return _check(lib().psm_set_graph(ctx, int(bool(enable))))


def psm_set_timing(ctx, enable):
    return _check(lib().psm_set_timing(ctx, int(bool(enable))))


def psm_pattern_copy(ctx, shifted, nrep):
    ms = ctypes.c_double(0)
    _check(lib().psm_pattern_copy(ctx, int(shifted), int(nrep), ctypes.byref(ms)))
    return ms.value


def psm_get_timing(ctx):
    n = ctypes.c_longlong(0)
    ms = ctypes.c_double(0)
    _check(lib().psm_get_timing(ctx, ctypes.byref(n), ctypes.byref(ms)))
    return int(n.value), ms.value


def psm_reset_timing(ctx):
    return _check(lib().psm_reset_timing(ctx))


def psm_field_stats_noalloc(f_ptr, ncells, out_ptr, stream):
    return _check(lib().psm_field_stats_noalloc(_P(f_ptr), ctypes.c_longlong(ncells), _P(out_ptr), _P(stream)))


def psm_stream_copy(src_ptr, dst_ptr, nbytes, stream):
    return _check(lib().psm_stream_copy(_P(src_ptr), _P(dst_ptr), ctypes.c_size_t(nbytes), _P(stream)))


# --- convenience owner of device memory (torch) -----------------------------

class Engine:
    """A context over one or more periodic boxes, with its workspace and I/O
    buffers held as torch tensors on ``device``; the library and every torch
    operation of the engine run on one HIP stream of the engine's own."""

    def __init__(self, descs, storage=PSM_FP64, fp16_scale=0.0, device="cuda:0"):
        import torch

        self.torch = torch
        self.device = torch.device(device)
        self.descs = list(descs)
        self.storage = int(storage)
        # a stream of its own (default priority): graph capture needs a
        # non-legacy stream, and every torch op of this engine runs on it
        self.stream = torch.cuda.Stream(self.device)
        nbytes = psm_workspace_size(self.descs, self.storage)
        with torch.cuda.stream(self.stream):
            self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.ctx = psm_create(self.descs, self.storage, fp16_scale, self.stream.cuda_stream,
                              self.workspace.data_ptr(), nbytes)
        self.np = [0] * len(self.descs)

    def N(self, box=0):
        d = self.descs[box]
        return d.nx * d.ny * d.nz

    def close(self):
        if getattr(self, "ctx", None) is not None:
            psm_destroy(self.ctx)   # waits for the stream
            self.ctx = None
        self.workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _enter(self):
        """Order the engine stream after the caller's current stream."""
        self.stream.wait_stream(self.torch.cuda.current_stream(self.device))
        return self.torch.cuda.stream(self.stream)

    def _hand_back(self, *tensors):
        """Order the caller's current stream after the engine stream."""
        cur = self.torch.cuda.current_stream(self.device)
        cur.wait_stream(self.stream)
        for t in tensors:
            t.record_stream(cur)
        return tensors if len(tensors) > 1 else tensors[0]

    def _dev(self, a, dtype=None):
        t = self.torch
        if isinstance(a, t.Tensor):
            return a.to(device=self.device, dtype=dtype or a.dtype).contiguous()
        return t.as_tensor(np.ascontiguousarray(a), device=self.device, dtype=dtype)

    def set_equilibrium(self, box, u, rho=None):
        with self._enter():
            u_d = self._dev(u, self.torch.float64).reshape(3, -1)
            rho_d = None if rho is None else self._dev(rho, self.torch.float64).reshape(-1)
            psm_set_equilibrium(self.ctx, box, None if rho_d is None else rho_d.data_ptr(), u_d.data_ptr())
            self._keep = (u_d, rho_d)   # alive until the copy kernel has run

    def set_pdfs(self, box, f):
        with self._enter():
            f_d = self._dev(f, self.torch.float64).reshape(19, -1)
            psm_set_pdfs(self.ctx, box, f_d.data_ptr())
            self._keep = (f_d,)

    def get_pdfs(self, box=0):
        with self._enter():
            f = self.torch.empty((19, self.N(box)), dtype=self.torch.float64, device=self.device)
            psm_get_pdfs(self.ctx, box, f.data_ptr())
        return self._hand_back(f)

    def get_pdfs_at(self, box, cells):
        with self._enter():
            cells = np.asarray(cells, dtype=np.int64)
            if len(cells) and (cells.min() < 0 or cells.max() >= self.N(box)):
                raise ValueError("cell index outside the box")
            c = self._dev(cells.astype(np.int32), self.torch.int32)
            out = self.torch.empty((19, len(c)), dtype=self.torch.float64, device=self.device)
            psm_get_pdfs_at(self.ctx, box, len(c), c.data_ptr(), out.data_ptr())
        return self._hand_back(out)

    def get_macroscopic(self, box=0):
        with self._enter():
            rho = self.torch.empty(self.N(box), dtype=self.torch.float64, device=self.device)
            u = self.torch.empty((3, self.N(box)), dtype=self.torch.float64, device=self.device)
            psm_get_macroscopic(self.ctx, box, rho.data_ptr(), u.data_ptr())
        return self._hand_back(rho, u)

    def set_particles(self, box, x, r, U, omega=None):
        psm_set_particles(self.ctx, box, x, r, U, omega)
        self.np[box] = int(len(np.atleast_1d(r)))

    def set_particle_positions(self, box, x):
        psm_set_particle_positions(self.ctx, box, x)

    def set_particle_velocities(self, box, U, omega=None):
        psm_set_particle_velocities(self.ctx, box, U, omega)

    def step(self, n=1):
        psm_step(self.ctx, n)

    def get_forces(self, box=0, F=None, T=None):
        return psm_get_forces(self.ctx, box, self.np[box], F, T)

    def set_dynamics(self, box, density_ratio, accel=None):
        psm_set_dynamics(self.ctx, box, density_ratio, accel)

    def integrate(self, dt=1.0, scheme=PSM_VERLET):
        psm_integrate(self.ctx, dt, scheme)

    def run(self, nsteps, dt=1.0, scheme=PSM_VERLET):
        psm_run(self.ctx, nsteps, dt, scheme)

    def get_particles(self, box=0):
        return psm_get_particles(self.ctx, box, self.np[box])

    def get_solid_fraction(self, box=0):
        with self._enter():
            B = self.torch.empty((2, self.N(box)), dtype=self.torch.float64, device=self.device)
            pid = self.torch.empty((2, self.N(box)), dtype=self.torch.int32, device=self.device)
            psm_get_solid_fraction(self.ctx, box, B.data_ptr(), pid.data_ptr())
        return self._hand_back(B, pid)

    def get_stats(self, box=0):
        return psm_get_stats(self.ctx, box)

    def set_drift_check(self, box, rel_tol):
        psm_set_drift_check(self.ctx, box, rel_tol)

    def set_strict_slots(self, enable):
        psm_set_strict_slots(self.ctx, enable)

    def set_force_readback(self, enable):
        psm_set_force_readback(self.ctx, enable)

    def set_launch(self, tx, ty, tz, flags=0):
        psm_set_launch(self.ctx, tx, ty, tz, flags)

    def get_launch(self):
        return psm_get_launch(self.ctx)

    def autotune(self, trial_steps=5):
        return psm_autotune(self.ctx, trial_steps)

    def set_graph(self, enable):
        psm_set_graph(self.ctx, enable)

    def set_timing(self, enable):
        psm_set_timing(self.ctx, enable)

    def get_timing(self):
        return psm_get_timing(self.ctx)

    def reset_timing(self):
        psm_reset_timing(self.ctx)

    def pattern_copy(self, shifted, nrep):
        """Average ms of one access-pattern copy launch (psm_pattern_copy)."""
        return psm_pattern_copy(self.ctx, shifted, nrep)

    def synchronize(self):
        self.stream.synchronize()


def desc_from_spec(spec, max_particles=None, max_radius=None):
    """Box descriptor for an :class:`inputs.BoxSpec`."""
    n = spec.n_particles if max_particles is None else max_particles
    rmax = (float(np.max(spec.r)) if len(spec.r) else 1.0) if max_radius is None else max_radius
    return make_desc(*spec.dims, spec.tau, spec.fext, max_particles=n, max_radius=max(rmax, 1.0),
                     mapping=spec.mapping, subsample_n=spec.nsub, walls_z=spec.walls_z, wall_u=spec.wall_u,
                     face_type=spec.face_type, face_rho=spec.face_rho, walls_x=spec.walls_x, walls_y=spec.walls_y)
