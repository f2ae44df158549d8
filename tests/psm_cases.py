"""Shared drivers for the GPU parity tests: run a seeded box on the oracle and
on the engine (through the C ABI) and compare with stated tolerances."""
from __future__ import annotations

import numpy as np

import oracle
import paper_2303_11811_amd as psm


def oracle_box(spec):
    return oracle.Box(*spec.dims, tau=spec.tau, fext=spec.fext, mapping=spec.mapping, nsub=spec.nsub,
                      walls_z=spec.walls_z, wall_u=spec.wall_u)


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
