"""Deviation storage forms against the FP64 oracle.

FP32 stores d = f - w_q, FP16 stores 2^10 d; both collide in FP32 and keep
forces, torques and mass sums in FP64. Their error against the oracle is a
property of the rounding, not a parity bar; the bounds asserted here are the
stated error bounds of these forms (about three times the measured values).

Velocity error: L2 of u over all cells relative to the L2 of the oracle's u.
Force error: max over spheres of |dF_p| / max(|F_p|, 0.01 A_p), A_p the sum
over the sphere's cells of B |g| (the magnitude of the terms of eq. 21): a
sphere whose force nearly cancels is measured against 1 % of its terms.

(a) The precision copy of the 512^3 workload: 64^3 periodic box, tau 0.55,
body force 1e-6 along +x, fluid at rest, 6 spheres of radius 10 (10 % solid,
seed 1) with velocities in [-0.005, 0.005]^3, linear mapping, 1000 steps:
  FP32-dev: L2 velocity error <= 5e-5, force error <= 4e-4
  FP16-dev: L2 velocity error <= 6e-4, force error <= 7e-3
(b) 100 steps of a 32^3 Taylor-Green box with 4 spheres (r = 4, tau 0.6):
  FP32-dev: L2 velocity error <= 2e-5, force error <= 1e-4
  FP16-dev: L2 velocity error <= 3e-3, force error <= 2e-2
"""
import os
import time

import numpy as np
import pytest

import oracle
import paper_2303_11811_amd as psm
from paper_2303_11811_amd import inputs
from psm_cases import initial_f, make_engine, run_oracle

pytestmark = pytest.mark.gpu

BOUNDS = {psm.PSM_FP32DEV: (2e-5, 1e-4), psm.PSM_FP16DEV: (3e-3, 2e-2)}
BOUNDS_COPY = {psm.PSM_FP32DEV: (5e-5, 4e-4), psm.PSM_FP16DEV: (6e-4, 7e-3)}


def force_error(F, F_ref, A):
    """max_p |dF_p| / max(|F_p|, 0.01 A_p)."""
    d = np.linalg.norm(F - F_ref, axis=1)
    return float(np.max(d / np.maximum(np.linalg.norm(F_ref, axis=1), 0.01 * A)))


@pytest.fixture(scope="module")
def copy_reference():
    """The oracle on the 64^3 precision copy, 1000 steps. It runs the OpenMP
    timing build of the oracle (the same arithmetic per cell; only the order
    of the force sums over cells differs, far below these bounds)."""
    spec = inputs.paper_scale(n=64, seed=1)
    box = oracle.Box(*spec.dims, tau=spec.tau, fext=spec.fext)
    f0 = oracle.equilibrium(box, np.zeros((3, spec.N)))
    oracle.threads(min(16, os.cpu_count() or 1))
    print(f"[precision copy] oracle 64^3 x 1000 steps, {len(spec.r)} spheres ...", flush=True)
    t0 = time.perf_counter()
    ref = oracle.run(box, f0, 1000, spec.x, spec.r, spec.U, spec.Om, timing_build=True)
    print(f"[precision copy] oracle done in {time.perf_counter() - t0:.1f} s", flush=True)
    _, u_ref = oracle.macroscopic(box, ref.f)
    return spec, u_ref, ref


@pytest.mark.parametrize("storage", [psm.PSM_FP32DEV, psm.PSM_FP16DEV])
def test_precision_copy_of_the_paper_scale_workload(storage, copy_reference):
    spec, u_ref, ref = copy_reference
    eng = make_engine([spec], storage=storage)
    eng.set_equilibrium(0, np.zeros((3, spec.N)))
    eng.set_particles(0, spec.x, spec.r, spec.U, spec.Om)
    eng.set_graph(True)
    eng.step(1000)
    _, u = eng.get_macroscopic(0)
    F, _ = eng.get_forces(0)
    eng.close()
    u = u.cpu().numpy()
    l2 = float(np.linalg.norm(u - u_ref) / np.linalg.norm(u_ref))
    fe = force_error(F, ref.F, ref.A)
    print(f"[precision copy] storage {storage}: L2 u {l2:.3e}, force {fe:.3e}", flush=True)
    bu, bf = BOUNDS_COPY[storage]
    assert l2 <= bu and fe <= bf


def _spec():
    rng = np.random.default_rng(17)
    dims = (32, 32, 32)
    x, r = inputs.rsa_spheres(dims, np.full(4, 4.0), rng)
    U = inputs.uniform_velocities(rng, len(r), 0.01)
    return inputs.BoxSpec(dims=dims, tau=0.6, mapping=0, x=x, r=r, U=U, Om=np.zeros_like(U),
                          u0=inputs.taylor_green(dims, 0.01))


@pytest.mark.parametrize("storage", [psm.PSM_FP32DEV, psm.PSM_FP16DEV])
def test_deviation_storage_error_bounds(storage):
    spec = _spec()
    steps = 100
    ref = run_oracle(spec, steps)
    box = oracle.Box(*spec.dims, tau=spec.tau)
    _, u_ref = oracle.macroscopic(box, ref.f)
    eng = make_engine([spec], storage=storage)
    eng.set_pdfs(0, initial_f(spec))
    eng.set_particles(0, spec.x, spec.r, spec.U, spec.Om)
    eng.step(steps)
    _, u = eng.get_macroscopic(0)
    F, T = eng.get_forces(0)
    u = u.cpu().numpy()
    l2 = np.linalg.norm(u - u_ref) / np.linalg.norm(u_ref)
    fe = force_error(F, ref.F, ref.A)
    print(f"[precision] storage {storage}: L2 u {l2:.3e}, force {fe:.3e}", flush=True)
    bu, bf = BOUNDS[storage]
    assert l2 <= bu and fe <= bf
    # FP64 mass bookkeeping of the rounded state stays close to the true mass
    mass, _, _ = eng.get_stats(0)
    assert abs(mass - ref.f.sum()) / ref.f.sum() < (1e-7 if storage == psm.PSM_FP32DEV else 1e-4)


@pytest.mark.parametrize("storage", [psm.PSM_FP32DEV, psm.PSM_FP16DEV])
def test_deviation_storage_roundtrip(storage):
    """set_pdfs -> get_pdfs rounds d = f - w_q once: exact for FP32 where d is
    representable, within one FP16 ulp of 2^10 d otherwise."""
    spec = inputs.random_small((20, 16, 12), 0, (2, 3), seed=4, tau=0.7)
    f0 = initial_f(spec)
    eng = make_engine([spec], storage=storage)
    eng.set_pdfs(0, f0)
    f = eng.get_pdfs(0).cpu().numpy()
    w = oracle.lattice()[1][:, None]
    d0 = f0 - w
    if storage == psm.PSM_FP32DEV:
        assert np.array_equal(f, d0.astype(np.float32).astype(np.float64) + w)
    else:
        ulp = np.abs(d0) * 2.0 ** -10 + 2.0 ** -24 / 1024 + 1e-16
        assert np.all(np.abs(f - f0) <= ulp)


@pytest.mark.parametrize("scale", [2.0 ** 8, 2.0 ** 12])
def test_fp16_scale_choice(scale):
    """Other power-of-two FP16 scales (the scale is folded into the collision
    constants) give the same physics within the FP16 bounds, and the state
    round trip keeps one FP16 rounding of scale * d."""
    spec = _spec()
    steps = 100
    ref = run_oracle(spec, steps)
    box = oracle.Box(*spec.dims, tau=spec.tau)
    _, u_ref = oracle.macroscopic(box, ref.f)
    eng = make_engine([spec], storage=psm.PSM_FP16DEV, fp16_scale=scale)
    f0 = initial_f(spec)
    eng.set_pdfs(0, f0)
    w = oracle.lattice()[1][:, None]
    back = eng.get_pdfs(0).cpu().numpy()
    # store: FP64 -> FP32 -> FP16 of scale * d; read: FP32 product with 1/scale, then + w in FP64
    h = ((f0 - w) * scale).astype(np.float32).astype(np.float16)
    expect = (h.astype(np.float32) * np.float32(1.0 / scale)).astype(np.float64) + w
    assert np.array_equal(back, expect)
    eng.set_particles(0, spec.x, spec.r, spec.U, spec.Om)
    eng.step(steps)
    _, u = eng.get_macroscopic(0)
    F, T = eng.get_forces(0)
    u = u.cpu().numpy()
    l2 = np.linalg.norm(u - u_ref) / np.linalg.norm(u_ref)
    fe = force_error(F, ref.F, ref.A)
    print(f"[precision] FP16 scale {scale:g}: L2 u {l2:.3e}, force {fe:.3e}", flush=True)
    bu, bf = BOUNDS[psm.PSM_FP16DEV]
    assert l2 <= bu and fe <= bf
    eng.close()


@pytest.mark.parametrize("dims", [(63, 14, 10), (64, 12, 9), (70, 9, 8)])
def test_fp16_one_step_every_cell_row_layouts(dims):
    """Every value of an FP16-deviation box after one step from the engine's
    own state agrees with the FP64 oracle's step from that state to the
    one-step bound of psm_cases.deviation_bound. The widths cover the three
    row layouts of the PDF grid: rows padded to whole 64-cell blocks with an
    odd and with an even width, and rows packed back to back (a wave's cells
    then straddle blocks); two tile widths each, with spheres and a body
    force."""
    from psm_cases import deviation_bound

    rng = np.random.default_rng(23)
    x, r = inputs.rsa_spheres(dims, np.array([2.0, 1.5, 1.8]), rng)
    U = inputs.uniform_velocities(rng, len(r), 0.01)
    spec = inputs.BoxSpec(dims=dims, tau=0.6, mapping=0, x=x, r=r, U=U, Om=np.zeros_like(U),
                          u0=inputs.taylor_green(dims, 0.02), fext=(1e-5, 0.0, 0.0))
    box = oracle.Box(*dims, tau=spec.tau, fext=spec.fext)
    for launch in ((64, 4, 4, 0), (32, 8, 2, 0)):
        print(f"[case] fp16 one step dims={dims} launch={launch}", flush=True)
        eng = make_engine([spec], storage=psm.PSM_FP16DEV, max_radius=2.0)
        eng.set_launch(*launch)
        eng.set_pdfs(0, initial_f(spec))
        eng.set_particles(0, spec.x, spec.r, spec.U, spec.Om)
        eng.step(3)
        f_t = eng.get_pdfs(0).cpu().numpy()
        eng.step(1)
        got = eng.get_pdfs(0).cpu().numpy()
        eng.close()
        ref = oracle.run(box, f_t, 1, x, r, U, spec.Om).f
        bound = deviation_bound(ref.T, psm.PSM_FP16DEV).T
        ratio = np.max(np.abs(got - ref) / bound)
        print(f"[ratio] max |err|/bound = {ratio:.3g}", flush=True)
        assert np.all(np.abs(got - ref) <= bound), ratio
