"""The OpenMP timing build of the oracle (the CPU baseline's all-core
figure) against the plain build every other test uses: the same source, with
the collide-and-stream loop split over z-planes and the force and torque
summed per thread. PDFs, slots and overflow counts must be bitwise equal at
any thread count, forces and torques equal up to the order of the sums
(R11: 1e-14 of the force's term magnitude), and the pins of the PSM step and
the pressure face hold for it as they do for the plain build."""
import functools

import numpy as np
import pytest

import oracle
from paper_2303_11811_amd import inputs

import test_oracle_lbm as pins_lbm
import test_oracle_psm as pins_psm

_plain_run = oracle.run


@pytest.mark.parametrize("threads", [1, 3, 8])
@pytest.mark.parametrize("case", ["spheres", "overlap_subsample", "walls"])
def test_timing_build_matches_plain_build(case, threads):
    if case == "spheres":
        spec = inputs.random_small((30, 26, 22), 6, (2.5, 4.0), seed=41, tau=0.8, fext=(3e-5, 0, 1e-5),
                                   omamp=0.003)
        box = oracle.Box(*spec.dims, tau=spec.tau, fext=spec.fext)
    elif case == "overlap_subsample":
        spec = inputs.random_small((24, 20, 18), 5, (2.0, 3.5), seed=5, tau=0.7, overlap=True)
        box = oracle.Box(*spec.dims, tau=spec.tau, mapping=oracle.MAP_SUBSAMPLE, nsub=4)
    else:
        spec = inputs.random_small((20, 18, 24), 3, (2.0, 3.0), seed=9, tau=0.75, fext=(1e-5, 0, 2e-5))
        spec.x[:, 2] = np.clip(spec.x[:, 2], 5.0, 19.0)
        box = oracle.Box(*spec.dims, tau=spec.tau, fext=spec.fext, walls_z=True,
                         wall_u=((0.0, 0.0, 0.01), (0.0, 0.0, 0.0)),
                         face_type=(oracle.FACE_VELOCITY, oracle.FACE_PRESSURE), face_rho=(1.0, 0.998),
                         walls_x=True)
    f0 = oracle.equilibrium(box, spec.u0, spec.rho0)
    a = _plain_run(box, f0, 6, spec.x, spec.r, spec.U, spec.Om)
    assert oracle.threads(threads) == threads
    b = _plain_run(box, f0, 6, spec.x, spec.r, spec.U, spec.Om, timing_build=True)
    assert np.array_equal(a.f, b.f)
    assert np.array_equal(a.B, b.B) and np.array_equal(a.pid, b.pid) and a.overflow == b.overflow
    tol = 1e-14 * a.A[:, None] + 1e-12 * np.abs(a.F)
    assert np.all(np.abs(a.F - b.F) <= tol)
    assert np.all(np.abs(a.T - b.T) <= tol * (spec.r.max() + 1))
    assert np.allclose(a.A, b.A, rtol=1e-14, atol=0)


PINS = [
    (pins_psm.test_first_step_force_and_torque_closed_form, ((0.0, 0.0, 0.0),)),
    (pins_psm.test_first_step_force_and_torque_closed_form, ((3e-4, -2e-4, 1e-4),)),
    (pins_psm.test_comoving_particle_feels_no_force, ()),
    (pins_psm.test_rotating_particle_in_resting_fluid, ()),
    (pins_psm.test_momentum_balance_every_step, (False,)),
    (pins_psm.test_momentum_balance_every_step, (True,)),
    (pins_psm.test_b_zero_cells_evolve_as_plain_lbm, ()),
    (pins_lbm.test_uniform_force_from_rest, (0.8,)),
    (pins_lbm.test_pressure_face_first_step_mass_balance, ("velocity_in", 2e-3)),
    (pins_lbm.test_pressure_face_first_step_mass_balance, ("both_pressure", -1.5e-3)),
]


@pytest.mark.parametrize("pin,args", PINS, ids=[f"{p.__name__}{a}" for p, a in PINS])
def test_pins_hold_for_the_timing_build(monkeypatch, pin, args):
    oracle.threads(4)
    monkeypatch.setattr(oracle, "run", functools.partial(_plain_run, timing_build=True))
    pin(*args)
