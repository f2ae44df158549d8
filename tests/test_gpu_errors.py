"""Errors only the device can see, reported by the next synchronising call:
a cell index outside the box given to psm_get_pdfs_at (device memory), a
third sphere overlapping a cell in strict-slot mode, and the mass drift
watchdog of psm_get_stats."""
import ctypes

import numpy as np
import pytest
import torch

import paper_2303_11811_amd as psm
from paper_2303_11811_amd import inputs
from psm_cases import initial_f, make_engine

pytestmark = pytest.mark.gpu


def test_pdfs_at_bad_index_reads_nan_and_is_reported():
    spec = inputs.random_small((24, 20, 16), 2, (2.5, 3.0), seed=5, tau=0.7)
    eng = make_engine([spec])
    f0 = initial_f(spec)
    eng.set_pdfs(0, f0)
    eng.set_particles(0, spec.x, spec.r, spec.U, spec.Om)
    N = spec.N
    cells = torch.tensor([5, -1, N, N - 1, -2 ** 31], dtype=torch.int32, device=eng.device)
    out = torch.empty((19, len(cells)), dtype=torch.float64, device=eng.device)
    # the raw C call: the Python wrapper would refuse these indices on the host
    eng.synchronize()
    rc = psm.lib().psm_get_pdfs_at(eng.ctx, 0, len(cells), ctypes.c_void_p(cells.data_ptr()),
                                   ctypes.c_void_p(out.data_ptr()))
    assert rc == psm.PSM_OK
    eng.synchronize()
    o = out.cpu().numpy()
    assert np.array_equal(o[:, 0], f0[:, 5]) and np.array_equal(o[:, 3], f0[:, N - 1])
    assert np.all(np.isnan(o[:, [1, 2, 4]]))
    with pytest.raises(psm.PsmError) as e:
        eng.get_stats(0)
    assert e.value.code == psm.PSM_EINVAL and "outside the box" in str(e.value)
    # reported once; the context keeps working
    mass, _, _ = eng.get_stats(0)
    assert abs(mass - f0.sum()) <= 1e-12 * f0.sum()
    eng.step(2)
    F, _ = eng.get_forces(0)
    assert np.all(np.isfinite(F))
    eng.close()


def _triple_overlap_spec():
    dims = (32, 28, 24)
    x = np.array([[12.0, 13.0, 11.0], [12.6, 13.2, 11.4], [11.7, 12.5, 10.8], [24.0, 6.0, 6.0]])
    r = np.array([3.0, 3.5, 2.5, 3.0])
    U = np.array([[0.01, 0.0, 0.0], [0.0, -0.01, 0.0], [0.0, 0.0, 0.005], [0.0, 0.0, 0.0]])
    return inputs.BoxSpec(dims=dims, tau=0.7, fext=(0.0, 0.0, 0.0), mapping=psm.PSM_MAP_LINEAR, nsub=4,
                          x=x, r=r, U=U, Om=np.zeros_like(U))


@pytest.mark.parametrize("readback", [False, True])
def test_strict_slots_turn_a_third_overlap_into_an_error(readback):
    """Also with the force read-back, where the error word comes with the
    copy the step makes."""
    spec = _triple_overlap_spec()
    f0 = initial_f(spec)
    print(f"[case] strict slots readback={readback}", flush=True)
    # default: the third overlap is dropped and counted, the run goes on
    eng = make_engine([spec])
    eng.set_force_readback(readback)
    eng.set_pdfs(0, f0)
    eng.set_particles(0, spec.x, spec.r, spec.U, spec.Om)
    eng.step(2)
    F_loose, _ = eng.get_forces(0)
    _, _, ov = eng.get_stats(0)
    assert ov > 0
    f_loose = eng.get_pdfs(0).cpu().numpy()
    # strict: the same step runs, then the next synchronising call refuses
    eng.set_strict_slots(True)
    eng.set_pdfs(0, f0)
    eng.set_particles(0, spec.x, spec.r, spec.U, spec.Om)
    eng.step(2)
    assert np.array_equal(eng.get_pdfs(0).cpu().numpy(), f_loose)
    with pytest.raises(psm.PsmError) as e:
        eng.get_forces(0)
    assert e.value.code == psm.PSM_ECAPACITY and "more than two" in str(e.value)
    with pytest.raises(psm.PsmError) as e:
        eng.step(1)
    assert e.value.code == psm.PSM_ESTATE
    # spheres without a third overlap: usable again, and nothing is reported
    keep = [0, 3]
    eng.set_particles(0, spec.x[keep], spec.r[keep], spec.U[keep], spec.Om[keep])
    eng.set_pdfs(0, f0)
    eng.step(2)
    F, _ = eng.get_forces(0)
    assert np.all(np.isfinite(F)) and np.all(np.isfinite(F_loose))
    eng.close()


def test_strict_slots_from_the_environment(monkeypatch):
    monkeypatch.setenv("PSM_STRICT_SLOTS", "1")
    spec = _triple_overlap_spec()
    eng = make_engine([spec])
    eng.set_pdfs(0, initial_f(spec))
    eng.set_particles(0, spec.x, spec.r, spec.U, spec.Om)
    eng.step(1)
    with pytest.raises(psm.PsmError) as e:
        eng.get_stats(0)
    assert e.value.code == psm.PSM_ECAPACITY
    eng.close()


def test_drift_watchdog():
    """FP64 keeps the mass of a periodic coupled box to round-off, so a
    1e-12 tolerance holds over many steps; FP16-deviation storage rounds
    every stored value and its mass moves by more than that; a box with a
    pressure face cannot be watched."""
    spec = inputs.random_small((32, 28, 24), 4, (2.5, 3.5), seed=9, tau=0.65, fext=(1e-5, 0.0, 0.0),
                               omamp=0.002)
    f0 = initial_f(spec)
    for storage, drifts in ((psm.PSM_FP64, False), (psm.PSM_FP16DEV, True)):
        eng = make_engine([spec], storage=storage)
        eng.set_drift_check(0, 1e-12)
        eng.set_pdfs(0, f0)
        eng.set_particles(0, spec.x, spec.r, spec.U, spec.Om)
        m0, _, _ = eng.get_stats(0)          # the reference
        eng.step(40)
        if drifts:
            with pytest.raises(psm.PsmError) as e:
                eng.get_stats(0)
            assert e.value.code == psm.PSM_EDRIFT
            eng.set_drift_check(0, 0.0)      # off: the same totals are returned without error
            m, _, _ = eng.get_stats(0)
            assert abs(m - m0) > 1e-12 * m0
        else:
            m, _, _ = eng.get_stats(0)
            assert abs(m - m0) <= 1e-12 * m0
        eng.close()
    d = psm.make_desc(16, 16, 16, 0.7, walls_z=True, face_type=(psm.PSM_FACE_VELOCITY, psm.PSM_FACE_PRESSURE))
    eng = psm.Engine([d])
    with pytest.raises(psm.PsmError) as e:
        eng.set_drift_check(0, 1e-12)
    assert e.value.code == psm.PSM_EINVAL
    eng.set_drift_check(0, 0.0)
    eng.close()
