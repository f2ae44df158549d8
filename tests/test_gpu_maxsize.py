"""The largest box the engine takes: 1280 x 1280 x 1310 = 2,146,304,000 cells
(just below 2^31) in FP16-deviation storage (163 GB of PDFs in HBM), with
spheres and a body force. Sampled cells agree with the oracle's one-step
recomputation to the FP16 storage bound, the FP64 mass stays N to the FP16
rounding of the stored deviations, and forces are finite."""
import numpy as np
import pytest

import paper_2303_11811_amd as psm
from paper_2303_11811_amd import inputs
from psm_cases import deviation_bound, one_step_sampled, sample_cells

pytestmark = pytest.mark.gpu


def test_largest_box_fp16():
    import torch

    torch.cuda.empty_cache()
    dims = (1280, 1280, 1310)
    N = dims[0] * dims[1] * dims[2]
    assert N < 2 ** 31
    rng = np.random.default_rng(41)
    x, r = inputs.rsa_spheres(dims, np.full(200, 10.0), rng)
    spec = inputs.BoxSpec(dims=dims, tau=0.6, fext=(1e-6, 0.0, 0.0), x=x, r=r,
                          U=inputs.uniform_velocities(rng, len(r), 0.005), Om=np.zeros_like(x))
    print(f"[case] largest box {dims} cells={N}", flush=True)
    eng = psm.Engine([psm.desc_from_spec(spec)], storage=psm.PSM_FP16DEV)
    with torch.cuda.stream(eng.stream):
        u0 = torch.zeros((3, N), dtype=torch.float64, device=eng.device)
    eng.set_equilibrium(0, u0)
    eng.synchronize()
    del u0
    torch.cuda.empty_cache()
    eng.set_particles(0, spec.x, spec.r, spec.U, spec.Om)
    eng.step(3)
    cells = sample_cells(spec, spec.x, spec.r, rng, n_surface=16, n_random=16)
    got, ref = one_step_sampled(eng, 0, spec, cells, spec.x, spec.r, spec.U, spec.Om)
    bound = deviation_bound(ref, psm.PSM_FP16DEV)
    print(f"[ratio] max |err|/bound = {np.max(np.abs(got - ref) / bound):.3g}", flush=True)
    assert np.all(np.abs(got - ref) <= bound)
    mass, mom, _ = eng.get_stats(0)
    F, T = eng.get_forces(0)
    eng.close()
    # the stored deviations start at zero and stay below 1e-3; each FP16
    # rounding is at most 2^-11 of one, so the mass drift is far below 1e-3 N
    assert abs(mass - N) < 1e-3 * N
    assert np.all(np.isfinite(F)) and np.all(np.isfinite(T)) and np.all(np.isfinite(mom))
