"""psm_field_stats_noalloc (the allocation-free entry point) against
psm_get_stats on the same state: FP64 mass and momentum agree to sums taken
in another order (1e-13 relative to the mass), on two calls in a row, the
second on a smaller field; both match the totals of the field in numpy."""
import numpy as np
import pytest
import torch

import paper_2303_11811_amd as psm
from paper_2303_11811_amd import inputs
from psm_cases import initial_f, make_engine

pytestmark = pytest.mark.gpu


def _totals_via_noalloc(eng, box):
    f = eng.get_pdfs(box)
    out = torch.full((4,), float("nan"), dtype=torch.float64, device=eng.device)
    eng.synchronize()
    s = torch.cuda.current_stream(eng.device)
    psm.psm_field_stats_noalloc(f.data_ptr(), f.shape[1], out.data_ptr(), s.cuda_stream)
    s.synchronize()
    return out.cpu().numpy(), f.cpu().numpy()


@pytest.mark.parametrize("storage", [psm.PSM_FP64, psm.PSM_FP32DEV])
def test_noalloc_stats_match_get_stats(storage):
    c = np.array([[0, 0, 0], [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1],
                  [1, 1, 0], [-1, -1, 0], [1, -1, 0], [-1, 1, 0], [1, 0, 1], [-1, 0, -1], [1, 0, -1],
                  [-1, 0, 1], [0, 1, 1], [0, -1, -1], [0, 1, -1], [0, -1, 1]], dtype=float)
    # the larger field spans many partial-sum blocks and a ragged last one
    for dims, n in (((130, 96, 70), 12), ((24, 20, 16), 2)):
        spec = inputs.random_small(dims, n, (2.5, 4.0), seed=31, tau=0.7, fext=(1e-5, -2e-6, 0.0), omamp=0.002)
        eng = make_engine([spec], storage=storage)
        eng.set_pdfs(0, initial_f(spec))
        eng.set_particles(0, spec.x, spec.r, spec.U, spec.Om)
        eng.step(3)
        mass, mom, _ = eng.get_stats(0)
        got, f = _totals_via_noalloc(eng, 0)
        ref = np.concatenate([[mass], mom])
        tol = 1e-13 * mass
        assert np.all(np.abs(got - ref) <= tol), (got, ref)
        assert np.all(np.abs(got - np.concatenate([[f.sum()], f.T.reshape(-1, 19) .sum(0) @ c])) <= tol)
        eng.close()


def test_noalloc_stats_limits():
    s = torch.cuda.current_stream()
    out = torch.full((4,), float("nan"), dtype=torch.float64, device="cuda")
    psm.psm_field_stats_noalloc(0, 0, out.data_ptr(), s.cuda_stream)
    s.synchronize()
    assert np.array_equal(out.cpu().numpy(), np.zeros(4))
    with pytest.raises(psm.PsmError) as e:
        psm.psm_field_stats_noalloc(out.data_ptr(), 67108864 + 1, out.data_ptr(), s.cuda_stream)
    assert e.value.code == psm.PSM_EINVAL and "at most" in str(e.value)
