"""Physical validation beyond parity: Stokes flow through a simple cubic array
of fixed spheres (one sphere in a periodic box), driven by a body force. At
steady state the force on the sphere balances the body force on the fluid, and
the dimensionless drag K = F / (6 pi nu r U_s) (U_s the superficial velocity)
matches Hasimoto's expansion for simple cubic arrays,
K = 1 / (1 - 1.7601 c^(1/3) + c - 1.5593 c^2), within the few per cent that
the partially saturated cells representation of a sphere of radius 6 cells
allows."""
import math

import numpy as np
import pytest

import paper_2303_11811_amd as psm
from paper_2303_11811_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("r,L", [(6.0, 48), (8.0, 40)])
def test_stokes_drag_of_a_periodic_sphere_array(r, L):
    tau, g = 0.75, 2e-7
    nu = (tau - 0.5) / 3.0
    spec = inputs.BoxSpec(dims=(L, L, L), tau=tau, fext=(g, 0.0, 0.0), x=np.array([[L / 2, L / 2, L / 2]]),
                          r=np.array([r]), U=np.zeros((1, 3)), Om=np.zeros((1, 3)))
    eng = psm.Engine([psm.desc_from_spec(spec)], storage=psm.PSM_FP64)
    eng.set_particles(0, spec.x, spec.r, spec.U, spec.Om)
    eng.set_equilibrium(0, np.zeros((3, spec.N)))
    eng.set_graph(True)
    steps = int(6 * L * L / nu)
    eng.step(steps - steps % 10)
    F, _ = eng.get_forces(0)
    _, u = eng.get_macroscopic(0)
    B, _ = eng.get_solid_fraction(0)
    Us = float(u[0].sum().item()) / spec.N          # superficial velocity
    solid = float(B.sum().item())
    eng.close()
    # momentum balance at steady state: the sphere takes the fluid's body force
    assert abs(F[0, 0] - g * (spec.N - solid)) < 1e-6 * g * spec.N
    c = solid / spec.N
    K = F[0, 0] / (6.0 * math.pi * nu * r * Us)
    K_has = 1.0 / (1.0 - 1.7601 * c ** (1.0 / 3.0) + c - 1.5593 * c * c)
    print(f"[drag] r={r} L={L} c={c:.4f} K={K:.4f} Hasimoto={K_has:.4f} dev={K / K_has - 1:+.3%}", flush=True)
    assert abs(K / K_has - 1.0) < 0.05
