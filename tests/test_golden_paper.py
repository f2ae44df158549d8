"""Values the paper prints, kept as fixtures under tests/golden/: the
roofline estimate of Sec. 4.2.1 (eq. 28), which fixes the algorithmic bytes
per cell the measurements use, and the fluidized-bed workload of Sec. 4.1,
which the synthetic bed inputs stand in for."""
import math
import os

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLDEN = os.path.join(ROOT, "tests", "golden")


def _fixture(name):
    vals = {}
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if line:
                k, v = (t.strip() for t in line.split("=", 1))
                vals[k] = float(v)
    return vals


def test_roofline_bytes_and_time_match_eq28():
    import bench

    g = _fixture("roofline_lightspeed.txt")
    per_cell = (g["pdfs_read_per_cell"] + g["pdfs_written_per_cell"]) * g["bytes_per_value"]
    assert per_cell == g["bytes_per_cell"]
    assert bench.BYTES_PER_CELL[0] == g["bytes_per_cell"]
    # the deviation forms move the same 38 values per cell in 4 and 2 bytes
    assert bench.BYTES_PER_CELL[1] * 2 == bench.BYTES_PER_CELL[0]
    assert bench.BYTES_PER_CELL[2] * 4 == bench.BYTES_PER_CELL[0]
    t = bench.lightspeed_ms(g["cells"], 0, g["bandwidth_gb_per_s"])
    assert round(t, 1) == g["t_min_ms"]


def test_bed_inputs_match_the_papers_setup():
    from paper_2303_11811_amd import inputs

    g = _fixture("fluidized_bed.txt")
    for case, count in (("dilute", g["particles_dilute"]), ("dense", g["particles_dense"])):
        spec, rho_p, accel = inputs.fluidized_bed(case)
        assert tuple(spec.dims) == (g["nx"], g["ny"], g["nz"])
        assert int(np.prod(spec.dims)) == g["cells"]
        assert len(spec.r) == count
        assert np.all(2.0 * spec.r == g["cells_per_diameter"])
        assert rho_p == g["density_ratio"]
        # the dimensionless groups, with nu = (tau - 1/2)/3 in lattice units:
        # particle Reynolds number from the inflow speed, Galileo number from
        # the reduced gravity (gravity minus buoyancy, per unit particle mass)
        nu = (spec.tau - 0.5) / 3.0
        d = g["cells_per_diameter"]
        u_in = spec.wall_u[0][2]
        assert math.isclose(u_in * d / nu, g["particle_reynolds"], rel_tol=1e-12)
        gravity = -accel[2] / (1.0 - 1.0 / rho_p)
        ga = math.sqrt((rho_p - 1.0) * gravity * d ** 3) / nu
        assert math.isclose(ga, g["galileo"], rel_tol=1e-12)
        # every sphere inside the walled box, none overlapping
        L = np.asarray(spec.dims, dtype=float)
        assert np.all(spec.x - spec.r[:, None] >= 1.0 - 1e-12)
        assert np.all(spec.x + spec.r[:, None] <= L - 1.0 + 1e-12)
        from scipy.spatial import cKDTree

        dist, _ = cKDTree(spec.x).query(spec.x, k=2)
        assert dist[:, 1].min() >= d
