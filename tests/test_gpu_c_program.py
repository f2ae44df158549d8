"""The library driven from plain C (tests/c_abi_program.c: include/psm.h and
the HIP runtime only, no Python or torch in the process): a seeded box with
moving, rotating spheres and a body force, run from rest, must give the
oracle's forces, torques, mass and cell values to the FP64 tolerances of the
parity tests."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
import paper_2303_11811_amd as psm
from paper_2303_11811_amd import inputs
from psm_cases import assert_forces_close, run_oracle

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def test_c_program_matches_oracle(tmp_path):
    cc = shutil.which("gcc")
    if cc is None:
        pytest.skip("no C compiler")
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    libdir = os.path.dirname(psm.LIB_PATH)
    exe = tmp_path / "c_abi_program"
    subprocess.run([cc, "-std=c99", "-O2", "-Wall", "-D__HIP_PLATFORM_AMD__", f"-I{rocm}/include",
                    f"-I{os.path.join(ROOT, 'include')}", os.path.join(HERE, "c_abi_program.c"), "-o", str(exe),
                    f"-L{libdir}", "-lpsm", f"-L{rocm}/lib", "-lamdhip64",
                    f"-Wl,-rpath,{libdir}", f"-Wl,-rpath,{rocm}/lib"], check=True)
    spec = inputs.random_small((26, 22, 18), 3, (2.5, 4.0), seed=91, tau=0.72, fext=(1e-5, -4e-6, 2e-6),
                               vamp=0.01, omamp=0.002)
    spec.u0, spec.rho0 = None, None   # the program starts from rest
    steps = 12
    lines = [f"{spec.dims[0]} {spec.dims[1]} {spec.dims[2]} {spec.tau!r} "
             f"{spec.fext[0]!r} {spec.fext[1]!r} {spec.fext[2]!r} {steps} {len(spec.r)}"]
    for i in range(len(spec.r)):
        vals = [*spec.x[i], spec.r[i], *spec.U[i], *spec.Om[i]]
        lines.append(" ".join(repr(float(v)) for v in vals))
    inp = tmp_path / "box.txt"
    inp.write_text("\n".join(lines) + "\n")
    print(f"[case] C program dims={spec.dims} spheres={len(spec.r)} steps={steps}", flush=True)
    out = subprocess.run([str(exe), str(inp)], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, (out.returncode, out.stdout, out.stderr)

    F = np.zeros((len(spec.r), 3))
    T = np.zeros((len(spec.r), 3))
    vals = {}
    for line in out.stdout.splitlines():
        tok = line.split()
        if tok[0] == "sphere":
            i = int(tok[1])
            F[i] = [float(v) for v in tok[2:5]]
            T[i] = [float(v) for v in tok[5:8]]
        else:
            vals[tok[0]] = [float(v) for v in tok[1:]]

    ref = run_oracle(spec, steps)
    assert_forces_close(F, ref.F, ref.A)
    assert_forces_close(T, ref.T, ref.A, lever=spec.r.max() + 1)
    assert abs(vals["mass"][0] - ref.f.sum()) <= 1e-12 * ref.f.sum()
    rho, u = oracle.macroscopic(oracle.Box(*spec.dims, tau=spec.tau, fext=spec.fext), ref.f)
    assert abs(vals["cell0"][0] - rho[0]) <= 1e-12 * abs(rho[0])
    assert np.all(np.abs(np.array(vals["cell0"][1:]) - u[:, 0]) <= 1e-14)
    assert vals["overflows"][0] == ref.overflow
