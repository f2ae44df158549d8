"""bench.py's host-side contract: more than one GPU is refused with a
message before anything touches a GPU, and the per-form byte accounting and
counter bookkeeping are consistent."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120)
    assert out.returncode == 2
    assert "one GPU" in out.stderr and out.stdout == ""


def test_counter_files_match_their_forms():
    import bench

    for st, name in bench.STORAGE_NAME.items():
        path = bench.counter_file(st)
        if not os.path.exists(path):
            continue
        c = json.load(open(path))
        assert f"St{ {0: 64, 1: 32, 2: 16}[st] }" in c["kernel"].replace(" ", "")
        assert c["algorithmic_bytes_per_launch"] == 512 ** 3 * bench.BYTES_PER_CELL[st]
        assert abs(c["hbm_bytes_per_launch"] - c["hbm_read_bytes_per_launch"] - c["hbm_write_bytes_per_launch"]) < 1.0
        # a fresh counter file is the one bench.py reports as traffic
        if c["kernel_src_sha"] == bench.kernel_source_hash():
            assert bench.measured_traffic(st)[0] == c["hbm_bytes_per_launch"]


class _StubEngine:
    """Stands in for paper_2303_11811_amd.Engine on the CPU: accepts every
    call bench.py makes and returns arrays of the right shapes, so that the
    host-side loops of the benchmark run end to end without a GPU."""

    def __init__(self, descs, storage=0, fp16_scale=0.0):
        import torch

        self.n = [d.nx * d.ny * d.nz for d in descs]
        self.np = [0] * len(descs)
        self.stream, self.device = None, "cpu"
        self.launch = (64, 4, 1, 0)
        self.calls = 0
        self._torch = torch

    def set_particles(self, b, x, r, U, Om=None):
        self.np[b] = len(r)

    def set_particle_positions(self, b, x):
        assert x.shape == (self.np[b], 3)

    def set_particle_velocities(self, b, U, Om=None):
        assert U.shape == (self.np[b], 3)

    def set_force_readback(self, enable):
        pass

    def set_equilibrium(self, b, u0):
        assert tuple(u0.shape) == (3, self.n[b])

    def autotune(self, trial_steps=4):
        return self.launch, 1.0

    def set_launch(self, *ln):
        self.launch = tuple(ln)

    def get_launch(self):
        return self.launch

    def step(self, n):
        self.calls += n

    def run(self, n, dt, scheme):
        self.calls += n

    def get_forces(self, b, F=None, T=None):
        import numpy as np

        F = np.empty((self.np[b], 3)) if F is None else F
        T = np.empty((self.np[b], 3)) if T is None else T
        assert F.shape == T.shape == (self.np[b], 3)
        F.fill(1e-6)
        T.fill(1e-7)
        return F, T

    def get_macroscopic(self, b):
        t = self._torch
        return t.ones(self.n[b], dtype=t.float64), t.full((3, self.n[b]), 1e-3, dtype=t.float64)

    def get_stats(self, b):
        return float(self.n[b]), (0.0, 0.0, 0.0), 0

    def get_timing(self):
        return max(self.calls, 1), 1.0 * max(self.calls, 1)

    def pattern_copy(self, shifted, nrep):
        return 1.0

    def set_dynamics(self, *a):
        pass

    def set_graph(self, *a):
        pass

    def set_timing(self, *a):
        pass

    def reset_timing(self):
        pass

    def synchronize(self):
        pass

    def close(self):
        pass


def _stub_modules():
    import contextlib
    import types

    import torch

    import paper_2303_11811_amd as psm

    class Ev:
        def __init__(self, enable_timing=False):
            pass

        def record(self, stream=None):
            pass

        def synchronize(self):
            pass

        def elapsed_time(self, other):
            return 1.0

    cuda = types.SimpleNamespace(Event=Ev, stream=lambda s: contextlib.nullcontext(), synchronize=lambda: None,
                                 empty_cache=lambda: None, is_available=lambda: True)
    fake_torch = types.SimpleNamespace(zeros=torch.zeros, ones=torch.ones, full=torch.full, empty=torch.empty,
                                       as_tensor=torch.as_tensor, float64=torch.float64, uint8=torch.uint8,
                                       cuda=cuda)
    fake_psm = types.SimpleNamespace(**{k: getattr(psm, k) for k in dir(psm) if not k.startswith("__")})
    fake_psm.Engine = _StubEngine
    return fake_psm, fake_torch


def test_bench_host_loops_run_against_a_stub_engine():
    """The Python side of every timed leg that fits a CPU (main case with its
    access-pattern copies, the batched boxes, the moving suspension with host
    and device updates) runs to the end and returns finite figures."""
    import math

    import bench
    from paper_2303_11811_amd import inputs

    fpsm, ftorch = _stub_modules()
    spec = inputs.paper_scale(n=48, seed=1)
    r = bench.run_case(fpsm, ftorch, spec, 0, 60, 1, True)
    assert len(r["window_mlups"]) == 5
    s = bench.pattern_summary(r, spec.N * bench.BYTES_PER_CELL[0])
    assert s["kernel_over_pull"] == 1.0 and r["launch"] == [64, 4, 1, 0]
    b = bench.run_batched(fpsm, ftorch, inputs, steps=3, nbox=2)
    assert b["boxes"] == 2 and math.isfinite(b["mlups"])
    for device in (False, True):
        d = bench.run_dense_moving(fpsm, ftorch, inputs, n=48, steps=3, warmup=1, device=device)
        assert math.isfinite(d["coupling_overhead_frac"]) and d["steps"] == 3
        assert ("breakdown" in d) != device
