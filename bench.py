#!/usr/bin/env python
"""PSM-LBM benchmark on one MI355X.

Workload (default): 512^3 periodic box, FP64 PDFs, tau 0.55, body force
1e-6 along +x, 3204 seeded non-overlapping spheres of diameter 20 (10 %
solid volume fraction) with velocities in [-0.005, 0.005]^3. One timed
step is the whole coupled hot path of the paper's GPU time step: upload the
sphere table (positions, radii, f(r), velocities) and rebuild the per-tile
candidate lists, run the fused mapping + stream-collide + force/torque
launch and the per-sphere reduction, and read the forces and torques back.

Prints one JSON line. `value` is MLUPS (cells x steps / wall time / 1e6)
with the PDFs resident in HBM. `roofline` is the step kernel's algorithmic
PDF traffic (38 values per cell: 304 B FP64, 152 B FP32, 76 B FP16) per
launch over its average launch time (HIP events on its own stream) against
the 8 TB/s HBM peak. `cpu_baseline` is the FP64 oracle (single thread) on a
bounded sample of the same workload.
"""
import argparse
import gc
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
METRIC = "PSM-LBM MLUPS & % HBM roofline, FP64 vs FP32/FP16-storage at stated error"
BYTES_PER_CELL = {0: 304, 1: 152, 2: 76}
STORAGE_NAME = {0: "f64", 1: "f32dev", 2: "f16dev"}
STORAGE_OF = {v: k for k, v in STORAGE_NAME.items()}
DTYPE = {0: "f64", 1: "f32", 2: "f32"}   # arithmetic of the step in each storage form


def counter_file(storage):
    return os.path.join(ROOT, "profiles", f"k_psm_step_{STORAGE_NAME[storage]}_512_counters.json")


def lightspeed_ms(cells, storage, gbps):
    """Roofline time of one step (Sec. 4.2.1, eq. 28): the algorithmic PDF
    bytes of `cells` cells in the given storage form at `gbps` GB/s."""
    return cells * BYTES_PER_CELL[storage] / (gbps * 1e9) * 1e3


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("psm_kernels.hip", "psm_internal.h"):
        with open(os.path.join(ROOT, "paper_2303_11811_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(storage=0):
    """(HBM bytes per launch, launch shape of the counter run) from the
    committed rocprofv3 counters of the storage form, if they were taken on
    the current kernel source; (None, None) otherwise."""
    try:
        with open(counter_file(storage)) as fh:
            c = json.load(fh)
    except (OSError, ValueError):
        return None, None
    if c.get("kernel_src_sha") != kernel_source_hash():
        return None, None
    return c.get("hbm_bytes_per_launch"), c.get("launch")


def run_case(psm, torch, spec, storage, steps, warmup, autotune, launch=None, full_loop=True):
    """Time `steps` coupled steps of one box (a box without spheres when spec
    has none). Returns a dict of results."""
    eng = psm.Engine([psm.desc_from_spec(spec)], storage=storage)
    N = spec.N
    with torch.cuda.stream(eng.stream):
        u0 = torch.zeros((3, N), dtype=torch.float64, device=eng.device)
    eng.set_particles(0, spec.x, spec.r, spec.U, spec.Om)
    if launch is not None:
        eng.set_launch(*launch)
    elif autotune:
        eng.set_equilibrium(0, u0)
        shape, ms = eng.autotune(trial_steps=4)
        log(f"  autotune -> {shape} {ms:.3f} ms/step")
    eng.set_equilibrium(0, u0)
    del u0

    def one_step():
        if full_loop:
            eng.set_particles(0, spec.x, spec.r, spec.U, spec.Om)
        eng.step(1)
        if full_loop:
            eng.get_forces(0)

    for _ in range(warmup):
        one_step()
    torch.cuda.synchronize()
    eng.reset_timing()
    eng.set_timing(True)
    torch.cuda.synchronize()
    # no Python garbage collection inside the timed loop (as timeit does)
    gc.collect()
    gc.disable()
    # five consecutive windows of the timed steps (each step of the full loop
    # ends in a synchronising force read, so the marks need no extra sync)
    nwin = 5 if full_loop and steps >= 50 else 1
    edges = [steps * w // nwin for w in range(nwin + 1)]
    marks = []
    t0 = time.perf_counter()
    for i in range(steps):
        if i in edges:
            marks.append(time.perf_counter())
        one_step()
    eng.synchronize()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    gc.enable()
    marks.append(t1)
    n_launch, kern_ms = eng.get_timing()
    eng.set_timing(False)
    mass, mom, ov = eng.get_stats(0)
    win = [N * (edges[w + 1] - edges[w]) / (marks[w + 1] - marks[w]) / 1e6 for w in range(nwin)]
    res = dict(ms_per_step=(t1 - t0) * 1e3 / steps, mlups=N * steps / (t1 - t0) / 1e6,
               kernel_ms=kern_ms / max(n_launch, 1), launches=n_launch, launch=list(eng.get_launch()),
               mass=mass, slot_overflows=ov, window_mlups=[round(v, 1) for v in win])
    # the same tiles, pulls and stores with no arithmetic (after the timed
    # region; the state is not touched): the rate HBM serves this pattern
    res["pattern_copy_ms"] = {"pull": eng.pattern_copy(1, 10), "own_cell": eng.pattern_copy(0, 10)}
    eng.close()
    del eng
    torch.cuda.empty_cache()
    return res


def pattern_summary(res, algo_bytes):
    """The step kernel against the copy of its own access pattern (same
    launch, tiles, pulls and stores, no arithmetic): GB/s of the pulled
    copy, of the copy from each cell's own slots (no shifts), and the
    kernel's time over the pulled copy's."""
    pc = res["pattern_copy_ms"]
    return {"pull_GBps": round(algo_bytes / (pc["pull"] * 1e-3) / 1e9, 1),
            "own_cell_GBps": round(algo_bytes / (pc["own_cell"] * 1e-3) / 1e9, 1),
            "pull_ms": round(pc["pull"], 4), "own_cell_ms": round(pc["own_cell"], 4),
            "kernel_over_pull": round(res["kernel_ms"] / pc["pull"], 4)}


def stream_copy_gbps(psm, torch, nbytes=4 << 30, reps=20):
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    s = torch.cuda.current_stream()
    for _ in range(3):
        psm.psm_stream_copy(a.data_ptr(), b.data_ptr(), nbytes, s.cuda_stream)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        psm.psm_stream_copy(a.data_ptr(), b.data_ptr(), nbytes, s.cuda_stream)
    e1.record(s)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    torch.cuda.empty_cache()
    return 2.0 * nbytes / (ms * 1e-3) / 1e9


PRECISION_COPY = (64, 1000)   # edge and steps of the precision copy of the workload


def velocity_error(u, u_ref):
    """L2 of u - u_ref over all cells relative to the L2 of u_ref."""
    import numpy as np

    return float(np.linalg.norm(u - u_ref) / np.linalg.norm(u_ref))


def force_error(F, F_ref, A=None):
    """max_p |dF_p| / max(|F_p|, 0.01 A_p), A_p the sum of the terms' magnitudes
    B |g| over the sphere's cells (no floor when A is not known)."""
    import numpy as np

    d = np.linalg.norm(F - F_ref, axis=1)
    den = np.linalg.norm(F_ref, axis=1)
    if A is not None:
        den = np.maximum(den, 0.01 * A)
    return float(np.max(d / den))


def precision_copy_runs(psm, torch, inputs):
    """The three storage forms on the 64^3 copy of the workload for 1000
    steps: velocity field and forces of each (the errors against the oracle
    are taken in the CPU-baseline leg, which runs the oracle on the same copy),
    and the deviation forms' errors against the GPU FP64 path."""
    import numpy as np

    n, steps = PRECISION_COPY
    spec = inputs.paper_scale(n=n, seed=1)
    runs = {}
    for st in (0, 1, 2):
        eng = psm.Engine([psm.desc_from_spec(spec)], storage=st)
        eng.set_equilibrium(0, np.zeros((3, spec.N)))
        eng.set_particles(0, spec.x, spec.r, spec.U, spec.Om)
        eng.set_graph(True)
        eng.step(steps)
        _, u = eng.get_macroscopic(0)
        F, _ = eng.get_forces(0)
        runs[st] = (u.cpu().numpy(), F)
        eng.close()
    errs = {}
    for st in (1, 2):
        errs[STORAGE_NAME[st]] = {"l2_u_rel": velocity_error(runs[st][0], runs[0][0]),
                                  "force_rel": force_error(runs[st][1], runs[0][1])}
    return runs, errs


def run_batched(psm, torch, inputs, steps=500, nbox=64):
    """64 independent uneven boxes in one launch per step, replayed as
    captured 10-step HIP graphs at the autotuner's launch: FP32 deviation
    storage (the batched form), the same boxes in FP64 storage for its
    speed-up and velocity error, and the FP32 boxes once more on the
    persistent grid (an occupancy-sized grid whose workgroups walk the tiles
    of all boxes) at the same tile shape."""
    import numpy as np

    specs = inputs.batched_boxes(nbox=nbox, seed=3)
    descs = [psm.desc_from_spec(s, max_particles=max(s.n_particles, 1), max_radius=8.0) for s in specs]
    cells = sum(s.N for s in specs)

    def run(storage, persistent_too=False):
        eng = psm.Engine(descs, storage=storage)
        for b, s in enumerate(specs):
            if s.n_particles:
                eng.set_particles(b, s.x, s.r, s.U, s.Om)
        for b, s in enumerate(specs):
            eng.set_equilibrium(b, s.u0)
        shape, _ = eng.autotune(trial_steps=10)

        def timed():
            for b, s in enumerate(specs):
                eng.set_equilibrium(b, s.u0)
            eng.set_graph(True)
            eng.step(20)
            eng.synchronize()
            t0 = time.perf_counter()
            eng.step(steps)
            eng.synchronize()
            return time.perf_counter() - t0

        dt = timed()
        u = [eng.get_macroscopic(b)[1].cpu().numpy() for b in range(len(specs))]
        finite = all(np.isfinite(eng.get_stats(b)[0]) for b in range(len(specs)))
        res = {"dt": dt, "u": u, "shape": shape, "finite": finite}
        if persistent_too:
            pshape = (shape[0], shape[1], shape[2], shape[3] | psm.PSM_LAUNCH_PERSISTENT)
            eng.set_launch(*pshape)
            res["pshape"], res["dtp"] = pshape, timed()
        eng.close()
        torch.cuda.empty_cache()
        return res

    r32 = run(psm.PSM_FP32DEV, persistent_too=True)
    r64 = run(psm.PSM_FP64)
    num = sum(float(np.sum((a - b) ** 2)) for a, b in zip(r32["u"], r64["u"]))
    den = sum(float(np.sum(b ** 2)) for b in r64["u"])
    dt = r32["dt"]
    return {"boxes": len(specs), "cells": cells, "spheres": int(sum(s.n_particles for s in specs)),
            "steps": steps, "mlups": cells * steps / dt / 1e6, "ms_per_step": dt * 1e3 / steps,
            "storage": "f32dev", "launch": list(r32["shape"]), "graph_steps": 10, "finite": bool(r32["finite"]),
            "roofline_frac": cells * 152 / (dt / steps) / 1e9 / HBM_PEAK_GBPS,
            "f64_mlups": cells * steps / r64["dt"] / 1e6, "f64_launch": list(r64["shape"]),
            "speedup_vs_f64": r64["dt"] / dt,
            "l2_u_rel_vs_f64": (num / den) ** 0.5,
            "persistent_launch": list(r32["pshape"]), "mlups_persistent": cells * steps / r32["dtp"] / 1e6,
            "launch_form": "one workgroup per tile over the tiles of all boxes (mlups); the persistent grid is "
                           "reported beside it (mlups_persistent)"}


def run_dense_moving(psm, torch, inputs, n=768, steps=500, warmup=20, device=False):
    """Moving dense suspension advanced by explicit Euler (density ratio 2.5):
    x_{n+1} = x_n + U_n, U_{n+1} = U_n + F_n/m, Omega_{n+1} = Omega_n + T_n/I.
    Host form: every step the forces are read back and the spheres are
    updated on the host; the new positions (which do not need the forces)
    are computed and uploaded while the step runs (the upload and the device
    re-binning are ordered after the step on its stream), the new velocities
    once the forces are back. Device form (device=True): the same update and
    the re-binning run on the GPU (psm_run) with no per-step host round trip;
    the forces are read once at the end."""
    import numpy as np

    spec = inputs.dense_moving(n=n, seed=4)
    eng = psm.Engine([psm.desc_from_spec(spec, max_radius=8.0)], storage=psm.PSM_FP32DEV)
    with torch.cuda.stream(eng.stream):
        u0 = torch.zeros((3, spec.N), dtype=torch.float64, device=eng.device)
    eng.set_particles(0, spec.x, spec.r, spec.U, spec.Om)
    eng.set_equilibrium(0, u0)
    shape, _ = eng.autotune(trial_steps=3)
    eng.set_equilibrium(0, u0)
    del u0
    x, U, Om = spec.x.copy(), spec.U.copy(), spec.Om.copy()
    xn, F, T = np.empty_like(x), np.empty_like(x), np.empty_like(x)
    mass = 2.5 * 4.0 / 3.0 * np.pi * spec.r ** 3
    inv_m = np.repeat((1.0 / mass)[:, None], 3, axis=1)
    inv_I = np.repeat((1.0 / (0.4 * mass * spec.r ** 2))[:, None], 3, axis=1)
    L = float(spec.dims[0])
    assert spec.dims[0] == spec.dims[1] == spec.dims[2]
    eng.set_particles(0, x, spec.r, U, Om)
    if not device:
        # the forces are copied at the end of each step: reading them does not
        # wait for the position upload and re-binning enqueued after the step
        eng.set_force_readback(True)

    # per-module record of the host loop: host times around each call, and
    # events on the engine's stream around the step launches and the
    # position upload + re-binning
    rec = {"step_call": 0.0, "positions": 0.0, "set_positions": 0.0, "get_forces": 0.0, "velocities": 0.0,
           "set_velocities": 0.0}
    evs = []

    def one(record=False):
        nonlocal x, xn
        t0 = time.perf_counter()
        if record:
            e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
            e[0].record(eng.stream)
        eng.step(1)
        if record:
            e[1].record(eng.stream)
        t1 = time.perf_counter()
        np.add(x, U, out=xn)               # x_{n+1} = x_n + U_n, while the step runs
        xn[xn >= L] -= L                   # |U| < 1: one period at most
        xn[xn < 0.0] += L
        t2 = time.perf_counter()
        eng.set_particle_positions(0, xn)  # copied before the call returns
        if record:
            e[2].record(eng.stream)
        t3 = time.perf_counter()
        eng.get_forces(0, F, T)            # waits for the step
        t4 = time.perf_counter()
        np.multiply(F, inv_m, out=F)       # U_{n+1} = U_n + F_n / m
        np.add(U, F, out=U)
        np.multiply(T, inv_I, out=T)       # Omega_{n+1} = Omega_n + T_n / I
        np.add(Om, T, out=Om)
        t5 = time.perf_counter()
        eng.set_particle_velocities(0, U, Om)
        t6 = time.perf_counter()
        x, xn = xn, x
        if record:
            evs.append(e)
            for k, dt_ in (("step_call", t1 - t0), ("positions", t2 - t1), ("set_positions", t3 - t2),
                           ("get_forces", t4 - t3), ("velocities", t5 - t4), ("set_velocities", t6 - t5)):
                rec[k] += dt_

    if device:
        # kernel time from an eager timed pass, wall time from graph replays
        # of 10 (step + update) pairs with the host out of the loop
        eng.set_dynamics(0, 2.5)
        eng.reset_timing()
        eng.set_timing(True)
        eng.run(warmup + 10, 1.0, psm.PSM_EULER)
        nl, kms = eng.get_timing()
        eng.set_timing(False)
        eng.set_graph(True)
        eng.run(10, 1.0, psm.PSM_EULER)
        eng.synchronize()
        t0 = time.perf_counter()
        eng.run(steps, 1.0, psm.PSM_EULER)
        eng.get_forces(0)   # synchronises; reports a device-side list overflow
        dt = time.perf_counter() - t0
    else:
        for _ in range(warmup):
            one()
        # the timed loop carries no instrumentation; a second loop of up to
        # 100 steps, with events and host clocks around every call, gives the
        # kernel time and the per-module breakdown
        eng.synchronize()
        gc.collect()
        gc.disable()
        t0 = time.perf_counter()
        for _ in range(steps):
            one()
        eng.get_forces(0)
        dt = time.perf_counter() - t0
        nrec = min(steps, 100)
        eng.reset_timing()
        eng.set_timing(True)
        for _ in range(nrec):
            one(record=True)
        eng.get_forces(0)
        gc.enable()
        nl, kms = eng.get_timing()
        eng.set_timing(False)
        launches = sum(a.elapsed_time(b) for a, b, _ in evs) / nrec
        upbin = sum(b.elapsed_time(c) for _, b, c in evs) / nrec
        # the force read alone on an idle stream: the wait for the copy the
        # step made and the host's copy into F and T
        eng.synchronize()
        t0r = time.perf_counter()
        for _ in range(20):
            eng.get_forces(0, F, T)
        d2h = (time.perf_counter() - t0r) * 1e3 / 20
        kern_ms = kms / max(nl, 1)
        per = {k: v * 1e3 / nrec for k, v in rec.items()}
        breakdown = {
            "gpu_step_kernel_ms": kern_ms,
            "gpu_force_reduction_copy_to_host_and_gaps_ms": launches - kern_ms,
            "gpu_position_upload_and_binning_ms": upbin,
            "host_force_read_ms": d2h,
            "host_position_update_ms (overlaps the step)": per["positions"],
            "host_set_positions_call_ms (overlaps the step)": per["set_positions"],
            "host_velocity_update_ms": per["velocities"],
            "host_set_velocities_call_ms": per["set_velocities"],
            "host_step_call_ms": per["step_call"],
            "host_wait_in_get_forces_ms": per["get_forces"],
            "wall_ms": dt * 1e3 / steps,
            "instrumented_wall_ms": sum(rec.values()) * 1e3 / nrec,
            "note": "wall_ms from the timed loop, which has no instrumentation; the other figures from a "
                    "second loop of up to 100 steps: host times around each call, GPU times from events on "
                    "the engine stream (the position upload and re-binning are ordered after the step and "
                    "its force reduction)",
        }
    _, _, ov = eng.get_stats(0)
    kern0 = kernel_ms_without_spheres(eng) if device else None
    eng.close()
    torch.cuda.empty_cache()
    step_ms = dt * 1e3 / steps
    kern = kms / max(nl, 1)
    extra = {} if kern0 is None else {"kernel_ms_no_spheres": kern0, "kernel_over_no_spheres": kern / kern0 - 1.0}
    if not device:
        extra["breakdown"] = breakdown
    return {"cells": spec.N, "spheres": int(len(spec.r)), "steps": steps, "storage": "f32dev",
            "mlups": spec.N * steps / dt / 1e6, "ms_per_step": step_ms, "kernel_ms": kern, **extra,
            "coupling_overhead_frac": (step_ms - kern) / step_ms, "launch": list(shape),
            "slot_overflows_last_map": ov,
            "particle_update": "device explicit Euler (psm_run: graphs of 10 step + update pairs)" if device
                               else "host explicit Euler; positions uploaded while the step runs (re-binned "
                                    "while the host reads the forces, which each step copies to the host), "
                                    "velocities after the force read-back"}


def run_fluidized_bed(psm, torch, inputs, case, steps=200, warmup=5):
    """The paper's fluidized-bed geometry (500 x 200 x 800, FP64, no-slip
    sides, velocity inflow, pressure outflow, spheres of diameter 20) with
    synthetic spheres (627 dilute / 8073 dense), advanced on the GPU each step
    by velocity Verlet (psm_integrate) under gravity minus buoyancy."""
    import numpy as np

    spec, rho_p, accel = inputs.fluidized_bed(case)
    eng = psm.Engine([psm.desc_from_spec(spec, max_radius=10.0)], storage=psm.PSM_FP64)
    with torch.cuda.stream(eng.stream):
        u0 = torch.as_tensor(spec.u0, dtype=torch.float64).to(eng.device)
    eng.set_particles(0, spec.x, spec.r, spec.U, spec.Om)
    eng.set_equilibrium(0, u0)
    shape, _ = eng.autotune(trial_steps=3)
    eng.set_equilibrium(0, u0)
    del u0
    eng.set_particles(0, spec.x, spec.r, spec.U, spec.Om)
    eng.set_dynamics(0, rho_p, accel)
    # kernel time from an eager timed pass, wall time from graph replays
    eng.reset_timing()
    eng.set_timing(True)
    eng.run(warmup + 10, 1.0, psm.PSM_VERLET)
    nl, kms = eng.get_timing()
    eng.set_timing(False)
    eng.set_graph(True)
    eng.run(10, 1.0, psm.PSM_VERLET)
    eng.synchronize()
    t0 = time.perf_counter()
    eng.run(steps, 1.0, psm.PSM_VERLET)
    F, _ = eng.get_forces(0)   # synchronises; reports a device-side list overflow
    dt = time.perf_counter() - t0
    _, _, ov = eng.get_stats(0)
    kern = kms / max(nl, 1)
    # the paper's comparison (Sec. 4.2.1): the same kernel, launch, memory and
    # boundaries with the spheres removed
    kern0 = kernel_ms_without_spheres(eng)
    eng.close()
    torch.cuda.empty_cache()
    return {"case": case, "cells": spec.N, "spheres": int(len(spec.r)), "steps": steps, "storage": "f64",
            "mlups": spec.N * steps / dt / 1e6, "ms_per_step": dt * 1e3 / steps, "kernel_ms": kern,
            "roofline_frac": spec.N * BYTES_PER_CELL[0] / (kern * 1e-3) / 1e9 / HBM_PEAK_GBPS,
            "kernel_ms_no_spheres": kern0, "kernel_over_no_spheres": kern / kern0 - 1.0,
            "launch": list(shape), "slot_overflows_last_map": ov, "forces_finite": bool(np.all(np.isfinite(F))),
            "particle_update": "device velocity Verlet (psm_run: graphs of 10 step + update pairs)"}


def kernel_ms_without_spheres(eng, steps=30):
    """Average step-kernel time of box 0 of `eng` after its spheres are
    removed (eager steps; the PDF state is advanced)."""
    import numpy as np

    eng.set_graph(False)
    eng.set_particles(0, np.zeros((0, 3)), np.zeros(0), np.zeros((0, 3)), np.zeros((0, 3)))
    eng.step(3)
    eng.synchronize()
    eng.reset_timing()
    eng.set_timing(True)
    eng.step(steps)
    eng.synchronize()
    nl, kms = eng.get_timing()
    eng.set_timing(False)
    return kms / max(nl, 1)


def host_cpu():
    """CPU model and the number of cores this process may use."""
    model, fam, mod = "unknown", "?", "?"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                k, _, v = line.partition(":")
                k, v = k.strip(), v.strip()
                if k == "model name" and model == "unknown":
                    model = v
                elif k == "cpu family" and fam == "?":
                    fam = v
                elif k == "model" and mod == "?":
                    mod = v
    except OSError:
        pass
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    return f"{model} (family {fam}, model {mod})", cores


def cpu_baseline(inputs, n, steps, copy_runs=None):
    """The FP64 C oracle as written on the host's cores: single-threaded (the
    build every test uses) and on all cores (the OpenMP timing build of the
    same source) on an n^3 sample of the workload for `steps` steps; then,
    on all cores, the oracle on the 64^3 precision copy (1000 steps), which is
    the reference of the deviation forms' errors in `copy_runs`."""
    import numpy as np
    import oracle

    oracle.build(force=False)
    model, cores = host_cpu()
    spec = inputs.paper_scale(n=n, seed=1)
    box = oracle.Box(*spec.dims, tau=spec.tau, fext=spec.fext)
    f0 = oracle.equilibrium(box, np.zeros((3, spec.N)))
    t0 = time.perf_counter()
    oracle.run(box, f0, steps, spec.x, spec.r, spec.U, spec.Om)
    dt1 = time.perf_counter() - t0
    log(f"  1 thread: {spec.N * steps / dt1 / 1e6:.2f} MLUPS ({dt1:.1f} s)")
    nth = oracle.threads(cores)
    t0 = time.perf_counter()
    oracle.run(box, f0, steps, spec.x, spec.r, spec.U, spec.Om, timing_build=True)
    dtn = time.perf_counter() - t0
    log(f"  {nth} threads: {spec.N * steps / dtn / 1e6:.2f} MLUPS ({dtn:.1f} s)")
    del f0
    out = {"value": spec.N * steps / dtn / 1e6, "unit": "MLUPS", "cores": nth, "kind": "oracle",
           "sample": f"{n}^3 periodic box with the workload's sphere size, solid fraction (0.10, {len(spec.r)} "
                     f"spheres), tau and body force, {steps} FP64 steps; all-core figure from the OpenMP build of "
                     f"the C oracle ({dtn:.1f} s), single-thread figure from the plain build ({dt1:.1f} s)",
           "single_thread": {"value": spec.N * steps / dt1 / 1e6, "cores": 1},
           "host_cpu": model, "host_cores": cores}
    if copy_runs is not None:
        cn, csteps = PRECISION_COPY
        cs = inputs.paper_scale(n=cn, seed=1)
        cbox = oracle.Box(*cs.dims, tau=cs.tau, fext=cs.fext)
        t0 = time.perf_counter()
        ref = oracle.run(cbox, oracle.equilibrium(cbox, np.zeros((3, cs.N))), csteps, cs.x, cs.r, cs.U, cs.Om,
                         timing_build=True)
        dtc = time.perf_counter() - t0
        _, u_ref = oracle.macroscopic(cbox, ref.f)
        errs = {}
        for st, (u, F) in copy_runs.items():
            errs[STORAGE_NAME[st]] = {"l2_u_rel": velocity_error(u, u_ref), "force_rel": force_error(F, ref.F, ref.A)}
        out["precision_copy_oracle"] = {"value": cs.N * csteps / dtc / 1e6, "cores": nth, "seconds": dtc}
        out["_errors_vs_oracle"] = errs
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--size", type=int, default=512)
    ap.add_argument("--launch", type=str, default=None, help="tx,ty,tz,flags (skips the autotuner)")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--retune", action="store_true",
                    help="autotune the main run even where a committed counter run fixes its launch")
    ap.add_argument("--kernel-only", action="store_true", help="time psm_step alone (no upload/readback)")
    ap.add_argument("--no-spheres", action="store_true",
                    help="the main run's box without its spheres (the same fluid workload)")
    ap.add_argument("--storage", choices=list(STORAGE_OF), default="f64",
                    help="storage form of the main run (another than f64 skips the precision-form runs)")
    ap.add_argument("--precision-steps", type=int, default=None, help="steps of the FP32/FP16 runs (default --steps)")
    ap.add_argument("--no-precision", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-size", type=int, default=256)
    ap.add_argument("--cpu-steps", type=int, default=5)
    ap.add_argument("--batched-steps", type=int, default=500)
    ap.add_argument("--dense-steps", type=int, default=500)
    ap.add_argument("--dense-size", type=int, default=768)
    ap.add_argument("--bed-steps", type=int, default=200)
    ap.add_argument("--no-extra", action="store_true", help="skip the batched and dense workloads")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the engine has no multi-GPU path (it would shard the box by "
              "domain decomposition across GPUs). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2303_11811_amd as psm
    from paper_2303_11811_amd import inputs

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    psm.lib()
    launch = tuple(int(v) for v in args.launch.split(",")) if args.launch else None

    def counter_launch(st):
        """The launch of the committed counter run of this storage form (chosen
        by the autotuner in that run), so that the timed launch is the one the
        HBM traffic was counted at; None if the counters are stale."""
        if args.launch or args.retune or args.no_autotune or args.size != 512:
            return None
        _, cl = measured_traffic(st)
        return tuple(cl) if cl else None

    spec = inputs.paper_scale(n=args.size, seed=1)
    log(f"workload: {args.size}^3, {len(spec.r)} spheres, tau {spec.tau}, g {spec.fext[0]}")

    main_st = STORAGE_OF[args.storage]
    if args.no_spheres:
        import numpy as np
        spec.x, spec.r, spec.U, spec.Om = np.zeros((0, 3)), np.zeros(0), np.zeros((0, 3)), np.zeros((0, 3))
    main_launch = launch or counter_launch(main_st)
    log(f"{args.storage} main run" + (f" at the counter run's launch {main_launch}" if main_launch and not launch else ""))
    main_res = run_case(psm, torch, spec, main_st, args.steps, args.warmup, not args.no_autotune, main_launch,
                        full_loop=not args.kernel_only)
    log(f"  {main_res}")

    def traffic_at(st, used_launch):
        traffic, tl = measured_traffic(st)
        return (traffic, tl) if tl is not None and list(tl) == list(used_launch) else (None, tl)

    forms = {}
    copy_runs = None
    if not args.no_precision and main_st == 0:
        psteps = args.precision_steps or args.steps
        for st in (1, 2):
            log(f"{STORAGE_NAME[st]} run")
            r = run_case(psm, torch, spec, st, psteps, args.warmup, not args.no_autotune, counter_launch(st),
                         full_loop=not args.kernel_only)
            r["roofline_frac"] = spec.N * BYTES_PER_CELL[st] / (r["kernel_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBPS
            traffic, traffic_launch = traffic_at(st, r["launch"])
            forms[STORAGE_NAME[st]] = {"mlups": r["mlups"], "ms_per_step": r["ms_per_step"], "steps": psteps,
                                       "kernel_ms": r["kernel_ms"], "launch": r["launch"],
                                       "roofline_frac": r["roofline_frac"],
                                       "pattern_copy": pattern_summary(r, spec.N * BYTES_PER_CELL[st]),
                                       "traffic": traffic, "traffic_launch": traffic_launch,
                                       "speedup_vs_f64": r["mlups"] / main_res["mlups"],
                                       "kernel_speedup_vs_f64": main_res["kernel_ms"] / r["kernel_ms"]}
            log(f"  {forms[STORAGE_NAME[st]]}")
        log("precision copy (64^3, 1000 steps) in the three storage forms")
        copy_runs, err = precision_copy_runs(psm, torch, inputs)
        for k, v in err.items():
            forms[k]["error_vs_gpu_f64_64cubed_1000steps"] = v
        log(f"  vs the GPU FP64 path: {err}")

    extra = {}
    if not args.no_extra:
        log("batched boxes")
        extra["batched"] = run_batched(psm, torch, inputs, steps=args.batched_steps)
        log(f"  {extra['batched']}")
        log("dense moving spheres")
        extra["dense_moving"] = run_dense_moving(psm, torch, inputs, n=args.dense_size, steps=args.dense_steps)
        log(f"  {extra['dense_moving']}")
        for case in ("dilute", "dense"):
            log(f"fluidized bed 500x200x800, {case}")
            extra[f"fluidized_bed_{case}"] = run_fluidized_bed(psm, torch, inputs, case, steps=args.bed_steps)
            log(f"  {extra[f'fluidized_bed_{case}']}")
        log(f"dense moving suspension {args.dense_size}^3, device integrator")
        extra["dense_moving_device"] = run_dense_moving(psm, torch, inputs, n=args.dense_size,
                                                        steps=args.dense_steps, device=True)
        log(f"  {extra['dense_moving_device']}")

    log("stream copy")
    copy_gbps = stream_copy_gbps(psm, torch)
    log(f"  {copy_gbps:.0f} GB/s")

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        cpu = cpu_baseline(inputs, args.cpu_size, args.cpu_steps, copy_runs)
        errs = cpu.pop("_errors_vs_oracle", {})
        for k, v in errs.items():
            if k in forms:
                forms[k]["error_vs_oracle_64cubed_1000steps"] = v
            elif k == "f64":
                forms["f64_error_vs_oracle_64cubed_1000steps"] = v
        log(f"  {cpu}")
        log(f"  errors vs the oracle: {errs}")

    for case in ("dilute", "dense"):
        bed = extra.get(f"fluidized_bed_{case}")
        if bed is not None:
            # the paper's lightspeed (eq. 28) with this box's measured copy rate
            t_min = lightspeed_ms(bed["cells"], 0, copy_gbps)
            bed["lightspeed_ms_at_copy_rate"] = t_min
            bed["kernel_over_lightspeed"] = bed["kernel_ms"] / t_min - 1.0

    algo_bytes = spec.N * BYTES_PER_CELL[main_st]
    achieved = algo_bytes / (main_res["kernel_ms"] * 1e-3) / 1e9
    traffic, traffic_launch = traffic_at(main_st, main_res["launch"])
    form = {0: "FP64", 1: "FP32-deviation storage", 2: "FP16-deviation storage"}[main_st]
    out = {
        "metric": METRIC,
        "value": round(main_res["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(main_res["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[main_st],
        "data": "synthetic",
        "config": {
            "workload": f"PSM-LBM D3Q19 SRT, {args.size}^3 periodic, {form}, tau 0.55, body force 1e-6 +x, "
                        f"{len(spec.r)} spheres d=20 (10% solid), mapping + force/torque every step",
            "cells": spec.N, "spheres": int(len(spec.r)), "storage": args.storage,
            "launch": main_res["launch"],
            "step": "kernel only" if args.kernel_only else
                    "upload spheres (lists rebuilt only when positions change) + fused map/stream-collide/force + reduce + read forces",
        },
        "roofline": {
            "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBPS, 4),
            "traffic": traffic,
            "traffic_launch": traffic_launch,
            "kernel": f"k_psm_step<{args.storage}>", "kernel_ms": round(main_res["kernel_ms"], 4),
            "algorithmic_bytes_per_launch": algo_bytes,
            "frac_of_stream_copy": round(achieved / copy_gbps, 4),
            "pattern_copy": pattern_summary(main_res, algo_bytes),
        },
        "cpu_baseline": cpu,
        "stream_copy_GBps": round(copy_gbps, 1),
        "mlups_frac_of_stream_copy": round(main_res["mlups"] * 1e6 * BYTES_PER_CELL[main_st] / 1e9 / copy_gbps, 4),
        "window_mlups": main_res["window_mlups"],
        "window_mlups_median": round(float(sorted(main_res["window_mlups"])[len(main_res["window_mlups"]) // 2]), 1),
        "precision_forms": forms,
        "other_workloads": extra,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
