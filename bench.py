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
    """Time `steps` coupled steps of one box. Returns a dict of results."""
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
    t0 = time.perf_counter()
    for _ in range(steps):
        one_step()
    eng.synchronize()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    n_launch, kern_ms = eng.get_timing()
    eng.set_timing(False)
    mass, mom, ov = eng.get_stats(0)
    res = dict(ms_per_step=(t1 - t0) * 1e3 / steps, mlups=N * steps / (t1 - t0) / 1e6,
               kernel_ms=kern_ms / max(n_launch, 1), launches=n_launch, launch=list(eng.get_launch()),
               mass=mass, slot_overflows=ov)
    eng.close()
    del eng
    torch.cuda.empty_cache()
    return res


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


def precision_errors(psm, torch, inputs, n=64, steps=1000):
    """L2 velocity error and max relative force error of the deviation
    storage forms against the FP64 path on an n^3 copy of the workload."""
    import numpy as np

    spec = inputs.paper_scale(n=n, seed=1)
    out = {}
    ref = None
    for st in (0, 1, 2):
        eng = psm.Engine([psm.desc_from_spec(spec)], storage=st)
        eng.set_equilibrium(0, np.zeros((3, spec.N)))
        eng.set_particles(0, spec.x, spec.r, spec.U, spec.Om)
        eng.step(steps)
        _, u = eng.get_macroscopic(0)
        F, _ = eng.get_forces(0)
        u = u.cpu().numpy()
        eng.close()
        if st == 0:
            ref = (u, F)
            continue
        l2 = float(np.linalg.norm(u - ref[0]) / np.linalg.norm(ref[0]))
        fe = float(np.max(np.linalg.norm(F - ref[1], axis=1) / np.linalg.norm(ref[1], axis=1)))
        out[STORAGE_NAME[st]] = {"l2_u_rel": l2, "max_force_rel": fe}
    return out


def run_batched(psm, torch, inputs, steps=500, nbox=64):
    """64 independent uneven boxes in one launch per step, FP32 deviation
    storage, replayed as captured 10-step HIP graphs, at the autotuner's
    launch and at the same tile shape on the persistent grid (an
    occupancy-sized grid whose workgroups walk the tiles of all boxes)."""
    import numpy as np

    specs = inputs.batched_boxes(nbox=nbox, seed=3)
    descs = [psm.desc_from_spec(s, max_particles=max(s.n_particles, 1), max_radius=8.0) for s in specs]
    eng = psm.Engine(descs, storage=psm.PSM_FP32DEV)
    for b, s in enumerate(specs):
        if s.n_particles:
            eng.set_particles(b, s.x, s.r, s.U, s.Om)
    for b, s in enumerate(specs):
        eng.set_equilibrium(b, s.u0)
    shape, _ = eng.autotune(trial_steps=10)
    for b, s in enumerate(specs):
        eng.set_equilibrium(b, s.u0)
    eng.set_graph(True)

    def timed():
        eng.step(20)
        eng.synchronize()
        t0 = time.perf_counter()
        eng.step(steps)
        eng.synchronize()
        return time.perf_counter() - t0

    dt = timed()
    cells = sum(s.N for s in specs)
    mass_ok = all(np.isfinite(eng.get_stats(b)[0]) for b in range(len(specs)))
    pshape = (shape[0], shape[1], shape[2], shape[3] | psm.PSM_LAUNCH_PERSISTENT)
    eng.set_launch(*pshape)
    dtp = timed()
    eng.close()
    torch.cuda.empty_cache()
    return {"boxes": len(specs), "cells": cells, "spheres": int(sum(s.n_particles for s in specs)),
            "steps": steps, "mlups": cells * steps / dt / 1e6, "ms_per_step": dt * 1e3 / steps,
            "storage": "f32dev", "launch": list(shape), "graph_steps": 10, "finite": bool(mass_ok),
            "roofline_frac": cells * 152 / (dt / steps) / 1e9 / HBM_PEAK_GBPS,
            "persistent_launch": list(pshape), "mlups_persistent": cells * steps / dtp / 1e6}


def run_dense_moving(psm, torch, inputs, n=768, steps=500, warmup=5, device=False):
    """Moving dense suspension: every step the forces are read back, the
    spheres advance by explicit Euler on the host (density ratio 2.5), are
    uploaded, re-binned and re-mapped. With device=True the same Euler update
    and the re-binning run on the GPU (psm_integrate) with no per-step host
    round trip; the forces are read once at the end."""
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
    mass = 2.5 * 4.0 / 3.0 * np.pi * spec.r ** 3
    inertia = 0.4 * mass * spec.r ** 2
    L = np.asarray(spec.dims, dtype=np.float64)

    def one():
        nonlocal x, U, Om
        eng.set_particles(0, x, spec.r, U, Om)
        eng.step(1)
        F, T = eng.get_forces(0)
        x = np.mod(x + U, L)
        U = U + F / mass[:, None]
        Om = Om + T / inertia[:, None]

    if device:
        # kernel time from an eager timed pass, wall time from graph replays
        # of 10 (step + update) pairs with the host out of the loop
        eng.set_particles(0, x, spec.r, U, Om)
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
        eng.synchronize()
        eng.reset_timing()
        eng.set_timing(True)
        t0 = time.perf_counter()
        for _ in range(steps):
            one()
        dt = time.perf_counter() - t0
        nl, kms = eng.get_timing()
    _, _, ov = eng.get_stats(0)
    kern0 = kernel_ms_without_spheres(eng) if device else None
    eng.close()
    torch.cuda.empty_cache()
    step_ms = dt * 1e3 / steps
    kern = kms / max(nl, 1)
    extra = {} if kern0 is None else {"kernel_ms_no_spheres": kern0, "kernel_over_no_spheres": kern / kern0 - 1.0}
    return {"cells": spec.N, "spheres": int(len(spec.r)), "steps": steps, "storage": "f32dev",
            "mlups": spec.N * steps / dt / 1e6, "ms_per_step": step_ms, "kernel_ms": kern, **extra,
            "coupling_overhead_frac": (step_ms - kern) / step_ms, "launch": list(shape),
            "slot_overflows_last_map": ov,
            "particle_update": "device explicit Euler (psm_run: graphs of 10 step + update pairs)" if device
                               else "host explicit Euler, upload, read-back"}


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


def cpu_baseline(inputs, n, steps):
    import numpy as np
    import oracle

    oracle.build(force=False)
    spec = inputs.paper_scale(n=n, seed=1)
    box = oracle.Box(*spec.dims, tau=spec.tau, fext=spec.fext)
    f0 = oracle.equilibrium(box, np.zeros((3, spec.N)))
    t0 = time.perf_counter()
    oracle.run(box, f0, steps, spec.x, spec.r, spec.U, spec.Om)
    dt = time.perf_counter() - t0
    return {"value": spec.N * steps / dt / 1e6, "unit": "MLUPS", "cores": 1, "kind": "oracle",
            "sample": f"{n}^3 periodic box with the same sphere size, solid fraction (0.10, "
                      f"{len(spec.r)} spheres), tau and body force, {steps} FP64 steps, "
                      f"single-threaded C oracle, {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--size", type=int, default=512)
    ap.add_argument("--launch", type=str, default=None, help="tx,ty,tz,flags (skips the autotuner)")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--kernel-only", action="store_true", help="time psm_step alone (no upload/readback)")
    ap.add_argument("--storage", choices=list(STORAGE_OF), default="f64",
                    help="storage form of the main run (another than f64 skips the precision-form runs)")
    ap.add_argument("--precision-steps", type=int, default=200)
    ap.add_argument("--no-precision", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-size", type=int, default=128)
    ap.add_argument("--cpu-steps", type=int, default=30)
    ap.add_argument("--batched-steps", type=int, default=500)
    ap.add_argument("--dense-steps", type=int, default=200)
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

    spec = inputs.paper_scale(n=args.size, seed=1)
    log(f"workload: {args.size}^3, {len(spec.r)} spheres, tau {spec.tau}, g {spec.fext[0]}")

    main_st = STORAGE_OF[args.storage]
    log(f"{args.storage} main run")
    main_res = run_case(psm, torch, spec, main_st, args.steps, args.warmup, not args.no_autotune, launch,
                        full_loop=not args.kernel_only)
    log(f"  {main_res}")

    forms = {}
    if not args.no_precision and main_st == 0:
        for st in (1, 2):
            log(f"{STORAGE_NAME[st]} run")
            r = run_case(psm, torch, spec, st, args.precision_steps, 10, not args.no_autotune, None,
                         full_loop=not args.kernel_only)
            r["roofline_frac"] = spec.N * BYTES_PER_CELL[st] / (r["kernel_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBPS
            traffic, traffic_launch = measured_traffic(st)
            forms[STORAGE_NAME[st]] = {"mlups": r["mlups"], "ms_per_step": r["ms_per_step"],
                                       "kernel_ms": r["kernel_ms"], "launch": r["launch"],
                                       "roofline_frac": r["roofline_frac"],
                                       "traffic": traffic, "traffic_launch": traffic_launch,
                                       "speedup_vs_f64": r["mlups"] / main_res["mlups"]}
            log(f"  {forms[STORAGE_NAME[st]]}")
        log("precision errors (64^3 copy, 1000 steps, vs the FP64 path)")
        err = precision_errors(psm, torch, inputs)
        for k, v in err.items():
            forms[k]["error_vs_f64_64cubed_1000steps"] = v
        log(f"  {err}")

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
        cpu = cpu_baseline(inputs, args.cpu_size, args.cpu_steps)
        log(f"  {cpu}")

    for case in ("dilute", "dense"):
        bed = extra.get(f"fluidized_bed_{case}")
        if bed is not None:
            # the paper's lightspeed (eq. 28) with this box's measured copy rate
            t_min = lightspeed_ms(bed["cells"], 0, copy_gbps)
            bed["lightspeed_ms_at_copy_rate"] = t_min
            bed["kernel_over_lightspeed"] = bed["kernel_ms"] / t_min - 1.0

    algo_bytes = spec.N * BYTES_PER_CELL[main_st]
    achieved = algo_bytes / (main_res["kernel_ms"] * 1e-3) / 1e9
    traffic, traffic_launch = measured_traffic(main_st)
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
        },
        "cpu_baseline": cpu,
        "stream_copy_GBps": round(copy_gbps, 1),
        "mlups_frac_of_stream_copy": round(main_res["mlups"] * 1e6 * BYTES_PER_CELL[main_st] / 1e9 / copy_gbps, 4),
        "precision_forms": forms,
        "other_workloads": extra,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
