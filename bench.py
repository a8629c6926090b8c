"""Throughput of the site-based suspension LBM hot path on one MI355X.

Workload: D3Q19, 256^3 periodic box, 500 spheres of radius 6 (density ratio
1.2, gravity 1e-6, zero-net-force frame), tau 0.6, distributions stored in
FP32.  A step is the whole hot path (sweep, BS substep + per-particle sums,
particle update, map rebuild, IS substep) over the box.  Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--storage fp32|fp64]
                  [--no-cpu-baseline]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBPS = 8000.0  # MI355X HBM3E


def copy_ceiling(torch, lbm, stream, nbytes=2 << 30, reps=10):
    """Bandwidth of the library's plain device copy (read + write bytes / time)."""
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(2):
        lbm.lbm_device_copy(dst.data_ptr(), src.data_ptr(), nbytes, stream.cuda_stream)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        lbm.lbm_device_copy(dst.data_ptr(), src.data_ptr(), nbytes, stream.cuda_stream)
    e1.record(stream)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    return 2 * nbytes / (ms * 1e-3) / 1e9


def cpu_baseline(cfg, steps):
    """The FP64 oracle on the same box and particles, a bounded number of steps."""
    import oracle
    p = cfg["particles"]
    o = oracle.Oracle(19, *cfg["box"], cfg["tau"], gravity=cfg["gravity"], zero_net_force=True)
    o.add_particles(p["x"], radius=p["radius"], mass=p["mass"], inertia=p["inertia"])
    t0 = time.perf_counter()
    o.step(steps)
    dt = time.perf_counter() - t0
    N = cfg["box"][0] * cfg["box"][1] * cfg["box"][2]
    o.close()
    return {"value": N * steps / dt / 1e6, "unit": "MLUPS", "cores": 1, "kind": "oracle",
            "sample": "%d steps of the full 256^3 D3Q19 box with 500 spheres (FP64, one thread), %.1f s"
                      % (steps, dt)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--storage", default="fp32", choices=["fp32", "fp64", "fp16", "bf16"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=2)
    ap.add_argument("--particles", type=int, default=-1,
                    help="particles in the box (default: the workload's; fewer only to measure overheads)")
    ap.add_argument("--workload", default="spheres-3d", choices=["spheres-3d", "disks-2d"],
                    help="spheres-3d: D3Q19 256^3, 500 spheres (the headline); "
                         "disks-2d: D2Q9 1024^2, 200 disks")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the slab decomposition across GPUs is a design, not code)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1105_2904_amd import lbm
    from paper_1105_2904_amd import workloads as wl

    torch.cuda.set_device(0)
    cfg = wl.spheres_3d_config(storage=args.storage) if args.workload == "spheres-3d" else wl.disks_2d_config()
    q = cfg["q"]
    if args.particles < 0:
        args.particles = len(cfg["particles"]["radius"])
    p = {k: v[:args.particles] for k, v in cfg["particles"].items()}
    nx, ny, nz = cfg["box"]
    N = nx * ny * nz
    sim = lbm.Simulation(q, nx, ny, nz, tau=cfg["tau"], gravity=cfg["gravity"], zero_net_force=True,
                         storage=args.storage, max_particles=max(len(p["radius"]), 1),
                         max_radius=float(np.max(cfg["particles"]["radius"])))
    if args.particles:
        sim.add_particles(p["x"], radius=p["radius"], mass=p["mass"], inertia=p["inertia"])
    bps = lbm.lbm_bytes_per_site(sim.params)
    stream = sim.stream

    sim.step(args.warmup)
    torch.cuda.synchronize()
    print("warmup done (%d steps)" % args.warmup, file=sys.stderr, flush=True)

    sim.set_profiling(True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    sim.step(args.steps)
    e1.record(stream)
    e1.synchronize()
    torch.cuda.synchronize()
    ms_total = e0.elapsed_time(e1)
    sweep_ms, sweeps = sim.profile()
    sim.set_profiling(False)
    F = sim.forces()[0]
    assert F.shape == (args.particles, 3) and np.isfinite(F).all()

    ms_step = ms_total / args.steps
    mlups = N / (ms_step * 1e-3) / 1e6
    sweep_avg_ms = sweep_ms / max(sweeps, 1)
    achieved = bps * N / (sweep_avg_ms * 1e-3) / 1e9
    ceiling = copy_ceiling(torch, lbm, stream)
    out = {
        "metric": "MLUPS + % HBM roofline, D3Q19 256³ 500 spheres; FP16-store/batched vs FP32",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "f32", "fp64": "f64", "fp16": "f16-store/f32", "bf16": "bf16-store/f32"}[args.storage],
        "data": "synthetic",
        "config": {"workload": cfg["name"], "lattice": "D3Q19" if q == 19 else "D2Q9", "box": [nx, ny, nz],
                   "tau": cfg["tau"], "particles": args.particles,
                   "radius": float(np.max(cfg["particles"]["radius"])),
                   "density_ratio": 1.2 if q == 19 else 1.5, "gravity": float(-min(cfg["gravity"])),
                   "storage": args.storage, "parallelism": "single-gpu"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBPS, "unit": "GB/s",
                     "frac": round(achieved / PEAK_HBM_GBPS, 4), "traffic": None,
                     "kernel": "k_sweep<%d,%s>" % (q, {"fp32": "float", "fp64": "double", "fp16": "_Float16",
                                                      "bf16": "bf16s"}[args.storage]),
                     "kernel_avg_ms": round(sweep_avg_ms, 4), "bytes_per_site": bps},
        "step_roofline_frac": round(bps * mlups * 1e6 / 1e9 / PEAK_HBM_GBPS, 4),
        "copy_ceiling_GBps": round(ceiling, 1),
    }
    if not args.no_cpu_baseline and args.workload == "spheres-3d":
        print("cpu baseline: %d oracle steps" % args.cpu_steps, file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(cfg, args.cpu_steps)
    print(json.dumps(out), flush=True)
    sim.close()


if __name__ == "__main__":
    main()
