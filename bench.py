"""Throughput of the site-based suspension LBM hot path on one MI355X.

Workload: D3Q19, 256^3 periodic box, 500 spheres of radius 6 (density ratio
1.2, gravity 1e-6, zero-net-force frame), tau 0.6, distributions stored in
FP32.  A step is the whole hot path (sweep, BS substep + per-particle sums,
particle update, map rebuild, IS substep) over the box.  Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--storage fp32|fp64|fp16|bf16]
                  [--no-cpu-baseline] [--no-variants] [--no-autotune] [--workload spheres-3d|disks-2d]
                  [--accuracy-steps N] [--no-batched] [--no-disks-2d]

The FP32 run also times the FP16 and BF16 storage variants of the same
workload ("variants") and, outside every timed region, runs the workload for
--accuracy-steps steps in FP64, FP32, FP16 and BF16 to give each variant its
drag and settling-velocity error against FP64 ("accuracy"); it times a 64-box
D2Q9 ensemble stepped by one launch per kernel with a tuned sweep shape and
step graphs against a loop of one-box contexts ("batched"), and the FP64
oracle on a few steps of the same box ("cpu_baseline").  copy_ceiling_GBps is
the library's 2 GiB device copy with the faster of its two load kinds (and,
for a population footprint that fits the last-level cache, the same copy at
that footprint: copy_ceiling_cache_resident_GBps).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBPS = 8000.0  # MI355X HBM3E
MALL_BYTES = 256 << 20  # MI355X last-level (Infinity) cache
COUNTERS = os.path.join(ROOT, "profiles", "k_sweep_d3q19_256cubed_500spheres_hbm_counters.json")


def pair_rows(tname, layout, nx):
    """True when the row kernel of this storage takes two sites per lane
    (16-bit storage, two arrays, an even row length)."""
    return tname in ("_Float16", "bf16s") and layout == "0" and nx % 2 == 0


def sweep_geometry(box, launch, pairs=False):
    """Workgroup size and grid (threads) of the sweep launch (width, grid,
    blocks_per_cu) on one box: the row kernel runs 256-wide workgroups over
    ceil(nx/256) blocks per row, or with two sites per lane one 64-lane wave
    per 128 sites of a row, four waves to a workgroup; tiles are w
    consecutive sites of the box, one per workgroup unless a smaller
    persistent grid is set."""
    import math
    nx, ny, nz = box
    w, g = launch["width"], launch["grid"]
    if w == 0 and pairs:
        return 256, math.ceil(math.ceil(nx / 128) * ny * nz / 4) * 256
    if w == 0:
        return 256, math.ceil(nx / 256) * ny * nz * 256
    nt = math.ceil(nx * ny * nz / w)
    return w, (g if 0 < g < nt else nt) * w


def sweep_kernel(width, q, tname, particles, layout, nx):
    """Name of a one-box sweep kernel as the profiler lists it: the row kernel
    (width 0; k_sweep_pairs where it takes two sites per lane) or the tile
    kernel with streaming loads."""
    part = "true" if particles else "false"
    if width == 0 and pair_rows(tname, layout, nx):
        return "k_sweep_pairs<%d,%s,%s>" % (q, tname, part)
    if width == 0:
        return "k_sweep<%d,%s,%s,%s>" % (q, tname, part, layout)
    return "k_sweep_tiles<%d,%s,%s,%s,true>" % (q, tname, part, layout)


def measured_traffic(kernel, workload, box, launch):
    """HBM bytes per launch of `kernel` at this launch geometry from the
    committed FETCH_SIZE/WRITE_SIZE counter runs (copy-kernel calibrated), or
    None when no run covers it or the kernel sources changed since."""
    import hashlib
    try:
        with open(COUNTERS) as fh:
            c = json.load(fh)
    except OSError:
        return None
    if c["workload"] != workload:
        return None
    h = hashlib.sha256()
    for f in c["sources"]:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest() != c["source_sha256"]:
        return None
    wg, grid = sweep_geometry(box, launch, pairs=kernel.startswith("k_sweep_pairs"))
    col = {k: i for i, k in enumerate(c["columns"])}
    for e in c["entries"]:
        if (e[col["kernel"]], e[col["workgroup_size"]], e[col["grid_threads"]]) == (kernel, wg, grid):
            rd, wr = e[col["hbm_read_bytes"]], e[col["hbm_write_bytes"]]
            return {"read": rd, "write": wr, "total": rd + wr}
    return None


def copy_ceiling(torch, lbm, stream, nbytes=2 << 30, reps=10):
    """Bandwidth of the library's device copy (read + write bytes / time),
    the faster of its two load kinds: streaming loads win from HBM, plain
    loads from the last-level cache."""
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    best = 0.0
    for streaming in (True, False):
        for _ in range(2):
            lbm.lbm_device_copy(dst.data_ptr(), src.data_ptr(), nbytes, stream.cuda_stream, streaming)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            lbm.lbm_device_copy(dst.data_ptr(), src.data_ptr(), nbytes, stream.cuda_stream, streaming)
        e1.record(stream)
        e1.synchronize()
        ms = e0.elapsed_time(e1) / reps
        best = max(best, 2 * nbytes / (ms * 1e-3) / 1e9)
    del src, dst
    return best


def storage_accuracy(lbm, cfg, steps):
    """The same workload run for `steps` steps (outside any timed region) in
    FP64, FP32, FP16 and BF16 storage: the velocity field (relative L2 norm
    of the difference), the per-sphere drag and the mean settling velocity of
    each against the FP64 run.  The reference is the GPU's FP64 path, which
    matches the FP64 oracle to 1e-12 wherever the oracle has followed it (the
    oracle itself would take hours for 2000 steps of this box)."""
    p = cfg["particles"]
    res = {}
    u64 = None
    for st in ("fp64", "fp32", "fp16", "bf16"):
        sim = lbm.Simulation(19, *cfg["box"], tau=cfg["tau"], gravity=cfg["gravity"], zero_net_force=True,
                             storage=st, max_particles=len(p["radius"]), max_radius=float(np.max(p["radius"])))
        sim.add_particles(p["x"], radius=p["radius"], mass=p["mass"], inertia=p["inertia"])
        sim.set_graph(50)
        sim.step(steps)
        F, _, _, u, _ = sim.forces()
        uf = sim.fields()[1]
        sim.close()
        if u64 is None:
            u64 = uf
            ev = 0.0
        else:
            ev = float(np.linalg.norm(uf - u64) / np.linalg.norm(u64))
        del uf
        res[st] = (F, u[:, 2].mean(), ev)
    F64, w64, _ = res["fp64"]
    scale = float(np.linalg.norm(F64, axis=1).max())
    out = {"reference": {"storage": "fp64", "path": "GPU FP64 (oracle-matched)", "steps": steps,
                         "mean_settling_velocity": w64, "max_drag": scale,
                         "velocity_field_l2": float(np.linalg.norm(u64))}}
    for st in ("fp32", "fp16", "bf16"):
        F, w, ev = res[st]
        out[st] = {"velocity_field_error_vs_fp64": ev,
                   "drag_error_vs_fp64": float(np.linalg.norm(F - F64, axis=1).max() / scale),
                   "settling_error_vs_fp64": float(abs(w - w64) / abs(w64)), "accuracy_steps": steps}
    return out


def disks_2d_rates(torch, lbm, wl, steps, warmup, graph_steps=20):
    """The D2Q9 1024^2 workload with 200 disks (FP32): the launch tuned in
    whole steps, replayed in step graphs.  Its two population arrays (75 MB) fit the
    256 MB last-level cache, so its ceiling is a copy of the same footprint."""
    cfg = wl.disks_2d_config()
    p = cfg["particles"]
    nx, ny, nz = cfg["box"]
    N = nx * ny * nz
    sim = lbm.Simulation(9, nx, ny, nz, tau=cfg["tau"], gravity=cfg["gravity"], zero_net_force=True,
                         storage="fp32", max_particles=len(p["radius"]), max_radius=float(np.max(p["radius"])))
    sim.add_particles(p["x"], radius=p["radius"], mass=p["mass"], inertia=p["inertia"])
    sim.step(warmup)
    sim.set_graph(graph_steps)  # the tuner then times whole graphs
    w, g, k, _, _ = sim.autotune_steps(steps=graph_steps)
    sim.step(max(warmup, graph_steps))
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(sim.stream)
    sim.step(steps)
    e1.record(sim.stream)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / steps
    assert np.isfinite(sim.forces()[0]).all()
    bps = lbm.lbm_bytes_per_site(sim.params)
    sim.close()
    footprint = bps * N
    cache = copy_ceiling(torch, lbm, torch.cuda.current_stream(), nbytes=footprint // 32 * 16, reps=200)
    gbps = bps * N / (ms * 1e-3) / 1e9
    return {"workload": cfg["name"], "value": round(N / (ms * 1e-3) / 1e6, 1), "unit": "MLUPS",
            "ms_per_step": round(ms, 5), "steps": steps, "graph_steps": graph_steps,
            "sweep_launch": {"width": w, "grid": g, "blocks_per_cu": k}, "bytes_per_site": bps,
            "step_GBps": round(gbps, 1), "step_frac_of_hbm_peak": round(gbps / PEAK_HBM_GBPS, 4),
            "copy_ceiling_cache_resident_GBps": round(cache, 1),
            "step_frac_of_cache_resident_copy": round(gbps / cache, 4)}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(cfg, steps_one, steps_all):
    """The FP64 oracle on the same box and particles, a bounded number of
    steps on one thread and on the host's share of cores (its per-site loops
    run on OpenMP threads with the same bits as one thread)."""
    import oracle
    p = cfg["particles"]
    N = cfg["box"][0] * cfg["box"][1] * cfg["box"][2]

    def run(threads, steps):
        oracle.set_threads(threads)
        o = oracle.Oracle(19, *cfg["box"], cfg["tau"], gravity=cfg["gravity"], zero_net_force=True)
        o.add_particles(p["x"], radius=p["radius"], mass=p["mass"], inertia=p["inertia"])
        used = oracle.threads()
        t0 = time.perf_counter()
        o.step(steps)
        dt = time.perf_counter() - t0
        o.close()
        return N * steps / dt / 1e6, dt, used

    one, dt1, _ = run(1, steps_one)
    allc, dta, used = run(0, steps_all)
    oracle.set_threads(0)
    return {"value": allc, "unit": "MLUPS", "cores": used, "kind": "oracle",
            "sample": "%d steps of the full 256^3 D3Q19 box with 500 spheres (FP64) on %d threads, %.1f s"
                      % (steps_all, used, dta),
            "single_thread": {"value": one, "unit": "MLUPS", "cores": 1,
                              "sample": "%d steps of the same box on one thread, %.1f s" % (steps_one, dt1)},
            "cpu_model": cpu_model(), "nproc": os.cpu_count()}


def ensemble_rates(torch, lbm, wl, steps, warmup, graph_steps=20):
    """The 64-box D2Q9 ensemble (seeded sides 128..512, 10..80 disks of radius
    6..12): MLUPS of one ensemble context with eager launches, of the same
    context after tuning its launch in whole steps and with step graphs, and of a loop over 64
    one-box contexts (each box's steps launched back to back)."""
    cfg = wl.ensemble_2d_config()
    dims = [tuple(int(v) for v in d) for d in cfg["boxes"]]
    NT = int(np.prod(cfg["boxes"], axis=1).sum())
    npart = sum(len(p["radius"]) for p in cfg["particles"])
    kw = dict(tau=cfg["tau"], gravity=cfg["gravity"], zero_net_force=True, storage="fp32", max_radius=12.0)

    def clock(fn):
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        e1.synchronize()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1)

    ens = lbm.Simulation(9, 1, 1, 1, max_particles=npart, boxes=dims, **kw)
    for b, p in enumerate(cfg["particles"]):
        ens.add_particles(p["x"], radius=p["radius"], mass=p["mass"], inertia=p["inertia"], box=b)
    ens.step(warmup)
    ms_eager = clock(lambda: ens.step(steps))
    ens.set_graph(graph_steps)  # the tuner then times whole graphs
    width, grid, occ, _, _ = ens.autotune_steps(steps=graph_steps)
    ens.step(max(warmup, graph_steps))
    ms_graph = clock(lambda: ens.step(steps))
    assert np.isfinite(ens.forces()[0]).all()
    ens.close()
    singles = []
    for d, p in zip(dims, cfg["particles"]):
        s1 = lbm.Simulation(9, *d, max_particles=len(p["radius"]), **kw)
        s1.add_particles(p["x"], radius=p["radius"], mass=p["mass"], inertia=p["inertia"])
        s1.step(warmup)
        singles.append(s1)

    def loop():
        for s1 in singles:
            s1.step(steps)
    ms_loop = clock(loop)
    for s1 in singles:
        s1.close()
    rate = lambda ms: NT * steps / (ms * 1e-3) / 1e6
    return {"workload": cfg["name"], "boxes": len(dims), "sites": NT, "particles": npart,
            "clipped_particles": int(sum(cfg["clipped"])), "steps": steps,
            "value": round(rate(ms_graph), 1), "unit": "MLUPS",
            "ms_per_step": round(ms_graph / steps, 4),
            "eager_one_launch_per_kernel": round(rate(ms_eager), 1),
            "loop_of_single_boxes": round(rate(ms_loop), 1),
            "speedup_vs_loop": round(ms_loop / ms_graph, 2),
            "tuned_sweep_shape": {"tile_width": width, "grid": grid, "blocks_per_cu": occ},
            "graph_steps": graph_steps,
            "step_roofline_frac": round(72 * rate(ms_graph) * 1e6 / 1e9 / PEAK_HBM_GBPS, 4)}


def closure_mlp_rates(torch, lbm, rows=1 << 22, reps=20, train_steps=2000):
    """Forward rate of the closure network's MFMA kernel on `rows` random
    inputs, and Adam steps per second of the training kernel (256-row
    batches).  Algorithmic FLOPs per row: 2 (8*64 + 64*64 + 64*2) = 9472."""
    from paper_1105_2904_amd import workloads as wl
    g = torch.Generator(device="cuda").manual_seed(5)
    x = (torch.rand((rows, 8), device="cuda", generator=g) * 2 - 1).contiguous()
    t = (torch.rand((rows, 2), device="cuda", generator=g) - 0.5).contiguous()
    p = torch.tensor(wl.mlp_init(3).astype(np.float32), device="cuda")
    lbm.mlp_forward(p, x)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        lbm.mlp_forward(p, x)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    m, v = torch.zeros_like(p), torch.zeros_like(p)
    xs, ts = x[:65536].contiguous(), t[:65536].contiguous()
    lbm.mlp_train(p, m, v, xs, ts, batch=256, steps=10)
    torch.cuda.synchronize()
    e0.record()
    lbm.mlp_train(p, m, v, xs, ts, batch=256, steps=train_steps, step0=10)
    e1.record()
    e1.synchronize()
    tms = e0.elapsed_time(e1)
    tflops = 9472.0 * rows / (ms * 1e-3) / 1e12
    return {"kernel": "k_mlp_forward", "rows": rows, "forward_ms": round(ms, 4),
            "rows_per_s": round(rows / (ms * 1e-3), 1), "achieved_tflops": round(tflops, 2),
            "peak_tflops_fp16_mfma": 2500.0, "frac_of_mfma_peak": round(tflops / 2500.0, 4),
            "train_steps_per_s": round(train_steps / (tms * 1e-3), 1), "train_batch": 256}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--storage", default="fp32", choices=["fp32", "fp64", "fp16", "bf16"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=3, help="oracle steps on one thread")
    ap.add_argument("--cpu-steps-all", type=int, default=12, help="oracle steps on all the host's cores")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip timing the FP16/BF16 storage variants of the same workload")
    ap.add_argument("--particles", type=int, default=-1,
                    help="particles in the box (default: the workload's; fewer only to measure overheads)")
    ap.add_argument("--workload", default="spheres-3d", choices=["spheres-3d", "disks-2d"],
                    help="spheres-3d: D3Q19 256^3, 500 spheres (the headline); "
                         "disks-2d: D2Q9 1024^2, 200 disks")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default sweep launch instead of the autotuner's pick")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip timing the 64-box D2Q9 ensemble (batched) variant")
    ap.add_argument("--batched-steps", type=int, default=200)
    ap.add_argument("--no-disks-2d", action="store_true",
                    help="skip timing the D2Q9 1024^2 workload with 200 disks (disks_2d)")
    ap.add_argument("--accuracy-steps", type=int, default=2000,
                    help="steps of the storage-accuracy leg (FP32/FP16/BF16 against FP64; 0 skips it)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
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

    def timed(sim_, steps, warmup, profile):
        """Whole-step time of `steps` uninstrumented steps and, with profile,
        the summed time and count of the sweep launches of a further
        min(steps, 100) steps bracketed by HIP events on the sim's stream (the
        events cost about 1 % of a step, so they stay out of the step time).
        Unless --no-autotune, the library's in-step tuner picks the sweep
        launch after the warm-up (its steps are further warm-up), outside the
        timed region."""
        sim_.step(warmup)
        if not args.no_autotune:
            sim_.autotune_steps(steps=16)
            sim_.step(2)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(sim_.stream)
        sim_.step(steps)
        e1.record(sim_.stream)
        e1.synchronize()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        sw = None
        if profile:
            sim_.set_profiling(True)
            sim_.step(min(steps, 100))
            sw = sim_.profile()
            sim_.set_profiling(False)
        F_ = sim_.forces()[0]
        assert F_.shape == (args.particles, 3) and np.isfinite(F_).all()
        return ms, sw

    ms_total, (sweep_ms, sweeps) = timed(sim, args.steps, args.warmup, True)
    print("timed %d steps" % args.steps, file=sys.stderr, flush=True)
    ms_step = ms_total / args.steps
    mlups = N / (ms_step * 1e-3) / 1e6
    kname = {"fp32": "float", "fp64": "double", "fp16": "_Float16", "bf16": "bf16s"}[args.storage]
    sweep_avg_ms = sweep_ms / max(sweeps, 1)
    achieved = bps * N / (sweep_avg_ms * 1e-3) / 1e9
    ceiling = copy_ceiling(torch, lbm, stream)
    # a population footprint (both arrays) that fits the 256 MB last-level cache
    # streams from there, not from HBM: its ceiling is a copy of the same size
    footprint = bps * N
    cache_ceiling = None
    if footprint <= MALL_BYTES * 3 // 4:
        cache_ceiling = copy_ceiling(torch, lbm, stream, nbytes=footprint // 32 * 16, reps=200)
    launch = dict(zip(("width", "grid", "blocks_per_cu"), sim.sweep_config()))
    kernel = sweep_kernel(launch["width"], q, kname, bool(args.particles), "0", nx)
    traffic = None
    if args.particles == len(cfg["particles"]["radius"]):
        traffic = measured_traffic(kernel.replace(",", ", "), cfg["name"], cfg["box"], launch)
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
                   "storage": args.storage, "parallelism": "single-gpu",
                   "sweep_launch": launch},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBPS, "unit": "GB/s",
                     "frac": round(achieved / PEAK_HBM_GBPS, 4),
                     "traffic": None if traffic is None else traffic["total"],
                     "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                     "traffic_read_write": None if traffic is None else [traffic["read"], traffic["write"]],
                     "algorithmic_bytes_per_launch": bps * N,
                     "kernel": kernel, "kernel_avg_ms": round(sweep_avg_ms, 4), "sites_per_launch": N,
                     "bytes_per_site": bps,
                     "sweep_frac": round(achieved / PEAK_HBM_GBPS, 4),
                     "step_achieved": round(bps * N / (ms_step * 1e-3) / 1e9, 1),
                     "step_frac": round(bps * mlups * 1e6 / 1e9 / PEAK_HBM_GBPS, 4)},
        "step_roofline_frac": round(bps * mlups * 1e6 / 1e9 / PEAK_HBM_GBPS, 4),
        "copy_ceiling_GBps": round(ceiling, 1),
    }
    if cache_ceiling is not None:
        out["copy_ceiling_cache_resident_GBps"] = round(cache_ceiling, 1)
        out["population_bytes_both_arrays"] = footprint
    if not args.no_variants and args.storage == "fp32":
        out["variants"] = {}
        sim.close()
        for name in ("fp16", "bf16", "fp32_aa"):
            st, aa = ("fp32", True) if name == "fp32_aa" else (name, False)
            v = lbm.Simulation(q, nx, ny, nz, tau=cfg["tau"], gravity=cfg["gravity"], zero_net_force=True,
                               storage=st, max_particles=max(len(p["radius"]), 1),
                               max_radius=float(np.max(cfg["particles"]["radius"])), aa=aa)
            if args.particles:
                v.add_particles(p["x"], radius=p["radius"], mass=p["mass"], inertia=p["inertia"])
            vms, (vsw, vn) = timed(v, args.steps, args.warmup, True)
            vb = lbm.lbm_bytes_per_site(v.params)
            vl = dict(zip(("width", "grid", "blocks_per_cu"), v.sweep_config()))
            tn = {"fp16": "_Float16", "bf16": "bf16s", "fp32": "float"}[st]
            # the AA pattern alternates two sweep kernels (layouts 1 and 2)
            halves = ["1", "2"] if aa else ["0"]
            vks = [sweep_kernel(vl["width"], q, tn, bool(args.particles), h, nx).replace(",", ", ") for h in halves]
            vk = vks[0] if not aa else sweep_kernel(vl["width"], q, tn, bool(args.particles), "1/2", nx)
            vt = None
            if args.particles == len(cfg["particles"]["radius"]):
                ts = [measured_traffic(k_, cfg["name"], cfg["box"], vl) for k_ in vks]
                if all(t_ is not None for t_ in ts):
                    vt = {"total": sum(t_["total"] for t_ in ts) / len(ts)}
            vm = N / (vms / args.steps * 1e-3) / 1e6
            vs = vsw / max(vn, 1)
            out["variants"][name] = {"value": round(vm, 1), "ms_per_step": round(vms / args.steps, 4),
                                   "sweep_launch": vl, "kernel": vk.replace(", ", ","),
                                   "traffic": None if vt is None else vt["total"],
                                   "speedup_vs_fp32": round(vm / mlups, 3), "bytes_per_site": vb,
                                   "sweep_avg_ms": round(vs, 4), "sweep_GBps": round(vb * N / (vs * 1e-3) / 1e9, 1)}
            v.close()
            if aa:
                out["variants"][name]["population_bytes"] = int(q * N * 4)
                out["variants"][name]["population_bytes_two_arrays"] = int(2 * q * N * 4)
            print("variant %s timed" % name, file=sys.stderr, flush=True)
        if args.accuracy_steps > 0 and args.workload == "spheres-3d" and args.particles:
            acc = storage_accuracy(lbm, cfg, args.accuracy_steps)
            out["accuracy"] = acc["reference"]
            for name in ("fp16", "bf16"):
                out["variants"][name].update(acc[name])
            out["accuracy"]["fp32"] = acc["fp32"]
            print("storage accuracy measured", file=sys.stderr, flush=True)
    if not args.no_batched and args.storage == "fp32" and args.workload == "spheres-3d":
        out["closure_mlp"] = closure_mlp_rates(torch, lbm)
        print("closure network timed", file=sys.stderr, flush=True)
        out["batched"] = ensemble_rates(torch, lbm, wl, args.batched_steps, args.warmup)
        print("batched ensemble timed", file=sys.stderr, flush=True)
        if not args.no_disks_2d:
            out["disks_2d"] = disks_2d_rates(torch, lbm, wl, 2000, args.warmup)
            print("D2Q9 1024^2 workload timed", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline and args.workload == "spheres-3d":
        print("cpu baseline: %d + %d oracle steps" % (args.cpu_steps, args.cpu_steps_all), file=sys.stderr,
              flush=True)
        out["cpu_baseline"] = cpu_baseline(cfg, args.cpu_steps, args.cpu_steps_all)
    print(json.dumps(out), flush=True)
    sim.close()


if __name__ == "__main__":
    main()
