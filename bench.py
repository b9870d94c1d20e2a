"""Benchmark of the fused lattice ES-BGK step on one MI355X.

Workload (the configuration the headline metric is quoted on): 2-D
force-driven Poiseuille flow with thermal walls, 1024 x 1024 cells, D2Q37
(Hermite order 4), periodic in x, diffuse walls in y at T = 1.0 / 1.05,
g_x = 1e-5 in lattice units, Kn = 0.05, Pr = 2/3, populations stored as FP32
deviations and collided in FP32. One "step" is one launch of the fused pull +
collide kernel over all cells, with the populations resident in HBM.

Printed: one JSON line with MLUPS (the metric), the roofline of the step
kernel (algorithmic bytes 2 Q s per cell update / measured kernel time
against the 8 TB/s HBM peak), the same workload with plain FP64 and with
FP16 storage, the batched-channel workload in one persistent launch against
a per-problem FP64 loop, the same channel at Pr = 1, the 1 x 32 Couette
channel in FP64 (latency-bound), 3-D workloads (the 256^3 box in FP32,
FP16 and FP64; the 512 x 512 x 256 FP16 channel), the paper's own TVD
scheme on the 6-point Gauss-Hermite set (1024 x 1024, FP32 and FP64), and
its 4- and 8-point sets (D2Q16, D2Q64) in FP32, its 3-D set D3Q216 on a
128^3 box in FP32, and the FP64 CPU oracle timed on a bounded sample.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--only-main]
"""

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_step_traffic_poiseuille1024.json")
PAIR_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_pair_traffic_poiseuille1024.json")
TVD_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_tvd_traffic_periodic1024.json")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def make_lattice(cfg, storage):
    from paper_1209_6548_amd import Lattice
    dims = tuple(cfg["dims"]) + (1,) * (3 - len(cfg["dims"]))
    lat = Lattice(cfg["velset"], dims[0], dims[1], dims[2], walls=cfg["walls"], storage=storage)
    lat.set_gas(cfg["Kn"], cfg["Pr"], cfg["varpi"])
    if cfg["walls"]:
        lat.set_wall(0, cfg["T_w"][0], cfg["u_w"][0])
        lat.set_wall(1, cfg["T_w"][1], cfg["u_w"][1])
    lat.set_body_force(cfg["g"])
    lat.init_equilibrium()
    return lat


def time_steps(lat, steps, warmup):
    """Average step time (ms) from HIP events on the stream the kernels run on
    (torch's current stream, which the binding hands to the library). Before
    the warmup steps, one untimed run of the graph length captures the step
    graphs (of the lattice path; the TVD path launches directly), so that
    their capture falls outside the timed region; an even K up to 64 is the
    graph length itself (the timed steps are one replay)."""
    import torch
    if hasattr(lat, "set_graph_steps"):
        g = steps if steps % 2 == 0 and 2 <= steps <= 64 else 32
        lat.set_graph_steps(g)
        lat.step(g)
    lat.step(warmup)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    lat.step(steps)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def bench_single(cfg, storage, steps, warmup, inplace=2):
    lat = make_lattice(cfg, storage)
    lat.set_inplace(inplace)
    ms = time_steps(lat, steps, warmup)
    cells = int(np.prod(cfg["dims"]))
    s = {"f64": 8, "f32": 4, "f16": 2}[storage]
    bytes_per_step = 2 * lat.Q * s * cells
    out = dict(storage=storage, ms_per_step=ms, mlups=cells / (ms * 1e-3) / 1e6,
               algorithmic_GBs=bytes_per_step / (ms * 1e-3) / 1e9, bytes_per_cell=2 * lat.Q * s,
               in_place_pairs=lat.inplace_active)
    red = lat.reduce()
    out["finite"] = bool(np.isfinite(red["mass"]) and np.isfinite(red["energy"]))
    lat.close()
    return out


TVD_CFG = dict(name="periodic_gas_1024x1024_d2q36", dims=(1024, 1024), Kn=0.05, Pr=2 / 3, cfl=0.45)


def bench_tvd(storage, steps, warmup, velset="D2Q36GH", dims=None):
    """The paper's own scheme (forward Euler, TVD minmod fluxes) on a
    Gauss-Hermite product set (the paper's D2Q36 by default), 1024 x 1024
    periodic cells (or dims, 3-D for D3Q216GH), from a perturbed equilibrium
    (the kernel's work does not depend on the state: the limiter branches
    are selects)."""
    from paper_1209_6548_amd import TVDLattice
    dims = tuple(dims or TVD_CFG["dims"])
    nx, ny = dims[0], dims[1]
    nz = dims[2] if len(dims) > 2 else 1
    # forward Euler on collision and advection together stays bounded while the sum of
    # |nu| over the axes the field varies along is at most 1 - dt/tau: 0.9 in 2-D and 3-D
    cfl = TVD_CFG["cfl"] if nz == 1 else 0.3
    lat = TVDLattice(nx, ny, nz=nz, storage=storage, cfl=cfl, velset=velset)
    Q = lat.Q
    lat.set_gas(TVD_CFG["Kn"], TVD_CFG["Pr"])
    lat.set_body_force((1e-3, 0.0, 0.0))
    rng = np.random.default_rng(1)
    lat.init_equilibrium(noise=rng.standard_normal((Q, nx * ny * nz)), amplitude=1e-3)
    ms = time_steps(lat, steps, warmup)
    cells = nx * ny * nz
    s = {"f64": 8, "f32": 4, "f16": 2}[storage]
    m = lat.read_moments()
    traffic = measured_traffic(storage, TVD_TRAFFIC_FILE) if velset == "D2Q36GH" else None
    name = TVD_CFG["name"].replace("d2q36", velset.lower())
    if dims != tuple(TVD_CFG["dims"]):
        name = f"periodic_gas_{'x'.join(map(str, dims))}_{velset.lower()}"
    out = dict(workload=name, storage=storage, cfl=round(cfl, 4), ms_per_step=ms,
               mlups=cells / (ms * 1e-3) / 1e6, algorithmic_GBs=2 * Q * s * cells / (ms * 1e-3) / 1e9,
               bytes_per_cell=2 * Q * s, kernel=f"k_tvd<{velset}, {storage}>", traffic=traffic,
               traffic_over_algorithmic=round(traffic / (2 * Q * s * cells), 4) if traffic else None,
               finite=bool(np.isfinite(m["rho"]).all()))
    lat.close()
    return out


def bench_couette_persistent(cfg, steps):
    """The 1 x 32 Couette channel as a batch of one: all steps in one
    persistent launch instead of one launch per step."""
    import torch

    from paper_1209_6548_amd import Batch, make_problem
    p = make_problem(cfg["velset"], cfg["dims"][0], cfg["dims"][1], storage="f64", Kn=cfg["Kn"], Pr=cfg["Pr"],
                     varpi=cfg["varpi"], T_w=cfg["T_w"], u_w=cfg["u_w"], g=cfg["g"])
    b = Batch([p])
    b.init_equilibrium()
    b.step(100)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    b.step(steps)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    cells = cfg["dims"][0] * cfg["dims"][1]
    b.close()
    return dict(steps=steps, ms_per_step=ms, mlups=cells / (ms * 1e-3) / 1e6)


def bench_batch(r, steps, warmup, fp64_sample=16, storage="f32", whole=False, **mix):
    """Batched channels in one persistent launch vs. the same channels stepped
    one problem at a time with the FP64 single-lattice path (fp64_sample
    problems; 0 skips that comparison). mix: arguments of
    workloads.channel_batch (default: the 512-channel mix); whole: keep every
    problem in one workgroup (no cut problems) whatever the autotuner would
    pick."""
    import torch

    from paper_1209_6548_amd import Batch, make_problem, workloads
    specs = workloads.channel_batch(r, **mix)
    probs = [make_problem("D2Q37", s["dims"][0], s["dims"][1], storage=storage, Kn=s["Kn"], Pr=s["Pr"],
                          T_w=s["T_w"], u_w=s["u_w"], g=s["g"]) for s in specs]
    cells = sum(s["dims"][0] * s["dims"][1] for s in specs)
    b = Batch(probs)
    b.autotune(20)
    if whole and b.split[1]:
        b.set_split(0)
    info = b.layout_info()
    b.init_equilibrium()
    b.set_reduce_interval(1000)      # the FP64 per-problem reductions ride along every 1000 steps
    b.step(warmup)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    b.step(steps)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    red = b.last_reduction() if steps + warmup >= 1000 else b.reduce()
    launch = ("one launch per step (problems cut into pieces over all workgroups), replayed from graphs of "
              "32 steps" if info["split"] else "one persistent kernel per step() call, captured in a HIP graph and "
              "replayed")
    out = dict(problems=len(specs), cells=cells, layout=info, launch=launch, reductions="FP64 per problem, fused "
               "every 1000 steps",
               ms_per_step=ms, mlups=cells / (ms * 1e-3) / 1e6,
               finite=bool(all(np.isfinite(x["mass"]) and np.isfinite(x["energy"]) for x in red)))
    b.close()
    if fp64_sample == 0:
        return out
    # per-problem FP64 loop on a sample of the same problems (same per-step work)
    rng = np.random.default_rng(0)
    pick = rng.choice(len(specs), fp64_sample, replace=False)
    lats = []
    for i in pick:
        s = specs[i]
        cfg = dict(s, dims=s["dims"])
        lats.append(make_lattice(cfg, "f64"))
    n = max(10, steps // 10)
    for L in lats:
        L.step(2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(n):
        for L in lats:
            L.step(1)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    c_s = sum(specs[i]["dims"][0] * specs[i]["dims"][1] for i in pick)
    out["per_problem_fp64"] = dict(sample_problems=int(fp64_sample), mlups=c_s * n / dt / 1e6)
    for L in lats:
        L.close()
    return out


def copy_bandwidth(nbytes=1 << 30, reps=10):
    """Context for the roofline: read+write GB/s of a plain device-to-device
    copy of nbytes (torch's copy, timed with HIP events)."""
    import torch
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    torch.cuda.empty_cache()
    return 2 * nbytes / (ms * 1e-3) / 1e9


def measured_traffic(storage, path=TRAFFIC_FILE):
    """HBM bytes per launch of a kernel on its 1024 x 1024 workload from the
    FETCH_SIZE / WRITE_SIZE counters (calibrated against a copy of known
    size), or None if the kernel's sources changed since they were taken."""
    import hashlib
    try:
        with open(path) as fh:
            rec = json.load(fh)
        h = hashlib.sha256()
        for f in rec["sources"]:
            with open(os.path.join(ROOT, f), "rb") as fh:
                h.update(fh.read())
        if h.hexdigest() != rec["source_sha256"]:
            return None
        return int(rec["per_launch_bytes"][storage]["hbm_bytes"])
    except (OSError, KeyError, ValueError):
        return None


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(r, budget_s=20.0, all_threads_s=8.0):
    """The FP64 oracle on a bounded sample of the same workload: the 1024 x
    1024 channel's per-cell work (D2Q37, walls, force, N = 4) on a 256 x 256
    instance with the same Kn, Pr and walls, stepped until the time budget on
    one core (numpy with its BLAS limited to one thread: the oracle's array
    operations do not run faster with more BLAS threads); then, for
    comparison, with numpy's default thread pools for a shorter budget."""
    from threadpoolctl import threadpool_info, threadpool_limits

    from oracle import lattice as OL
    from oracle import quadrature
    from paper_1209_6548_amd import workloads
    cfg = workloads.poiseuille_thermal_1024(r, n=256)
    vs = quadrature.d2q37()
    prob = OL.Problem(vs, cfg["dims"], Kn=cfg["Kn"], Pr=cfg["Pr"], varpi=cfg["varpi"], walls=True,
                      wall_lo=OL.Wall(cfg["T_w"][0]), wall_hi=OL.Wall(cfg["T_w"][1]), g=cfg["g"])
    M = prob.M

    def timed(budget):
        f = OL.equilibrium_state(prob, np.ones(M), np.zeros((M, 2)), np.ones(M))
        f = OL.step(f, prob)
        t0 = time.perf_counter()
        n = 0
        while time.perf_counter() - t0 < budget and n < 200:
            f = OL.step(f, prob)
            n += 1
        return n, time.perf_counter() - t0

    with threadpool_limits(limits=1):
        n, dt = timed(budget_s)
    threads = max([1] + [int(i.get("num_threads", 1)) for i in threadpool_info()])
    nm, dtm = timed(all_threads_s)
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count()
    return dict(value=M * n / dt / 1e6, unit="MLUPS", cores=1, kind="oracle",
                sample=f"256x256 D2Q37 channel (same Kn, Pr, walls, force as the 1024x1024 case), {n} steps in "
                       f"{dt:.1f} s on one core (numpy, BLAS limited to one thread)",
                all_threads=dict(value=M * nm / dtm / 1e6, steps=nm, seconds=round(dtm, 2), blas_threads=threads,
                                 note="numpy's default thread pools: no faster than one core for this oracle"),
                host=dict(cpu_model=_cpu_model(), cores_available=avail))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--only-main", action="store_true", help="time only the headline FP32 run")
    ap.add_argument("--profile", action="store_true",
                    help="headline kernel only, preceded by a 1 GiB device copy whose known size calibrates "
                         "the FETCH_SIZE / WRITE_SIZE counters")
    ap.add_argument("--storage", default="f32", choices=("f32", "f64", "f16"),
                    help="storage of the headline run (default f32)")
    ap.add_argument("--kernel", default="step", choices=("step", "tvd", "tvd3"),
                    help="with --profile: the kernel to run after the calibration copy (step: the headline "
                         "lattice step; tvd: the paper's own TVD scheme on D2Q36; tvd3: the same on D3Q216, "
                         "128^3)")
    args = ap.parse_args()
    if args.profile:
        args.only_main, args.no_cpu = True, True
    if args.gpus != 1:
        print(json.dumps({"error": "the library steps a lattice on one GPU (no halo exchange between GPUs "
                                    "is implemented); --gpus must be 1"}))
        sys.exit(2)

    import torch

    from paper_1209_6548_amd import lattice_info, workloads
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU"}))
        sys.exit(1)
    r = lattice_info("D2Q37")["r"]
    cfg = workloads.poiseuille_thermal_1024(r, storage=args.storage)
    copy_gbs = None
    if not args.profile:
        # context for the roofline, measured first: it also brings the GPU out of idle
        copy_gbs = copy_bandwidth()
        log(f"device copy: {copy_gbs:.0f} GB/s")
    if args.profile:
        n = 1 << 28                                   # 2^28 floats = 1 GiB each way
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        log("calibration copy: 1073741824 bytes read, 1073741824 bytes written")
        del a, b
        if args.kernel in ("tvd", "tvd3"):
            t = (bench_tvd(args.storage, args.steps, args.warmup) if args.kernel == "tvd" else
                 bench_tvd(args.storage, args.steps, args.warmup, velset="D3Q216GH", dims=(128, 128, 128)))
            log(f"tvd {args.storage}: {t['mlups']:.0f} MLUPS, {t['algorithmic_GBs']:.0f} GB/s")
            print(json.dumps(t), flush=True)
            return
    log(f"headline: {cfg['name']} {args.storage}, {args.steps} steps after {args.warmup} warmup")
    main_run = bench_single(cfg, args.storage, args.steps, args.warmup)
    log(f"{args.storage}: {main_run['mlups']:.0f} MLUPS, {main_run['algorithmic_GBs']:.0f} GB/s")
    variants = {}
    if not args.only_main:
        key = f"{args.storage}_two_buffers"
        variants[key] = bench_single(cfg, args.storage, max(20, args.steps // 2), args.warmup, inplace=0)
        log(f"{key}: {variants[key]['mlups']:.0f} MLUPS, {variants[key]['algorithmic_GBs']:.0f} GB/s")
        for st in ("f64", "f16"):
            variants[st] = bench_single(cfg, st, max(20, args.steps // 2), args.warmup)
            log(f"{st}: {variants[st]['mlups']:.0f} MLUPS, {variants[st]['algorithmic_GBs']:.0f} GB/s")
        cfg1 = workloads.poiseuille_thermal_1024(r, Pr=1.0)
        key = f"{cfg1['name']}_Pr1_f32"
        variants[key] = bench_single(cfg1, "f32", max(20, args.steps // 2), args.warmup)
        log(f"{key}: {variants[key]['mlups']:.0f} MLUPS, {variants[key]['algorithmic_GBs']:.0f} GB/s")
        c0 = workloads.couette_1x32(r)
        variants["couette_1x32_f64"] = bench_single(c0, "f64", 2000, 100)
        variants["couette_1x32_f64"]["regime"] = "latency-bound (32 cells): not an HBM-roofline regime"
        variants["couette_1x32_f64"]["persistent"] = bench_couette_persistent(c0, 20000)
        log(f"couette_1x32_f64: {variants['couette_1x32_f64']['mlups']:.1f} MLUPS in graphs, "
            f"{variants['couette_1x32_f64']['persistent']['mlups']:.1f} MLUPS in one persistent launch")
        # a persistent launch of ~30 us steps: time at least 1000 of them, so that the window is
        # long against the clock ramp after the nearly idle 1 x 32 channel run
        variants["batched_channels"] = bench_batch(r, max(1000, 5 * args.steps), max(100, args.warmup))
        variants["batched_channels"]["regime"] = ("cache-resident (about 160 MB of populations, inside the "
                                                  "256 MB Infinity Cache): not an HBM-roofline regime")
        log(f"batch: {variants['batched_channels']['mlups']:.0f} MLUPS")
        variants["batched_channels_f16"] = bench_batch(r, max(1000, 5 * args.steps), max(100, args.warmup),
                                                       fp64_sample=0, storage="f16")
        variants["batched_channels_f16"]["regime"] = "cache-resident (about 80 MB of populations)"
        log(f"batch f16: {variants['batched_channels_f16']['mlups']:.0f} MLUPS")
        # few large channels: 32 of 64 x 256..512 cells (about 24 000 each), fewer problems than compute units
        big = dict(n=32, nx=64, ny_range=(256, 512))
        steps_big = max(200, args.steps)
        variants["batched_channels_32_large"] = bench_batch(r, steps_big, 20, fp64_sample=0, **big)
        variants["batched_channels_32_large"]["whole_problems"] = bench_batch(r, steps_big, 20, fp64_sample=0,
                                                                              whole=True, **big)
        log(f"batch of 32 large channels: {variants['batched_channels_32_large']['mlups']:.0f} MLUPS "
            f"(whole problems: {variants['batched_channels_32_large']['whole_problems']['mlups']:.0f})")
        r3 = lattice_info("D3Q39")["r"]
        # 3-D workloads (timed from the rest state: the step's work does not depend on it)
        box = dict(name="shear_wave_256^3", velset="D3Q39", dims=(256, 256, 256), walls=False, Kn=0.02,
                   Pr=2 / 3, varpi=0.5, g=(0.0, 0.0, 0.0))
        for st in ("f32", "f16", "f64"):
            key = f"shear_wave_256^3_{st}"
            variants[key] = bench_single(box, st, max(10, args.steps // (4 if st != "f64" else 10)), 3)
            log(f"{key}: {variants[key]['mlups']:.0f} MLUPS, {variants[key]['algorithmic_GBs']:.0f} GB/s")
        ch = workloads.channel_3d(r3)
        key = f"{ch['name']}_f16"
        variants[key] = bench_single(ch, "f16", max(10, args.steps // 10), 3)
        log(f"{key}: {variants[key]['mlups']:.0f} MLUPS, {variants[key]['algorithmic_GBs']:.0f} GB/s")
        for st in ("f32", "f64"):
            key = f"{TVD_CFG['name']}_{st}"
            variants[key] = bench_tvd(st, max(20, args.steps // 2), 5)
            log(f"{key}: {variants[key]['mlups']:.0f} MLUPS, {variants[key]['algorithmic_GBs']:.0f} GB/s")
        for vs in ("D2Q16GH", "D2Q64GH"):          # the velocity-set study's other sets: cost grows with Q
            key = f"{TVD_CFG['name'].replace('d2q36', vs.lower())}_f32"
            variants[key] = bench_tvd("f32", max(20, args.steps // 2), 5, velset=vs)
            log(f"{key}: {variants[key]['mlups']:.0f} MLUPS, {variants[key]['algorithmic_GBs']:.0f} GB/s")
        key = "periodic_gas_128x128x128_d3q216gh_f32"   # the paper's 3-D set
        variants[key] = bench_tvd("f32", max(20, args.steps // 10), 25, velset="D3Q216GH", dims=(128, 128, 128))
        log(f"{key}: {variants[key]['mlups']:.0f} MLUPS, {variants[key]['algorithmic_GBs']:.0f} GB/s")
    cpu = None
    if not args.no_cpu:
        log("cpu baseline (oracle)")
        cpu = cpu_baseline(r)
        log(f"cpu: {cpu['value']:.3f} MLUPS")
    ms = main_run["ms_per_step"]
    achieved = main_run["algorithmic_GBs"]
    pairs = main_run["in_place_pairs"]
    traffic = measured_traffic(args.storage, PAIR_TRAFFIC_FILE if pairs else TRAFFIC_FILE)
    kernel = (f"k_pair<D2Q37, {args.storage}> (both steps of the in-place pair, one launch per step)" if pairs
              else f"k_step<D2Q37, {args.storage}>")
    line = {
        "metric": "MLUPS", "value": round(main_run["mlups"], 1), "unit": "MLUPS",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": args.storage,
        "data": "synthetic",
        "config": {"workload": cfg["name"], "velset": "D2Q37", "order_N": 4, "cells": 1024 * 1024,
                   "storage": f"{args.storage} deviational", "Kn": cfg["Kn"], "Pr": cfg["Pr"], "walls_T": list(cfg["T_w"]),
                   "g_x_nondim": cfg["g"][0], "scheme": "trapezoid", "in_place_pairs": pairs},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "traffic_over_algorithmic": (round(traffic / (main_run["bytes_per_cell"] * 1024 * 1024), 4)
                                                  if traffic else None),
                     "kernel": kernel, "bytes_per_cell": main_run["bytes_per_cell"],
                     "device_copy_GBs": round(copy_gbs, 1) if copy_gbs else None},
        "cpu_baseline": cpu,
        "variants": variants,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
