#!/usr/bin/env python3
"""Throughput benchmark of batched CDDT ray casting + beam sensor weights on one GPU.

Default workload (`--workload batched`; one step = one filter step of every
filter): 64 particle filters on room/corridor maps of uneven size (sides
512..4000), theta bins in {108, 200, 360}, 500..20000 particles each, 61 rays
per particle over 270 degrees, max range 500, fused cast + log-weight in one
persistent launch replayed from a hipGraph.  The same filters also run as
plain launches (one per filter) for comparison.  Inputs are seeded synthetic
data resident in HBM before timing starts.  The line also carries the gather
probe, a short serving measurement and the CPU oracle timed on this host.

Other workloads (each prints its own JSON line): `small` (256^2 rectangle map,
1000 particles x 61 rays, plain casts), `floor` (2000^2 floor, 2500 particles,
fused weights), `updates` (4000^2 floor, 1000 toggles + 1M particles x 61
casts per step), `serving` (8 resident maps, Poisson arrivals swept over load),
`suites` (the paper's grid and random query suites: per-query time distribution
and rays/s on CDDT, PCDDT, the dense lookup-table comparator and the cell-walk
comparator), `probe`
(random-gather bandwidth only).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "ray casts/sec on 1 MI355X (bit-exact vs oracle), batched vs plain; p99 serve latency"
PEAK_HBM_GBS = 8000.0
RAYS = 61
SEARCHES = 40         # 61 rays with radial pairing of rays r and r + 40 (21 pairs)
MAX_RANGE = 500
BUCKETS: int | None = 6  # log2 bucket width of the maps' bucket index (None: no index); set by --buckets
ZP16 = False  # 16-bit zero points in the bucket lines (results then follow the 16-bit reading); set by --zp16
PRUNE = False  # PCDDT: pruned static maps (exact for grid states only); set by --prune

# Algorithmic bytes per particle of the fused step, as the method defines it
# (a bin is a sorted array reached through its offset and length): pose 12 +
# occupancy byte 1 + log-weight out 4 + per search (band offset and length 8 +
# bracketing zero point 4) + the second bracketing zero point of each of the
# 21 pairs 4 + one table entry per ray 4.  The same figure is used with the
# bucket index, which reads no band header.
BYTES_PER_PARTICLE = 12 + 1 + 4 + SEARCHES * (8 + 4) + (RAYS - SEARCHES) * 4 + RAYS * 4
# Useful bytes per ray of the fused step, the figure the roofline fraction is
# taken on: band header 8 + both bracketing zero points 8 + one table entry 4 +
# the particle's pose 12, occupancy byte 1 and log-weight out 4 shared by its
# 61 rays (20.28 bytes).  It counts both neighbours of every ray, so it exceeds
# BYTES_PER_PARTICLE / 61 (13.5), which counts one zero point per search.
BYTES_PER_RAY_FUSED = 8 + 8 + 4 + (12 + 1 + 4) / RAYS
# Algorithmic bytes per plain cast: pose 12 + occupancy 1 + header 8 + zero point 4 + range out 4.
BYTES_PER_CAST = 12 + 1 + 8 + 4 + 4


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    # the batched kernel's own source: its body and everything it inlines
    for f in ("batch_kernel.h", "query_device.h", "band_layout.h", "device_types.h"):
        with open(os.path.join(ROOT, "paper_1705_01167_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def structure_layout() -> dict:
    """The maps' structure options; HBM traffic depends on them as much as on the kernel."""
    return {"bucket_log2": BUCKETS, "zp16": ZP16, "pcddt": PRUNE}


def measured_traffic(name: str, particles: int):
    """HBM bytes per launch from committed counter runs, if taken on the current kernel source,
    the same particle count and the same structure layout."""
    p = os.path.join(ROOT, "profiles", f"{name}_traffic.json")
    try:
        with open(p) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    if (d.get("kernel_source_hash") != kernel_source_hash() or d.get("particles") != particles
            or d.get("layout") != structure_layout()):
        return None
    return d.get("bytes_per_launch")


def t_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def timed(fn, steps: int, warmup: int, stream):
    """Run fn(stream) warmup + steps times; (wall seconds, HIP-event ms per step) over the timed steps."""
    import torch
    for _ in range(warmup):
        fn(stream)
    stream.synchronize()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(steps):
        fn(stream)
    e1.record(stream)
    stream.synchronize()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return wall, e0.elapsed_time(e1) / steps


# ---------------------------------------------------------------------------
# Batched filters (default workload)
# ---------------------------------------------------------------------------
def build_batched(n_filters: int, with_ranges: bool = False):
    """The many-filter workload's maps, particles, observations and tables on the device.

    with_ranges: every filter also gets an int32 [particle][ray] ranges output (kept in its entry of
    `keep` under "ranges"); the timed benchmark runs without them."""
    import torch
    from paper_1705_01167_amd import cddt
    from paper_1705_01167_amd import workloads as wl

    specs = wl.batched_specs(wl.rng_for(wl.BATCHED, wl.S_SPEC), n_filters=n_filters)
    off_h = wl.ray_offsets(RAYS)
    pair = cddt.pair_offset(off_h)
    off = t_dev(off_h)
    filters, keep, host = [], [], []
    t_gen = t_build = 0.0
    # every filter's poses are views of one buffer, so one copy can restore them all
    total_p = sum(sp["particles"] for sp in specs)
    pose_buf = torch.empty(3 * total_p, dtype=torch.float32, device="cuda")
    p_off = 0
    for f, sp in enumerate(specs):
        t0 = time.perf_counter()
        occ = wl.building_map(wl.rng_for(wl.BATCHED, wl.S_MAP, f), sp["side"], sp["side"])
        px, py, pth = wl.free_poses(wl.rng_for(wl.BATCHED, wl.S_POSES, f), occ, sp["particles"])
        obs, _ = wl.observations(wl.rng_for(wl.BATCHED, wl.S_OBS, f), occ, off_h, MAX_RANGE)
        table = wl.beam_table(MAX_RANGE, wl.beam_params(wl.rng_for(wl.BATCHED, wl.S_TABLE, f)))
        t1 = time.perf_counter()
        occ_d = t_dev(occ)
        m = cddt.Map(occ_d, sp["theta_bins"], buckets=BUCKETS, zp16=ZP16, prune=PRUNE)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        del occ_d
        d = {k: t_dev(v) for k, v in dict(obs=obs, table=table).items()}
        P = sp["particles"]
        for i, (k, v) in enumerate((("px", px), ("py", py), ("pth", pth))):
            d[k] = pose_buf[3 * p_off + i * P: 3 * p_off + (i + 1) * P]
            d[k].copy_(torch.from_numpy(v))
        p_off += P
        lw = torch.zeros(sp["particles"], dtype=torch.float32, device="cuda")
        if with_ranges:
            d["ranges"] = torch.empty((P, RAYS), dtype=torch.int32, device="cuda")
        d["off"] = off
        filters.append(cddt.make_filter(m, d["px"], d["py"], d["pth"], off, d["obs"], d["table"], MAX_RANGE,
                                        lw, ranges=d.get("ranges"), pair=pair))
        keep.append((m, d, lw))
        host.append(dict(occ=occ, px=px, py=py, pth=pth, obs=obs, table=table, n=sp["theta_bins"]))
        t_gen += t1 - t0
        t_build += t2 - t1
    return specs, filters, keep, host, off_h, dict(generate_s=t_gen, gpu_build_s=t_build, pose_buf=pose_buf)


def cpu_baseline(specs, host, off_h, budget_s: float, max_build_s: float = 40.0):
    """The C++ oracle (plain CDDT, std::thread over particles) on filters spread over map sizes."""
    from oracle import ref as oref
    flags = oref.select_native()
    threads = max(1, len(os.sched_getaffinity(0)))
    order = sorted(range(len(specs)), key=lambda f: specs[f]["side"])
    picks = sorted({order[int(round(q * (len(order) - 1)))] for q in (0.0, 0.25, 0.5, 0.75, 1.0)})
    built, build_s = [], 0.0
    for f in picks:
        h = host[f]
        t0 = time.perf_counter()
        built.append((f, oref.RefCDDT(h["occ"], h["n"], threads=threads, zp16=ZP16, prune=PRUNE)))
        build_s += time.perf_counter() - t0
        if build_s > max_build_s:
            break
    rays, secs, passes = 0, 0.0, 0
    while secs < budget_s and passes < 1000:
        for f, rm in built:
            h = host[f]
            t0 = time.perf_counter()
            rm.weight(h["px"], h["py"], h["pth"], off_h, h["obs"], h["table"], MAX_RANGE, threads=threads)
            secs += time.perf_counter() - t0
            rays += h["px"].size * RAYS
        passes += 1
    # one thread on the same filters, a bounded number of passes
    rays1, secs1 = 0, 0.0
    while secs1 < min(3.0, budget_s / 3):
        for f, rm in built:
            h = host[f]
            t0 = time.perf_counter()
            rm.weight(h["px"], h["py"], h["pth"], off_h, h["obs"], h["table"], MAX_RANGE, threads=1)
            secs1 += time.perf_counter() - t0
            rays1 += h["px"].size * RAYS
    names = [f"{specs[f]['side']}^2/n{specs[f]['theta_bins']}/{specs[f]['particles']}p" for f, _ in built]
    for _, rm in built:
        rm.close()
    return {"value": rays / secs, "unit": "rays/s", "cores": threads, "kind": "oracle",
            "single_thread_rays_per_s": rays1 / secs1, "cpu_model": cpu_model(),
            "sample": (f"plain C++ CDDT oracle (sorted vectors, std::upper_bound, double log-sum; {flags}) with "
                       f"{threads} threads on {len(built)} of {len(specs)} filters spread over map size "
                       f"[{', '.join(names)}], all their particles, {passes} passes, {rays} rays in "
                       f"{secs:.1f} s; oracle structure build ({build_s:.1f} s) excluded; one thread: "
                       f"{rays1} rays in {secs1:.1f} s")}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def run_batched(args) -> dict:
    import torch
    from paper_1705_01167_amd import cddt, tune

    log("bench: generating and building maps")
    specs, filters, keep, host, off_h, times = build_batched(args.filters)
    pose_buf = times.pop("pose_buf")
    particles = sum(s["particles"] for s in specs)
    rays_per_step = particles * RAYS
    stats = [k[0].info() for k in keep]
    log(f"bench: {len(specs)} filters, {particles} particles, {rays_per_step} rays/step, "
        f"{sum(s['zero_points'] for s in stats) / 1e6:.1f} M zero points, build {times}")

    stream = torch.cuda.Stream()
    plan = cddt.Plan(filters, stream=stream, keepalive=keep)
    sig = tune.signature(len(specs), particles, [s["theta_bins"] for s in specs], torch.cuda.get_device_name(0),
                         BUCKETS if not (ZP16 or PRUNE) else f"{BUCKETS}{'z16' if ZP16 else ''}{'p' if PRUNE else ''}")
    t0 = time.perf_counter()
    if args.tuning:
        best = tuple(int(v) for v in args.tuning.split(","))
        plan.tuning = best
        best_ms = float("nan")
    else:
        best, best_ms, _ = tune.autotune(plan, sig, use_cache=not args.no_tune_cache, stream=stream)
    log(f"bench: tuning {best} ({best_ms:.3f} ms) in {time.perf_counter() - t0:.1f} s")

    # reference outputs from plain launches; the batched graph must reproduce them
    plan.run_plain(stream)
    stream.synchronize()
    plain_out = [k[2].clone() for k in keep]
    for k in keep:
        k[2].zero_()
    torch.cuda.synchronize()
    step = plan.run if args.no_graph else plan.replay
    if not args.no_graph:
        plan.capture(stream)
    wall, batched_ms = timed(step, args.steps, args.warmup, stream)
    exact = all(torch.equal(a, k[2]) for a, k in zip(plain_out, keep))
    _, plain_ms = timed(plan.run_plain, args.steps, max(1, args.warmup // 2), stream)
    # The same persistent kernel and tuning, one launch per filter: splits the
    # gain over plain launches into the search strategy's and the batching's.
    singles = [cddt.Plan([f], tuning=tuple(best), stream=stream, keepalive=keep) for f in filters]

    def run_singles(st):
        for sp in singles:
            sp.run(st)

    _, single_ms = timed(run_singles, args.steps, max(1, args.warmup // 2), stream)
    for sp in singles:
        sp.close()
    log(f"bench: batched {batched_ms:.3f} ms, plain launches {plain_ms:.3f} ms, the batched kernel per filter "
        f"{single_ms:.3f} ms")

    mcl = None if args.no_mcl else run_mcl_step(args, plan, pose_buf, specs, stream, batched_ms)

    value = rays_per_step / (wall / args.steps)
    algo_bytes = rays_per_step * BYTES_PER_RAY_FUSED
    achieved = algo_bytes / (batched_ms * 1e-3) / 1e9
    traffic = measured_traffic("k_batch", particles)
    probe = cddt.probe_gather() if not args.no_probe else None
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "rays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic",
        "config": {
            "workload": (f"batched: {len(specs)} particle filters on room/corridor maps "
                         f"{min(s['side'] for s in specs)}^2..{max(s['side'] for s in specs)}^2, "
                         f"theta bins {{108,200,360}}, {min(s['particles'] for s in specs)}.."
                         f"{max(s['particles'] for s in specs)} particles each, {RAYS} rays, max range "
                         f"{MAX_RANGE}, fused cast + beam log-weight, one persistent hipGraph-replayed "
                         f"launch per step"),
            "filters": len(specs),
            "particles": particles,
            "rays_per_step": rays_per_step,
            "zero_points": int(sum(s["zero_points"] for s in stats)),
            "bands": int(sum(s["rows"] for s in stats)),
            "structure_bytes": int(sum(s["device_bytes"] for s in stats)),
            "bucket_index": ({"log2_width_cells": BUCKETS,
                              "lines": int(sum(s["bucket_lines"] for s in stats)),
                              "overflow_buckets": int(sum(s["bucket_overflow"] for s in stats)),
                              "zero_points_16bit": ZP16}
                             if BUCKETS is not None else None),
            "pcddt": PRUNE,
            "tuning": {"particles_per_tile": best[0], "waves_per_block": best[1], "blocks_per_cu": best[2],
                       "search_mode": best[3]},
            "parallelism": "single GPU",
        },
        "batched_rays_per_s_kernel": rays_per_step / (batched_ms * 1e-3),
        "plain_rays_per_s": rays_per_step / (plain_ms * 1e-3),
        "batched_over_plain": plain_ms / batched_ms,
        "per_filter_same_kernel_rays_per_s": rays_per_step / (single_ms * 1e-3),
        "batched_over_per_filter_same_kernel": single_ms / batched_ms,
        "batched_equals_plain": bool(exact),
        "build_seconds": times["gpu_build_s"],
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": PEAK_HBM_GBS,
            "unit": "GB/s",
            "frac": achieved / PEAK_HBM_GBS,
            "traffic": traffic,
            "kernel": "k_batch",
            "bytes_per_ray": BYTES_PER_RAY_FUSED,
            "bytes_per_launch": algo_bytes,
            "kernel_ms": batched_ms,
            "frac_at_one_zero_point_per_search": particles * BYTES_PER_PARTICLE / (batched_ms * 1e-3) / 1e9
            / PEAK_HBM_GBS,
        },
        "mcl_step": mcl,
        "gather_probe": probe,
        "cpu_baseline": None,
        "context": "paper: 2500 particles x 61 rays at 40 Hz = 6.1e6 rays/s on one Jetson TX1 CPU thread",
    }
    if traffic is not None and probe is not None:
        out["roofline"]["traffic_GBps"] = traffic / (batched_ms * 1e-3) / 1e9
        out["roofline"]["traffic_frac_of_probe"] = out["roofline"]["traffic_GBps"] / probe["GBps"]
    plan.close()
    del keep, filters
    torch.cuda.empty_cache()
    if not args.no_serving:
        log("bench: serving summary")
        out["serving"] = run_serving(args, ref_rays_per_s=rays_per_step / (batched_ms * 1e-3))
    if not args.no_cpu:
        log("bench: timing the CPU oracle")
        out["cpu_baseline"] = cpu_baseline(specs, host, off_h, args.cpu_budget)
    return out


def run_mcl_step(args, plan, pose_buf, specs, stream, sensor_ms: float) -> dict:
    """The whole particle-filter step of every filter (motion, weights, resampling), one captured graph.

    Each timed step first restores every filter's particles from a snapshot (one 3.8 MB device copy,
    included in the time), so every step starts from the same particles as the sensor-only step.
    """
    import torch
    from paper_1705_01167_amd import workloads as wl
    rng = wl.rng_for(wl.BATCHED, wl.S_MOTION)
    F = len(specs)
    P = sum(sp["particles"] for sp in specs)
    odom = t_dev(rng.normal(0, 0.5, 3 * F).astype(np.float32))
    u = t_dev(rng.integers(0, 2**32, F, dtype=np.uint64).astype(np.uint32).view(np.int32))
    noise = t_dev(rng.normal(0, 0.05, 3 * P).astype(np.float32))
    snapshot = pose_buf.clone()
    plan.set_mcl(odom, u, noise)
    plan.capture_mcl(stream)

    def step(s):
        with torch.cuda.stream(s):
            pose_buf.copy_(snapshot)
        plan.replay(s)

    wall, ms = timed(step, args.steps, args.warmup, stream)
    with torch.cuda.stream(stream):
        pose_buf.copy_(snapshot)
    stream.synchronize()
    return {"ms_per_step": wall / args.steps * 1e3, "kernel_ms": ms, "sensor_only_kernel_ms": sensor_ms,
            "particles_per_s": P / (wall / args.steps), "rays_per_s": P * RAYS / (wall / args.steps),
            "steps": "motion (odometry + caller noise) -> batched log-weights -> systematic resampling per "
                     "filter, in place; each step restores the particles first (one device copy)"}


# ---------------------------------------------------------------------------
# Single-map workloads
# ---------------------------------------------------------------------------
def run_small(args) -> dict:
    import torch
    from paper_1705_01167_amd import cddt
    from paper_1705_01167_amd import workloads as wl
    occ = wl.rect_map(wl.rng_for(wl.SMALL, wl.S_MAP))
    m = cddt.Map(t_dev(occ), 108, buckets=BUCKETS, zp16=ZP16, prune=PRUNE)
    px, py, pth = wl.free_poses(wl.rng_for(wl.SMALL, wl.S_POSES), occ, 1000)
    off = wl.ray_offsets(RAYS)
    x = t_dev(np.repeat(px, RAYS))
    y = t_dev(np.repeat(py, RAYS))
    th = t_dev((np.repeat(pth, RAYS) + np.tile(off, px.size)).astype(np.float32))
    out_r = torch.empty(x.numel(), dtype=torch.int32, device="cuda")
    stream = torch.cuda.Stream()
    wall, ms = timed(lambda s: m.cast(x, y, th, MAX_RANGE, out=out_r, stream=s), args.steps, args.warmup, stream)
    n = x.numel()
    return {"metric": "ray casts/sec (plain cddt_cast)", "value": n / (wall / args.steps), "unit": "rays/s",
            "ms_per_step": wall / args.steps * 1e3, "kernel_ms": ms, "steps": args.steps,
            "config": {"workload": "small: 256^2 rectangles map (~10% occupied), 108 bins, 1000 particles x 61 "
                                   "rays as 61000 plain casts, max range 500",
                       "occupancy": float(occ.mean()), **{k: v for k, v in m.info().items()
                                                          if k in ("zero_points", "rows", "edge_cells")}},
            "roofline": {"bound": "latency (L2-resident structure)", "algorithmic_GBps":
                         n * BYTES_PER_CAST / (ms * 1e-3) / 1e9}}


def run_floor(args) -> dict:
    import torch
    from paper_1705_01167_amd import cddt
    from paper_1705_01167_amd import workloads as wl
    occ = wl.building_map(wl.rng_for(wl.FLOOR, wl.S_MAP), 2000, 2000)
    m = cddt.Map(t_dev(occ), 200, buckets=BUCKETS, zp16=ZP16, prune=PRUNE)
    off_h = wl.ray_offsets(RAYS)
    px, py, pth = wl.free_poses(wl.rng_for(wl.FLOOR, wl.S_POSES), occ, 2500)
    table = t_dev(wl.beam_table(MAX_RANGE, wl.beam_params(wl.rng_for(wl.FLOOR, wl.S_TABLE))))
    obs, _ = wl.observations(wl.rng_for(wl.FLOOR, wl.S_OBS), occ, off_h, MAX_RANGE)
    d = [t_dev(a) for a in (px, py, pth, off_h, obs)]
    lw = torch.empty(2500, dtype=torch.float32, device="cuda")
    pair = cddt.pair_offset(off_h)
    stream = torch.cuda.Stream()
    wall, ms = timed(lambda s: m.weight(*d, table, MAX_RANGE, pair=pair, logw=lw, stream=s), args.steps,
                     args.warmup, stream)
    n = 2500 * RAYS
    return {"metric": "ray casts/sec (fused cddt_weight, one filter)", "value": n / (wall / args.steps),
            "unit": "rays/s", "ms_per_step": wall / args.steps * 1e3, "kernel_ms": ms, "steps": args.steps,
            "config": {"workload": "floor: 2000^2 room/corridor map (~4% occupied), 200 bins, 2500 particles x "
                                   "61 rays, fused beam log-weight (501^2 table), max range 500",
                       "occupancy": float(occ.mean()), **{k: v for k, v in m.info().items()
                                                          if k in ("zero_points", "rows", "edge_cells")}},
            "roofline": {"bound": "latency (MALL-resident structure)",
                         "algorithmic_GBps": 2500 * RAYS * BYTES_PER_RAY_FUSED / (ms * 1e-3) / 1e9}}


# The paper's query-time suites (Sec. VI): a uniformly spaced grid over the states and uniformly random states,
# on the building floor and on a 1000^2 stand-in for the paper's maps (which are not available)
SUITE_MAPS = (("floor 2000^2, 200 bins (the building-floor map)", 2000, 200),
              ("room map 1000^2, 108 bins (stand-in for the paper's ~1000^2 maps)", 1000, 108))
SUITE_LAYOUTS = (("cddt", {}), ("cddt, bucket index 2^7", {"buckets": 7}), ("pcddt", {"prune": True}))
SUITE_POSITIONS = 500  # grid positions per axis (stride = side / 500), at every bin: 250,000 x bins queries
SUITE_SAMPLE = 1 << 21  # per-query times summarised on this many queries (a seeded sample)
SUITE_CPU_QUERIES = 1 << 20  # queries the CPU oracle times per suite, one thread
# the paper's per-query times in seconds (one CPU thread; its Synthetic map, ~1000^2; its tables), as context
PAPER_SUITE_TIMES = {"random": {"cddt": (1.24e-07, 1.05e-07, 5.3e-08), "pcddt": (1.19e-07, 1.01e-07, 5e-08),
                                "lut": (1.82e-07, 1.68e-07, 1.4e-08)},
                     "grid": {"cddt": (7.02e-08, 6.8e-08, 1e-08), "pcddt": (6.94e-08, 6.8e-08, 9e-09),
                              "lut": (6.33e-08, 4.2e-08, 4.6e-08)}}


def per_query_stats(ticks, khz: int, seed: int) -> dict:
    """Mean, median and inter-quartile range of per-query times (ns) on a seeded sample."""
    import torch
    n = ticks.numel()
    g = torch.Generator(device="cpu").manual_seed(seed)
    idx = torch.randint(0, n, (min(n, SUITE_SAMPLE),), generator=g).to(ticks.device)
    ns = ticks[idx].double().cpu().numpy() * (1e6 / khz)
    q1, med, q3 = np.percentile(ns, [25, 50, 75])
    return {"mean_ns": float(ns.mean()), "median_ns": float(med), "iqr_ns": float(q3 - q1), "sampled": int(ns.size)}


def time_queries(fn, reps: int = 3) -> float:
    """Kernel milliseconds of fn(stream): best of reps, HIP events on the stream the launch uses."""
    import torch
    st = torch.cuda.Stream()
    fn(st)
    best = float("inf")
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        fn(st)
        e1.record(st)
        st.synchronize()
        best = min(best, e0.elapsed_time(e1))
    return best


def run_suites(args) -> dict:
    import torch
    from oracle import ref as oref
    from paper_1705_01167_amd import cddt
    from paper_1705_01167_amd import workloads as wl
    khz = cddt.device_clock_khz()
    out = []
    for mi, (name, side, n) in enumerate(SUITE_MAPS):
        seed_map = (wl.FLOOR, wl.S_MAP) if side == 2000 else (wl.SUITES, wl.S_MAP)
        occ = wl.building_map(wl.rng_for(*seed_map), side, side)
        stride = side // SUITE_POSITIONS
        suites = {"grid": wl.grid_states(side, side, n, stride),
                  "random": wl.random_states(wl.rng_for(wl.SUITES, wl.S_POSES, mi), side, side,
                                             SUITE_POSITIONS * SUITE_POSITIONS * n)}
        dev = {k: tuple(t_dev(a) for a in v) for k, v in suites.items()}
        log(f"bench: suites on {name}: {suites['grid'][0].size} queries per suite")
        entry = {"map": name, "occupancy": float(occ.mean()), "queries_per_suite": int(suites["grid"][0].size),
                 "grid_stride_cells": stride, "layouts": {}}
        plain_ranges = {}
        for lname, kw in SUITE_LAYOUTS:
            m = cddt.Map(t_dev(occ), n, **kw)
            info = m.info()
            res = {"structure_bytes": int(info["device_bytes"]), "zero_points": int(info["zero_points"])}
            for sname, (x, y, th) in dev.items():
                q = x.numel()
                ms = time_queries(lambda st: m.cast(x, y, th, MAX_RANGE, stream=st))
                rg = m.cast(x, y, th, MAX_RANGE)
                rg_t, ticks = m.cast_timed(x, y, th, MAX_RANGE)
                torch.cuda.synchronize()
                if lname == "cddt":
                    plain_ranges[sname] = rg
                res[sname] = {"rays_per_s": q / (ms * 1e-3), "ns_per_query_amortized": ms * 1e6 / q,
                              "kernel_ms": ms, "per_query": per_query_stats(ticks, khz, 7 + mi),
                              "timed_equals_untimed": bool(torch.equal(rg, rg_t)),
                              "equals_cddt": bool(torch.equal(rg, plain_ranges[sname]))
                              if sname in plain_ranges else None}
                log(f"bench: suites {name} / {lname} / {sname}: {res[sname]}")
            entry["layouts"][lname] = res
            m.close()
        # the dense lookup-table comparator, built from the plain map's casts at every discrete state
        m = cddt.Map(t_dev(occ), n)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lut = m.lut(MAX_RANGE)
        torch.cuda.synchronize()
        res = {"bytes": lut.numel() * 2, "build_s": time.perf_counter() - t0}
        for sname, (x, y, th) in dev.items():
            q = x.numel()
            ms = time_queries(lambda st: cddt.lut_cast(lut, x, y, th, stream=st))
            rg, ticks = cddt.lut_cast(lut, x, y, th, timed=True)
            torch.cuda.synchronize()
            res[sname] = {"rays_per_s": q / (ms * 1e-3), "ns_per_query_amortized": ms * 1e6 / q, "kernel_ms": ms,
                          "per_query": per_query_stats(ticks, khz, 9 + mi),
                          "agreement_with_cddt": float((rg == plain_ranges[sname]).double().mean())}
            log(f"bench: suites {name} / table / {sname}: {res[sname]}")
        entry["lut"] = res
        del lut
        # the cell-walk comparator (exact ray, theta not binned) on the same grid
        res = {}
        for sname, (x, y, th) in dev.items():
            q = x.numel()
            ms = time_queries(lambda st: m.march(x, y, th, MAX_RANGE, stream=st))
            rg, ticks = m.march(x, y, th, MAX_RANGE, timed=True)
            torch.cuda.synchronize()
            res[sname] = {"rays_per_s": q / (ms * 1e-3), "ns_per_query_amortized": ms * 1e6 / q, "kernel_ms": ms,
                          "per_query": per_query_stats(ticks, khz, 13 + mi),
                          "within_one_cell_of_cddt": float(((rg - plain_ranges[sname]).abs() <= 1).double().mean())}
            log(f"bench: suites {name} / cell walk / {sname}: {res[sname]}")
        entry["cell_walk"] = res
        m.close()
        # the CPU oracle (plain C++ CDDT) per query on one thread, a sample of each suite
        if not args.no_cpu:
            oref.select_native()
            rm = oref.RefCDDT(occ, n)
            cpu = {}
            for sname, (x, y, th) in suites.items():
                sel = np.random.default_rng(11 + mi).integers(0, x.size, SUITE_CPU_QUERIES)
                xs, ys, ts = x[sel], y[sel], th[sel]
                rm.cast(xs[:1024], ys[:1024], ts[:1024], MAX_RANGE)
                t0 = time.perf_counter()
                rm.cast(xs, ys, ts, MAX_RANGE)
                cpu[sname] = {"ns_per_query_amortized": (time.perf_counter() - t0) * 1e9 / xs.size,
                              "queries": int(xs.size), "threads": 1}
            rm.close()
            entry["cpu_oracle"] = cpu
        del dev
        torch.cuda.empty_cache()
        out.append(entry)
    return {"metric": "query-time suites: per-query time (mean, median, IQR) and rays/s, grid and random states",
            "device_clock_khz": khz, "maps": out, "paper_context_seconds_mean_median_iqr": PAPER_SUITE_TIMES,
            "per_query_note": "per-query time = device wall-clock ticks from a query's load to its result, for "
                              "its wave (64 queries, or 256 in the queued kernel) among all the waves in flight; "
                              "ns_per_query_amortized = kernel time / queries"}


def run_updates(args) -> dict:
    import torch
    from paper_1705_01167_amd import cddt
    from paper_1705_01167_amd import workloads as wl
    occ = wl.building_map(wl.rng_for(wl.UPDATES, wl.S_MAP), 4000, 4000)
    n, P = 200, 1_000_000
    t0 = time.perf_counter()
    m = cddt.Map(t_dev(occ), n, buckets=BUCKETS, zp16=ZP16, prune=PRUNE)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    off = t_dev(wl.ray_offsets(RAYS))
    px, py, pth = wl.free_poses(wl.rng_for(wl.UPDATES, wl.S_POSES), occ, P)
    x = t_dev(px).repeat_interleave(RAYS)
    y = t_dev(py).repeat_interleave(RAYS)
    th = (t_dev(pth)[:, None] + off[None, :]).reshape(-1).contiguous()
    out_r = torch.empty(x.numel(), dtype=torch.int32, device="cuda")
    rng = wl.rng_for(wl.UPDATES, wl.S_OPS)
    cur = occ.copy()
    steps = args.steps
    ops = []
    for _ in range(steps + args.warmup):
        xs, ys, vals = wl.toggle_ops(rng, cur, 1000)
        wl.apply_ops(cur, xs, ys, vals)
        ops.append((xs, ys, vals))
    stream = torch.cuda.Stream()
    upd_s = cast_s = 0.0
    upd_each = []
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for i, (xs, ys, vals) in enumerate(ops):
        t0 = time.perf_counter()
        m.update(xs, ys, vals, stream=stream)
        t1 = time.perf_counter()
        e0.record(stream)
        m.cast(x, y, th, MAX_RANGE, out=out_r, stream=stream)
        e1.record(stream)
        stream.synchronize()
        if i >= args.warmup:
            upd_s += t1 - t0
            upd_each.append(t1 - t0)
            cast_s += e0.elapsed_time(e1) / 1e3
    fresh = cddt.Map(t_dev(cur), n, buckets=BUCKETS, zp16=ZP16, prune=PRUNE)
    same = all((a == b).all() for a, b in zip(m.export(), fresh.export()))
    rays = x.numel()
    info = m.info()
    return {"metric": "ray casts/sec with 1000 cell toggles per step (plain cddt_cast)",
            "value": rays * steps / (upd_s + cast_s), "unit": "rays/s", "steps": steps,
            "cast_rays_per_s": rays * steps / cast_s, "update_ms_per_step": upd_s / steps * 1e3,
            "cast_ms_per_step": cast_s / steps * 1e3, "update_equals_rebuild": bool(same),
            "update_ms_median": float(np.median(upd_each) * 1e3), "update_ms_max": float(np.max(upd_each) * 1e3),
            "build_seconds": build_s, "rebuilds": info["rebuilds"],
            "config": {"workload": "updates: 4000^2 room/corridor map, 200 bins, each step 1000 random "
                                   "toggles (incremental update) then 1M particles x 61 rays as plain casts",
                       **{k: v for k, v in info.items() if k in ("zero_points", "rows", "edge_cells", "capacity")}},
            "roofline": {"bound": "hbm", "algorithmic_GBps": rays * BYTES_PER_CAST / (cast_s / steps) / 1e9,
                         "peak": PEAK_HBM_GBS}}


# ---------------------------------------------------------------------------
# Serving
# ---------------------------------------------------------------------------
SERVE_SIDES = (1000, 1500, 2000, 2500, 3000, 3500, 4000, 4000)
# offered load as fractions of the batched capacity (the many-filter step's rays/s, or a plan over one
# request per robot on the serving maps), converted to requests/s with the requests' mean ray count
SERVE_FRACTIONS = (0.10, 0.25, 0.40, 0.55, 0.70, 0.85, 1.00, 1.20)
SERVE_TIGHT_BUDGET = 2 << 20  # bytes: lanes share it, so each batch holds a few dozen requests at most
SERVE_SLOTS = 1024  # ring slots of the resident server (the budget is split among them)
SERVE_SLOT_MIN = 32 << 10  # bytes: a slot holds the largest request (1,639 particles)
SERVE_RESIDENT_TUNING = (8, 2, 8, 7)


def resident_slots(budget: int) -> int:
    return max(1, min(SERVE_SLOTS, budget // SERVE_SLOT_MIN))


def build_serving(buckets):
    import torch
    from paper_1705_01167_amd import cddt
    from paper_1705_01167_amd import workloads as wl
    rng = wl.rng_for(wl.SERVING, wl.S_SPEC)
    maps, offs, tabs, pools, obs = [], [], [], [], []
    off_h = wl.ray_offsets(RAYS)
    for i, side in enumerate(SERVE_SIDES):
        n = int(wl.THETA_CHOICES[int(rng.integers(0, 3))])
        occ = wl.building_map(wl.rng_for(wl.SERVING, wl.S_MAP, i), side, side)
        maps.append(cddt.Map(t_dev(occ), n, buckets=buckets))
        offs.append(off_h)
        tabs.append(t_dev(wl.beam_table(MAX_RANGE, wl.beam_params(wl.rng_for(wl.SERVING, wl.S_TABLE, i)))))
        pools.append(wl.free_poses(wl.rng_for(wl.SERVING, wl.S_POSES, i), occ, 20000))
        obs.append([wl.observations(wl.rng_for(wl.SERVING, wl.S_OBS, 1000 * i + r), occ, off_h, MAX_RANGE)[0]
                    for r in range(4)])
    torch.cuda.synchronize()
    return maps, offs, tabs, pools, obs


def make_requests(k: int, seed: int, pools, obs):
    """Request i: robot i mod 256 on map robot mod 8, log-uniform 17..1639 particles from the map's pool."""
    from paper_1705_01167_amd import workloads as wl
    rng = wl.rng_for(wl.SERVING, wl.S_ARRIVALS, seed)
    out = []
    for i in range(k):
        robot = int(rng.integers(0, 256))
        m = robot % len(pools)
        n = int(round(math.exp(rng.uniform(math.log(17), math.log(1639)))))
        s = int(rng.integers(0, 20000 - n))
        px, py, pth = (a[s:s + n] for a in pools[m])
        out.append((m, px, py, pth, obs[m][robot % len(obs[m])], n))
    return out


SERVE_THREADS = 2  # submitting threads of the load generator (--serve-threads)


def serve_at(srv, reqs, rate: float | None, seed: int):
    """Open-loop Poisson arrivals at `rate` requests/s (None: all at once); latency from scheduled arrival."""
    rng = np.random.default_rng(seed)
    k = len(reqs)
    gaps = rng.exponential(1.0 / rate, k) if rate else np.zeros(k)
    # submitted from native threads at the scheduled offsets (cddt_server_replay_threads)
    ids = srv.replay([r[:5] for r in reqs], np.cumsum(gaps), threads=SERVE_THREADS)
    t_sub = srv.last_replay_seconds
    if (ids < 0).any():
        raise RuntimeError("serving: a request was refused")
    arrive, done = np.empty(k), np.empty(k)
    for i, rid in enumerate(ids.tolist()):
        srv.wait(rid)
        arrive[i], done[i] = srv.times(rid)
    lat = done - arrive
    rays = sum(r[5] for r in reqs) * RAYS
    span = done.max() - arrive[0]
    return {"offered_rps": rate, "completed_rps": k / span, "rays_per_s": rays / span, "submit_seconds": t_sub,
            "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "requests": k}


def serving_plan_capacity(maps, offs, tabs, pools, obs) -> float:
    """Batched capacity on the serving maps: rays/s of one persistent launch over one request per robot."""
    import torch
    from paper_1705_01167_amd import cddt
    reqs = make_requests(256, 7, pools, obs)
    off = [t_dev(o) for o in offs]
    keep, filters = [], []
    for m, px, py, pth, ob, n in reqs:
        d = {"px": t_dev(px), "py": t_dev(py), "pth": t_dev(pth), "obs": t_dev(ob)}
        lw = torch.empty(n, dtype=torch.float32, device="cuda")
        filters.append(cddt.make_filter(maps[m], d["px"], d["py"], d["pth"], off[m], d["obs"], tabs[m], MAX_RANGE,
                                        lw))
        keep.append((d, lw))
    st = torch.cuda.Stream()
    plan = cddt.Plan(filters, stream=st, keepalive=(keep, off))
    plan.time(plan.tuning, reps=3, stream=st)
    ms = min(plan.time(plan.tuning, reps=20, stream=st) for _ in range(3))
    plan.close()
    return sum(r[5] for r in reqs) * RAYS / (ms * 1e-3)


def make_server(maps, offs, tabs, args, mode: str, budget: int):
    """mode: a lane count ('1'..'4': batches on that many streams) or 'r' (one resident kernel, ring slots)."""
    from paper_1705_01167_amd import cddt
    if mode == "r":
        return cddt.Server(maps, offs, tabs, [MAX_RANGE] * len(maps), budget_bytes=budget, n_lanes=1,
                           max_batch=resident_slots(budget), tuning=SERVE_RESIDENT_TUNING, resident=True)
    return cddt.Server(maps, offs, tabs, [MAX_RANGE] * len(maps), budget_bytes=budget, n_lanes=int(mode),
                       max_batch=args.serve_batch)


def run_serving(args, ref_rays_per_s: float | None = None, mode: str | None = None) -> dict:
    """Open-loop Poisson arrivals at SERVE_FRACTIONS of the batched capacity, args.serve_requests each."""
    # the serving maps take a 2^7-cell bucket index unless another layout is asked for
    buckets = 7 if args.buckets.lower() == "auto" else BUCKETS
    mode = mode or str(args.serve_lanes).split(",")[0]
    maps, offs, tabs, pools, obs = build_serving(buckets)
    ref_kind = "the many-filter step's kernel rays/s in this run"
    if ref_rays_per_s is None:
        ref_rays_per_s = serving_plan_capacity(maps, offs, tabs, pools, obs)
        ref_kind = "one persistent launch over one request per robot on the serving maps"
    srv = make_server(maps, offs, tabs, args, mode, args.serve_budget)
    warm = make_requests(500, 0, pools, obs)
    serve_at(srv, warm, None, 0)
    # burst capacity: median of three bursts (every request arrives at once, so batches are as large as the
    # lanes allow)
    caps = sorted((serve_at(srv, make_requests(args.serve_requests, 1 + b, pools, obs), None, 1 + b)
                   for b in range(3)), key=lambda c: c["completed_rps"])
    cap = caps[1]
    points = []
    for j, frac in enumerate(SERVE_FRACTIONS):
        reqs = make_requests(args.serve_requests, 10 + j, pools, obs)
        mean_rays = sum(r[5] for r in reqs) * RAYS / len(reqs)
        rate = frac * ref_rays_per_s / mean_rays
        points.append({"fraction_of_batched_capacity": frac, **serve_at(srv, reqs, float(rate), 10 + j)})
        log(f"bench: serving ({mode}) at {frac:.0%} of batched capacity: {points[-1]}")
    st = srv.stats()
    srv.close()
    # admission limited by memory: a budget of SERVE_TIGHT_BUDGET bytes (a few dozen requests in flight)
    # under the offered load of the 85% point
    tight = make_server(maps, offs, tabs, args, mode, SERVE_TIGHT_BUDGET)
    serve_at(tight, warm, None, 0)
    reqs = make_requests(args.serve_requests, 30, pools, obs)
    rate = 0.85 * ref_rays_per_s / (sum(r[5] for r in reqs) * RAYS / len(reqs))
    budget_point = {"budget_bytes": SERVE_TIGHT_BUDGET, **serve_at(tight, reqs, float(rate), 30),
                    "stats": tight.stats()}
    tight.close()
    log(f"bench: serving with a {SERVE_TIGHT_BUDGET >> 20} MiB budget: {budget_point}")
    return {"batched_capacity_rays_per_s": ref_rays_per_s, "batched_capacity_from": ref_kind,
            "burst_capacity_rps": cap["completed_rps"], "burst_capacity_rays_per_s": cap["rays_per_s"],
            "points": points, "stats": st, "budget_limited": budget_point,
            "config": {"maps": list(SERVE_SIDES), "theta_bins": [m.theta_bins for m in maps], "robots": 256,
                       "request_particles": "log-uniform 17..1639", "bucket_log2": buckets,
                       "budget_bytes": args.serve_budget,
                       "mode": "resident kernel, ring of slots" if mode == "r" else f"{mode} lanes",
                       "slots" if mode == "r" else "max_batch":
                           resident_slots(args.serve_budget) if mode == "r" else args.serve_batch,
                       "requests_per_rate": args.serve_requests, "submitting_threads": SERVE_THREADS,
                       "resident_tuning": list(SERVE_RESIDENT_TUNING) if mode == "r" else None}}


def copy_calibration(mib: int) -> None:
    """A plain device-to-device copy of known size, to scale the HBM byte counters."""
    import torch
    n = mib * (1 << 20)
    a = torch.ones(n, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n, "copy_bytes_written": n, "launches": 3}), flush=True)


def main():
    global BUCKETS, ZP16, PRUNE, SERVE_THREADS, SERVE_SLOTS, SERVE_RESIDENT_TUNING
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="batched",
                    choices=["batched", "small", "floor", "updates", "serving", "suites", "probe"])
    ap.add_argument("--filters", type=int, default=64)
    ap.add_argument("--buckets", type=str, default="auto",
                    help="log2 bucket width in cells of the maps' bucket index, 'none' for no index, or 'auto': "
                         "6 for the batched workload (185 GB of structure), 7 for floor, updates and the serving "
                         "maps, none for small (its map stays in cache)")
    ap.add_argument("--zp16", action="store_true",
                    help="16-bit zero points in the bucket lines (answers follow the 16-bit reading, not the "
                         "exact one; needs a bucket index)")
    ap.add_argument("--prune", action="store_true",
                    help="PCDDT: pruned static maps (answers equal the full structure only from grid states)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving summary")
    ap.add_argument("--no-probe", action="store_true", help="skip the gather-bandwidth probe")
    ap.add_argument("--no-mcl", action="store_true", help="skip the whole-filter-step (motion + resampling) timing")
    ap.add_argument("--cpu-budget", type=float, default=10.0, help="seconds of oracle timing to aim for")
    ap.add_argument("--no-tune-cache", action="store_true")
    ap.add_argument("--tuning", type=str, default=None,
                    help="fixed persistent-kernel tuning 'ppt,waves,blocks,K' (skips the autotuner)")
    ap.add_argument("--no-graph", action="store_true", help="launch the plan directly instead of a graph")
    ap.add_argument("--serve-requests", type=int, default=20000, help="requests per offered rate")
    ap.add_argument("--serve-budget", type=int, default=256 << 20)
    ap.add_argument("--serve-lanes", type=str, default="r",
                    help="batches in flight (streams, 1..4), or r for one resident kernel fed through a ring of "
                         "slots; the serving workload takes a comma-separated list")
    ap.add_argument("--serve-batch", type=int, default=512)
    ap.add_argument("--serve-slots", type=int, default=SERVE_SLOTS,
                    help="ring slots of the resident server (at most budget / 32 KiB)")
    ap.add_argument("--serve-tuning", type=str, default=",".join(map(str, SERVE_RESIDENT_TUNING)),
                    help="resident kernel tuning: particles/tile,waves/block,blocks/CU,search mode")
    ap.add_argument("--serve-threads", type=int, default=2,
                    help="threads of the load generator submitting the arrivals (one thread submits about "
                         "0.6 M requests/s)")
    ap.add_argument("--probe-gib", type=str, default="4", help="probe buffer sizes in GiB, comma separated")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of this many MiB (counter calibration) and exit")
    args = ap.parse_args()
    if args.buckets.lower() == "auto":
        BUCKETS = {"batched": 6, "floor": 7, "updates": 7}.get(args.workload)
    else:
        BUCKETS = None if args.buckets.lower() == "none" else int(args.buckets)
    ZP16 = bool(args.zp16)
    PRUNE = bool(args.prune)
    SERVE_THREADS = max(1, min(16, args.serve_threads))
    SERVE_SLOTS = max(1, min(65536, args.serve_slots))
    SERVE_RESIDENT_TUNING = tuple(int(v) for v in args.serve_tuning.split(","))
    if ZP16 and BUCKETS is None:
        print("--zp16 needs a bucket index (--buckets k)", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (run with --gpus 1).", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1705_01167_amd import cddt
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    cddt.lib()
    if args.workload == "batched":
        out = run_batched(args)
    elif args.workload == "small":
        out = run_small(args)
    elif args.workload == "floor":
        out = run_floor(args)
    elif args.workload == "updates":
        out = run_updates(args)
    elif args.workload == "suites":
        out = run_suites(args)
    elif args.workload == "serving":
        out = {"metric": "serving: completed rays/s and p50/p99 latency vs offered load",
               "runs": [run_serving(args, mode=v) for v in args.serve_lanes.split(",")]}
    else:
        out = {"gather_probe": [cddt.probe_gather(gib=float(g), depth=d) for g in args.probe_gib.split(",")
                                for d in (1, 4)]}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
