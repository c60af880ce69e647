#!/usr/bin/env python3
"""Throughput benchmark of the coarse-path ray launcher on one MI355X.

One step is one pass of the whole hot path over a synthetic scene already
resident in HBM: build_voxels (voxel hierarchy) -> launch_rays (all bounces)
-> collect_paths (dedup, kappa = 100 as in the paper's Table 1).  The
default workload is the furnished room: 12 x 10 x 3 m plus 30 boxes,
~1M points, 20 labels, 1 TX, 16 RX, 1M Fibonacci rays, K = 3, voxel levels
0.5 m / 0.05 m.

Prints ONE JSON line: rays/s of whole steps, plus bounce-segments/s, the
roofline of the dominant kernel (the bounce kernel: algorithmic bytes from
the exact byte counter of a statistics pass, divided by its duration measured
with HIP events in the timed steps) and the CPU oracle timed on a bounded
sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_workload(name):
    import scenes
    if name == "furnished_room":
        return scenes.furnished_room()
    if name == "box_room":
        return scenes.box_room()
    if name == "street_canyon":
        return scenes.street_canyon()
    raise SystemExit(f"unknown workload {name}")


def cpu_baseline(s, t_eps, seconds):
    """Oracle (FP64 brute force, all host threads) on an evenly spaced ray sample."""
    import oracle
    oracle.build(force=False)
    dirs = oracle.fibonacci(s.n_rays)
    threads = oracle.default_threads()
    n_total = s.n_rays * len(s.tx)

    def run(n):
        sel = (np.arange(n, dtype=np.int64) * (n_total // n)).astype(np.int64)
        t0 = time.perf_counter()
        oracle.launch(s.xyz, s.normal, s.label, s.tx, s.rx, dirs, K=s.max_reflections,
                      r_s=float(np.float32(s.surfel_radius)), t_eps=t_eps, sel=sel, n_threads=threads)
        return time.perf_counter() - t0

    n = max(threads, 8)
    dt = run(n)
    n2 = int(min(n_total, max(n, n * seconds / max(dt, 1e-6))))
    n2 = max(threads, (n2 // threads) * threads)
    dt2 = run(n2)
    return {"value": n2 / dt2, "unit": "rays/s", "cores": threads, "kind": "oracle",
            "sample": f"{n2} of {n_total} rays (every {n_total // n2}-th), all {s.max_reflections + 1} segments, "
                      f"FP64 brute force over all {s.n_points} points, {dt2:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="furnished_room", choices=["furnished_room", "box_room", "street_canyon"])
    ap.add_argument("--kappa", type=int, default=100)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-stats", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path "
              "(rays shard trivially; see DESIGN.md for the sharding design)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2402_13747_amd as pcrl
    from tests.parity import t_eps_of

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    log(f"[bench] generating {args.workload}")
    s = make_workload(args.workload)
    K = s.max_reflections
    n_total = s.n_rays * len(s.tx)
    t_eps = float(np.float32(t_eps_of(s)))
    r_s = float(np.float32(s.surfel_radius))
    xyz = torch.from_numpy(s.xyz).to(dev)
    nrm = torch.from_numpy(s.normal).to(dev)
    lab = torch.from_numpy(s.label.view(np.int32)).to(dev)
    tx = torch.from_numpy(s.tx).to(dev)
    rx = torch.from_numpy(s.rx).to(dev)
    torch.cuda.synchronize()
    log(f"[bench] {s.n_points} points, {n_total} rays, K={K}, {len(s.rx)} RX, levels {s.levels}")

    cap = [None]

    def step(timing=False, stats=False, phases=None):
        t0 = time.perf_counter()
        scene = pcrl.build_voxels(xyz, nrm, lab, s.levels, r_s, t_eps=t_eps, device=dev)
        if phases is not None:
            torch.cuda.synchronize()
            phases["build"].append(time.perf_counter() - t0)
            t0 = time.perf_counter()
        launch = pcrl.launch_rays(scene, tx, rx, n_rays=s.n_rays, max_reflections=K, timing=timing, stats=stats)
        if phases is not None:
            torch.cuda.synchronize()
            phases["launch"].append(time.perf_counter() - t0)
            t0 = time.perf_counter()
        paths = pcrl.collect_paths(launch, kappa=args.kappa, capacity=cap[0])
        if phases is not None:
            phases["collect"].append(time.perf_counter() - t0)
        st = launch.stats() if (timing or stats) else None
        info = scene.info()
        launch.release()
        scene.release()
        return st, paths, info

    # warm-up (also sizes the path buffers)
    for w in range(max(args.warmup, 1)):
        st, paths, info = step(timing=True)
        cap[0] = int(paths["n_rows"] * 1.2) + 1024
        log(f"[bench] warmup {w}: rows {paths['n_rows']} keys {paths['n_keys']}")

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    kern_ms = []
    segs = []
    for k in range(args.steps):
        st, paths, info = step(timing=True)
        kern_ms.append(sum(st["kernel_ms"]))
        segs.append(st["segments"])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    log(f"[bench] timed {args.steps} steps in {elapsed:.3f} s")

    ms_per_step = 1e3 * elapsed / args.steps
    rays_per_s = n_total * args.steps / elapsed
    seg_per_s = sum(segs) / elapsed

    # phase breakdown (untimed, synchronised after each phase)
    phases = {"build": [], "launch": [], "collect": []}
    for _ in range(3):
        step(phases=phases)
    breakdown = {k: 1e3 * float(np.median(v)) for k, v in phases.items()}

    roof = None
    algo = None
    if not args.no_stats:
        st_stats, _, _ = step(stats=True)
        algo = st_stats
        avg_ms = float(np.mean(kern_ms))
        bytes_per_step = float(st_stats["algo_bytes"])
        achieved = bytes_per_step / (avg_ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                "kernel": "k_trace (all K+1 bounce launches of a step)",
                "algo_bytes_per_step": int(bytes_per_step), "trace_ms_per_step": round(avg_ms, 4),
                "algo_bytes_per_segment": round(bytes_per_step / max(st_stats["segments"], 1), 1)}

    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle on a ray sample")
        cpu = cpu_baseline(s, t_eps, args.cpu_seconds)

    out = {
        "metric": "rays/s and bounce-segments/s (HBM GB/s % peak); p50/p99 query latency, served vs plain",
        "value": round(rays_per_s, 1),
        "unit": "rays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "points": s.n_points, "rays": n_total, "tx": len(s.tx),
                   "rx": len(s.rx), "max_reflections": K, "levels": list(s.levels), "surfel_radius": r_s,
                   "kappa": args.kappa, "step": "build_voxels + launch_rays + collect_paths"},
        "segments_per_s": round(seg_per_s, 1),
        "launch_rays_per_s": round(n_total / (float(np.mean(kern_ms)) * 1e-3), 1),
        "breakdown_ms": {k: round(v, 3) for k, v in breakdown.items()},
        "scene": {"entries": info["n_entries"], "leaves": info["n_leaves"], "nodes": info["n_nodes"]},
        "paths": {"rows": int(paths["n_rows"]), "keys": int(paths["n_keys"])},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    if algo is not None:
        out["trace_stats"] = {k: algo[k] for k in ("segments", "dda_steps", "leaves_visited", "node_lookups",
                                                   "surfel_tests", "hits", "records", "active")}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
