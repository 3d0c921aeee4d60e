#!/usr/bin/env python3
"""Throughput of the patch-batch hot path on one MI355X.

Default workload: 3D compressible Euler (gamma 1.4), 2048 patches of 16^3
cells (8,388,608 cells, 16x16x8 periodic patch grid), halo 1, first-order
Rusanov finite volumes with explicit Euler at CFL 0.4, FP64 state, smooth
seeded IC (sum of 8 random Fourier modes per primitive).  A step is one full
pass of the fused FV kernel (halo gather, per-cell primitives, face fluxes,
update, and the CFL reduction that yields the next dt on the device).

Prints one JSON line: cell-updates/s over the timed steps (state resident in
HBM), the roofline of the dominant kernel from live HIP-event timing, and the
single-threaded CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "cell-updates/s & % HBM roofline; SRHD step learned vs plain con2prim"
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_sha() -> str:
    h = hashlib.sha256()
    for f in ("pb_fv.hip", "pb_physics.h", "pb_common.h"):
        with open(os.path.join(ROOT, "paper_2608_19273_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(name: str, sha: str, launches_bytes_scale=1.0):
    """HBM bytes per launch of the FV kernel from the committed rocprofv3
    counter summary, if it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    try:
        with open(path) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return None
    if d.get("source_sha") != sha:
        return None
    return d.get("hbm_bytes_per_launch")


def cpu_baseline(target_s: float):
    """The oracle (single-threaded FP64 C) on a bounded sample of the
    workload: the same IC recipe on 4x4x4 patches of 16^3."""
    import oracle
    from paper_2608_19273_amd import inputs as I
    b = I.config1(grid=(4, 4, 4))
    q = b.state
    steps = 0
    t0 = time.perf_counter()
    while True:
        q, _, _ = oracle.fv_step(b, q, cfl=0.4, n_steps=2)
        steps += 2
        el = time.perf_counter() - t0
        if el >= target_s or steps >= 400:
            break
    return {"value": b.total_cells * steps / el, "unit": "cell-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"3D Euler Rusanov FV, same IC recipe on 4x4x4 patches of 16^3 ({b.total_cells} cells), "
                      f"{steps} steps, {el:.1f} s, single thread"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--storage", choices=["fp64", "fp32"], default="fp64")
    ap.add_argument("--slab", type=int, default=0, help="FV z-planes per work-group (0 = library default)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2608_19273_amd as pb
    from paper_2608_19273_amd import inputs as I

    log("building IC")
    b = I.config1(seed=1)
    cells = b.total_cells
    log(f"IC ready: {cells} cells")
    B = pb.PatchBatch(b, storage=args.storage)
    if args.slab:
        B.set_tuning(fv_slab=args.slab)
    B.fv_rusanov_step(cfl=0.4, n_steps=args.warmup)
    torch.cuda.synchronize()
    log("warmup done")

    B.profile(True)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record()
    B.fv_rusanov_step(cfl=0.4, n_steps=args.steps)
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = e0.elapsed_time(e1)
    kern_ms, launches = B.profile_read()
    B.profile(False)
    st = B.stats()
    log(f"timed {args.steps} steps: {gpu_ms:.3f} ms (events), {wall * 1e3:.3f} ms (wall)")

    elapsed = max(wall, gpu_ms / 1e3)
    value = cells * args.steps / elapsed
    es = 8 if args.storage == "fp64" else 4
    bytes_per_cell = 2 * b.n_unknowns * es
    avg_kernel_s = kern_ms / 1e3 / max(launches, 1)
    achieved = cells * bytes_per_cell / avg_kernel_s / 1e9
    sha = kernel_source_sha()
    traffic = load_traffic(f"fv_euler3d_2048x16c_{args.storage}_traffic.json", sha)
    result = {
        "metric": METRIC,
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.storage == "fp64" else "f64 arithmetic, f32 storage",
        "data": "synthetic",
        "config": {"workload": "3D Euler, Rusanov FV + explicit Euler, 2048 patches of 16^3 (8,388,608 cells), "
                               f"halo 1, CFL 0.4, {args.storage.upper()} state, seeded Fourier-mode IC",
                   "patches": b.K, "patch_cells": int(b.p[0]) ** 3, "storage": args.storage},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "fv_step_kernel<Euler<3>>", "avg_launch_us": avg_kernel_s * 1e6,
                     "launches": launches, "algorithmic_bytes_per_launch": cells * bytes_per_cell,
                     "kernel_source_sha": sha},
        "nonfinite_units": st["nonfinite_units"],
    }
    B.close()
    # attainable streaming bandwidth: the library's plain copy kernel, 512 MiB
    # read + 512 MiB written per launch (also the known-traffic reference for
    # the profiler's byte counters)
    src = torch.ones(64 << 20, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    pb.pb_stream_copy(src, dst)
    torch.cuda.synchronize()
    c0 = torch.cuda.Event(enable_timing=True)
    c1 = torch.cuda.Event(enable_timing=True)
    reps = 5
    c0.record()
    for _ in range(reps):
        pb.pb_stream_copy(src, dst)
    c1.record()
    torch.cuda.synchronize()
    copy_gbs = 2 * src.numel() * 8 * reps / (c0.elapsed_time(c1) / 1e3) / 1e9
    result["roofline"]["attainable_copy_GBs"] = copy_gbs
    result["roofline"]["frac_of_attainable"] = achieved / copy_gbs
    del src, dst
    if not args.no_cpu:
        log("timing the CPU oracle")
        result["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
