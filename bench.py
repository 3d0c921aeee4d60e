#!/usr/bin/env python3
"""Throughput of the patch-batch hot path on one MI355X.

Headline workload (the `value` of the JSON line): 3D compressible Euler
(gamma 1.4), 2048 patches of 16^3 cells (8,388,608 cells, 16x16x8 periodic
patch grid), halo 1, first-order Rusanov finite volumes with explicit Euler
at CFL 0.4, FP64 state, smooth seeded IC (sum of 8 random Fourier modes per
primitive).  A step is one full pass of the fused FV kernel (halo gather,
per-cell primitives, face fluxes, update, the largest-speed partials of the
new state) plus the one-work-group reduction that turns them into the next
dt on the device.  State is resident in HBM for the whole timed region.

Further workloads are reported under "workloads": the same Euler batch with
FP32 storage, the 2D Euler entropy wave (64x64 as 8x8 patches of 8^2) eager
and graph-replayed, the uneven 4096-patch batch of the 58-unknown linear
system (FD4 + KO6 + RK4, FP64 matrix cores), the 3D Euler batch advanced by
FD4 + KO6 + RK4 (halo 3, flux differencing), special-relativistic
hydrodynamics on 2048 x 16^3 with the plain, warm and learned con2prim guess,
advection by a velocity field held as material parameters,
the K sweep (runtime per cell against the number of independent patches
for p = 3, 6, 16, FV and FD4), and offload mode (host chunks in and out
through pinned staging and PCIe: total runtime against kernel time).

Prints one compact JSON line on stdout (headline, roofline, CPU baseline and
a one-line summary per further workload); the full result with every table
goes to --detail-out (default gpurun_out/bench_detail.json); progress goes to
stderr.
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
FP64_PEAK_TFLOPS = 78.6


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_sha(files) -> str:
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2608_19273_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(name: str, sha: str, kernel: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if
    it was taken on the current kernel source and the same kernel (else
    None)."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    try:
        with open(path) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return None
    if d.get("source_sha") != sha or d.get("kernel") != kernel:
        return None
    return d.get("hbm_bytes_per_launch")


def timed(torch, fn):
    """seconds taken by fn() (which enqueues GPU work), max of wall clock and
    events on the current stream, synchronised on both sides"""
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record()
    fn()
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return max(wall, e0.elapsed_time(e1) / 1e3)


def cpu_info():
    """CPU model, the logical CPUs of the host and the CPUs this process may
    run on"""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = os.cpu_count() or 1
    return {"cpu_model": model, "nproc": os.cpu_count() or 1, "usable_cpus": usable}


def _oracle_fd_worker(args):
    """one worker of the multi-process oracle leg: repeated one-step RK4
    updates of its own patches of the uneven linear-system batch for about
    `seconds`; returns (cell-steps, seconds)"""
    subset, seconds = args
    import oracle
    from paper_2608_19273_amd import inputs as I
    b = I.config2(subset=subset)
    q = b.state
    steps = 0
    t0 = time.perf_counter()
    while True:
        q = oracle.fd_step(b, q, cfl=0.5, sigma=0.1, n_steps=1)[0]
        steps += 1
        el = time.perf_counter() - t0
        if el >= seconds:
            return b.total_cells * steps, el


def cpu_oracle_multiprocess(workers: int, seconds: float):
    """The same single-threaded oracle run as `workers` independent processes
    (spawned, so none of them inherits the GPU context), each advancing its
    own patches of the uneven 58-unknown batch (one 4^3, two 8^3 and one 16^3
    patch per worker, the batch's 1:2:1 mix): an embarrassingly parallel
    oracle throughput over independent patches, labelled as such."""
    import multiprocessing as mp
    from paper_2608_19273_amd import inputs as I
    sizes = I.config2_sizes()
    pools = {p: list(map(int, (sizes == p).nonzero()[0])) for p in (4, 8, 16)}
    jobs = []
    for w in range(workers):
        sub = [pools[4][w], pools[8][2 * w], pools[8][2 * w + 1], pools[16][w]]
        jobs.append((sorted(sub), seconds))
    t0 = time.perf_counter()
    with mp.get_context("spawn").Pool(workers) as pool:
        res = pool.map(_oracle_fd_worker, jobs)
    wall = time.perf_counter() - t0
    rate = sum(c / s for c, s in res)
    return {"value": rate, "unit": "cell-steps/s", "cores": workers, "kind": "oracle, multi-process",
            "sample": f"{workers} spawned processes, each one-step RK4 FD4 + KO6 updates of its own 4 patches "
                      f"(4^3, 2x 8^3, 16^3) of the 58-unknown batch for {seconds:.0f} s; rate = sum of the "
                      f"per-process rates; wall {wall:.1f} s"}


def cpu_baseline(target_s: float):
    """The oracle (single-threaded FP64 C) on a bounded sample of the
    headline workload: the same IC recipe on 4x4x4 patches of 16^3."""
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
                      f"{steps} steps, {el:.1f} s, single thread", **cpu_info()}


def cpu_oracle_sample(kind: str, target_s: float):
    """The oracle (single-threaded FP64 C) on a bounded sample of a further
    workload, for context beside its GPU rate: the linear system on one 4^3,
    two 8^3 and one 16^3 patch of the uneven batch (its 1:2:1 size mix), SRHD
    on 2 x 2 x 1 patches of 16^3 with the same primitive recipe."""
    import oracle
    from paper_2608_19273_amd import inputs as I
    if kind == "linsym":
        b = I.config2(subset=I.config2_subset(n_per_size=(1, 2, 1)))
        step = lambda q: oracle.fd_step(b, q, cfl=0.5, sigma=0.1, n_steps=1)[0]
        unit, what = "cell-steps/s", "FD4 + KO6 + RK4 steps of the 58-unknown linear system"
    else:
        b = I.config3(grid=(2, 2, 1))
        step = lambda q: oracle.fv_step(b, q, cfl=0.4, n_steps=1)[0]
        unit, what = "cell-updates/s", "SRHD Rusanov FV steps with plain-guess con2prim"
    q = b.state
    steps = 0
    t0 = time.perf_counter()
    while True:
        q = step(q)
        steps += 1
        el = time.perf_counter() - t0
        if el >= target_s or steps >= 1000:
            break
    return {"value": b.total_cells * steps / el, "unit": unit, "cores": 1, "kind": "oracle",
            "sample": f"{what} on {b.p.size} patches ({b.total_cells} cells), {steps} steps, {el:.1f} s, "
                      f"single thread"}


def attainable_copy(torch, pb):
    """the library's streaming copy, 512 MiB read + 512 MiB written per launch"""
    src = torch.ones(64 << 20, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(5):
        pb.pb_stream_copy(src, dst)
    reps = 20
    el = timed(torch, lambda: [pb.pb_stream_copy(src, dst) for _ in range(reps)])
    return 2 * src.numel() * 8 * reps / el / 1e9


RETUNE = False
MIN_WARMUP_S = 0.5


def tune(B, kind, euler=False, **kw):
    """the library's autotuner on batch B (outside any timed region): the
    cached choice for this workload if the tuning file holds one, else a
    measured search; returns a summary of what was used (euler: the FD
    candidates are the Euler stage kernel's column runs)"""
    r = B.autotune(kind, trials=3, use_cache=not RETUNE, **kw)

    def name(t):
        if kind == "fv":
            if t.get("fv_column"):
                return f"column{t['fv_column']}/remap{t['fv_xcd_remap']}"
            if t.get("fv_persist"):
                return f"balanced{t['fv_persist']}/remap{t['fv_xcd_remap']}"
            return f"slab{t['fv_slab']}/remap{t['fv_xcd_remap']}/dma{t['fv_dma']}"
        if euler:
            return f"column{t['fd_column']}/remap{t['fd_xcd_remap']}"
        if t["fd_ws"]:
            return f"ws/remap{t['fd_xcd_remap']}"
        return f"remap{t['fd_xcd_remap']}/wg{t['fd_wg_per_cu']}"
    return {"chosen": name(r["best"]), "from_cache": r["from_cache"],
            "candidates_us": {name(t): round(us, 2) for t, us in r["candidates"]}}


def bench_euler3d(torch, pb, b, storage, steps, warmup):
    B = pb.PatchBatch(b, storage=storage)
    tuned = tune(B, "fv", cfl=0.4)
    extra = warm_up(torch, B, lambda n: B.fv_rusanov_step(cfl=0.4, n_steps=n), warmup, MIN_WARMUP_S)
    # one event pair over the call's back-to-back step launches (span mode):
    # a pair per launch costs the stream a few microseconds per step
    B.profile(True, span=True)
    el = timed(torch, lambda: B.fv_rusanov_step(cfl=0.4, n_steps=steps))
    kern_ms, launches = B.profile_read()
    B.profile(False)
    st = B.stats()
    tuning = B.get_tuning()
    B.close()
    cells = b.total_cells
    es = 8 if storage == "fp64" else 4
    bpc = 2 * b.n_unknowns * es
    avg_s = kern_ms / 1e3 / max(launches, 1)
    return {"cell_updates_per_s": cells * steps / el, "ms_per_step": el * 1e3 / steps,
            "kernel_avg_us": avg_s * 1e6, "launches": launches, "bytes_per_cell": bpc,
            "kernel_GBs": cells * bpc / avg_s / 1e9, "nonfinite_units": st["nonfinite_units"],
            "warmup_extra_steps": extra, "autotune": tuned, "tuning": tuning}


def bench_config0(torch, pb, I, calls):
    b = I.config0()
    out = {}
    for graph in (False, True):
        B = pb.PatchBatch(b)
        B.fv_rusanov_step(cfl=0.4, n_steps=10, use_graph=graph)
        el = timed(torch, lambda: [B.fv_rusanov_step(cfl=0.4, n_steps=10, use_graph=graph)
                                   for _ in range(calls)])
        B.close()
        out["graph" if graph else "eager"] = {"cell_updates_per_s": b.total_cells * 10 * calls / el,
                                              "us_per_step": el * 1e6 / (10 * calls)}
    return out


def bench_fd(torch, pb, I, steps, warmup):
    log("config-2 IC (4096 patches, 58 unknowns)")
    b = I.config2()
    cells = b.total_cells
    B = pb.PatchBatch(b)
    tuned = tune(B, "fd", cfl=0.5, sigma_ko=0.1)
    extra = warm_up(torch, B, lambda n: B.fd_ko_step(cfl=0.5, sigma_ko=0.1, n_steps=n), warmup, MIN_WARMUP_S,
                    chunk=5)
    # eager, with every stage launch timed by its own dispatch events
    B.profile(True)
    el_eager = timed(torch, lambda: B.fd_ko_step(cfl=0.5, sigma_ko=0.1, n_steps=steps))
    kern_ms, launches = B.profile_read()
    B.profile(False)
    # the same steps captured once into a HIP graph (outside the timed
    # region), then replayed: the configuration's execution mode
    B.fd_ko_step(cfl=0.5, sigma_ko=0.1, n_steps=steps, use_graph=True)
    el = timed(torch, lambda: B.fd_ko_step(cfl=0.5, sigma_ko=0.1, n_steps=steps, use_graph=True))
    st = B.stats()
    B.close()
    N = b.n_unknowns
    # per RK4 step: 4 x (3 dense N x N products + 3 D4 (4 flop) + 3 KO6 (9 flop) + update) per unknown
    flop_cell = 4 * (3 * 2 * N * N + N * (3 * 4 + 3 * 9 + 4))
    bytes_cell = 16 * N * 8
    step_kernel_s = kern_ms / 1e3 / max(launches, 1) * 4
    return {"workload": "linear symmetric system N=58, 4096 patches {4^3,8^3,16^3} 1:2:1 shuffled "
                        f"({cells} cells), FD4 + KO6 (sigma 0.1) + RK4, CFL 0.5, FP64",
            "cell_updates_per_s": cells * steps / el, "ms_per_step": el * 1e3 / steps, "use_graph": True,
            "ms_per_step_eager": el_eager * 1e3 / steps, "warmup_extra_steps": extra,
            "stage_kernel_avg_us": kern_ms * 1e3 / max(launches, 1), "nonfinite_units": st["nonfinite_units"],
            "hbm_frac": cells * bytes_cell / step_kernel_s / 1e9 / HBM_PEAK_GBS,
            "fp64_frac": cells * flop_cell / step_kernel_s / 1e12 / FP64_PEAK_TFLOPS,
            "algorithmic_bytes_per_cell_step": bytes_cell, "algorithmic_flop_per_cell_step": flop_cell,
            "autotune": tuned}


def bench_fd_euler(torch, pb, I, steps, warmup):
    log("config-1 IC with a halo of 3 (Euler FD4 + KO6 + RK4)")
    b = I.config1(seed=1, halo=3)
    cells = b.total_cells
    B = pb.PatchBatch(b)
    tuned = tune(B, "fd", euler=True, cfl=0.5, sigma_ko=0.1)
    extra = warm_up(torch, B, lambda n: B.fd_ko_step(cfl=0.5, sigma_ko=0.1, n_steps=n), warmup, MIN_WARMUP_S)
    B.profile(True)
    el = timed(torch, lambda: B.fd_ko_step(cfl=0.5, sigma_ko=0.1, n_steps=steps))
    kern_ms, launches = B.profile_read()
    B.profile(False)
    st = B.stats()
    B.close()
    N = b.n_unknowns
    # per RK4 step, state-sized arrays in + out: stage 1 reads Q^n, writes the
    # next stage value and the running sum; stages 2-3 read the stage value,
    # Q^n and the sum, write two; stage 4 reads the stage value and the sum,
    # writes Q^{n+1}: (1+2) + (3+2) + (3+2) + (2+1) = 16 arrays of N doubles
    bytes_cell = 16 * N * 8
    step_kernel_s = kern_ms / 1e3 / max(launches, 1) * 4
    return {"workload": "3D Euler, FD4 + KO6 (sigma 0.1) + RK4, CFL 0.5, 2048 patches of 16^3 "
                        f"({cells} cells) joined by face neighbours, halo 3, FP64, seeded Fourier-mode IC",
            "cell_updates_per_s": cells * steps / el, "ms_per_step": el * 1e3 / steps,
            "stage_kernel_avg_us": kern_ms * 1e3 / max(launches, 1), "launches": launches,
            "algorithmic_bytes_per_cell_step": bytes_cell,
            "kernel_GBs": cells * bytes_cell / step_kernel_s / 1e9,
            "hbm_frac": cells * bytes_cell / step_kernel_s / 1e9 / HBM_PEAK_GBS,
            "nonfinite_units": st["nonfinite_units"], "warmup_extra_steps": extra, "autotune": tuned}


KSWEEP_K = (1, 4, 16, 64, 256, 1024, 4096, 8694, 16384)


def bench_ksweep(torch, pb, I, k_max_16=8694):
    """Runtime per cell against the batch size K (the shape of the paper's
    main experiment): K independent 3D Euler patches of p^3 cells for
    p in {3, 6, 16} (smooth seeded state per patch), the FV step (CFL 0.4) and the FD4 + KO6 + RK4 step (CFL
    0.5, sigma 0.1), eager launches and the same steps replayed from a HIP
    graph, each timed by wall clock and events; per cell means per
    cell-update (FV) and per cell-step of all four RK stages (FD).  Also the
    58-unknown linear system (FD4 + KO6 + RK4 on the FP64 matrix cores) on K
    independent patches of p in {4, 8, 16}."""
    out = {}
    for scheme in ("fv", "fd"):
        for p in (3, 6, 16):
            rows = []
            for K in KSWEEP_K:
                if p == 16 and K > k_max_16:
                    continue
                b = I.independent_euler_patches_smooth(7, K, p, halo=3 if scheme == "fd" else 1)
                cells = b.total_cells
                B = pb.PatchBatch(b)
                if scheme == "fv":
                    step = lambda n, g: B.fv_rusanov_step(cfl=0.4, n_steps=n, use_graph=g)
                else:
                    step = lambda n, g: B.fd_ko_step(cfl=0.5, sigma_ko=0.1, n_steps=n, use_graph=g)
                n = int(min(200 if scheme == "fv" else 100,
                            max(3, round(5e7 / (cells * (4 if scheme == "fd" else 1))))))
                step(1, False)
                el = timed(torch, lambda: step(n, False))
                step(n, True)   # capture (and one replay) outside the timed region
                elg = timed(torch, lambda: step(n, True))
                st = B.stats()
                B.close()
                # a row that computed a non-finite value timed something else
                # than the update of a valid state: kept in the table, flagged
                rows.append({"K": K, "cells": cells, "steps": n, "ns_per_cell": el / (n * cells) * 1e9,
                             "us_per_step": el / n * 1e6, "ns_per_cell_graph": elg / (n * cells) * 1e9,
                             "us_per_step_graph": elg / n * 1e6, "nonfinite_units": st["nonfinite_units"],
                             "valid": st["nonfinite_units"] == 0})
                del b
            out[f"{scheme}_p{p}"] = rows
            log(f"k-sweep {scheme} p={p}: " + ", ".join(f"K={r['K']}: {r['ns_per_cell']:.3f}/{r['ns_per_cell_graph']:.3f} ns"
                                                      for r in rows))
    # the 58-unknown linear system (the FD4 path on the FP64 matrix cores) on
    # K independent patches of one size, i.i.d. U(-1, 1) state
    import numpy as np
    Bs, rhos = I.linsym_matrices(2, 58)
    prm = I.linsym_params(Bs, rhos)
    for p in (4, 8, 16):
        rows = []
        for K in (1, 16, 256, 1024, 4096):
            if p == 16 and K > 1024:
                continue
            cells = K * p ** 3
            b = I.Batch(dim=3, p=np.full(K, p, np.int32), dx=np.full(K, 1.0 / p), nbr=I.self_periodic(K, 3),
                        halo=3, pde="linsym", params=prm, n_unknowns=58,
                        state=I.uniform(13, cells * 58, -1.0, 1.0))
            B = pb.PatchBatch(b)
            n = int(min(50, max(2, round(2e6 / cells))))
            B.fd_ko_step(cfl=0.5, sigma_ko=0.1, n_steps=1)
            el = timed(torch, lambda: B.fd_ko_step(cfl=0.5, sigma_ko=0.1, n_steps=n))
            st = B.stats()
            B.close()
            rows.append({"K": K, "cells": cells, "steps": n, "ns_per_cell": el / (n * cells) * 1e9,
                         "us_per_step": el / n * 1e6, "nonfinite_units": st["nonfinite_units"],
                         "valid": st["nonfinite_units"] == 0})
            del b
        out[f"fd_linsym58_p{p}"] = rows
        log(f"k-sweep linsym58 p={p}: " + ", ".join(f"K={r['K']}: {r['ns_per_cell']:.2f} ns" for r in rows))
    return out


def bench_offload(pb, I):
    """Offload mode (the paper's pure kernel offloading): K host chunks of 3D
    Euler patches with a halo of 1 in, updated interiors out, one FV step per
    call, dt fixed; total runtime (wall clock of the call, host packing and
    PCIe copies included) against the kernel time, per cell.  Median of 5
    calls after one warm-up call."""
    import numpy as np
    out = {}
    for p, Ks in ((3, (1024, 16384)), (6, (256, 4096)), (16, (64, 512, 2048))):
        rows = []
        for K in Ks:
            chunks = I.independent_halo_chunks(11, K, p, 1)
            outs = [np.empty((p, p, p, 5)) for _ in range(K)]
            dx = np.full(K, 1.0 / p)
            o = pb.Offload(p, 1, "euler", [1.4], 5)
            o.fv_step(chunks, outs, dx, 1e-3)
            ts = [o.fv_step(chunks, outs, dx, 1e-3) for _ in range(5)]
            o.close()
            ts.sort(key=lambda t: t["total_ms"])
            t = ts[2]
            cells = K * p ** 3
            rows.append({"K": K, "cells": cells, "total_ns_per_cell": t["total_ms"] * 1e6 / cells,
                         "compute_ns_per_cell": t["compute_ms"] * 1e6 / cells,
                         **{k: round(v, 4) for k, v in t.items()}})
            del chunks, outs
        out[f"p{p}"] = rows
        log(f"offload p={p}: " + ", ".join(f"K={r['K']}: total {r['total_ns_per_cell']:.3f} ns, "
                                          f"compute {r['compute_ns_per_cell']:.3f} ns" for r in rows))
    return out


def bench_adv_var(torch, pb, I, steps, warmup):
    """Advection by a velocity field held as material parameters on 2048
    patches of 16^3 (the headline grid), FP64: the three field values per
    cell are read and carried through, so a cell-update moves 4 values in
    and 4 out (64 B)."""
    log("variable-coefficient advection IC (2048 x 16^3, field as material parameters)")
    b = I.adv_var_batch((16, 16, 8), 16, kappa=0.0, field="random")
    cells = b.total_cells
    B = pb.PatchBatch(b)
    B.fv_rusanov_step(cfl=0.5, n_steps=warmup)
    B.profile(True, span=True)
    el = timed(torch, lambda: B.fv_rusanov_step(cfl=0.5, n_steps=steps))
    kern_ms, launches = B.profile_read()
    B.profile(False)
    st = B.stats()
    B.close()
    avg_s = kern_ms / 1e3 / max(launches, 1)
    return {"workload": "3D linear advection, velocity field as M = 3 material parameters per cell, Rusanov FV, "
                        f"CFL 0.5, 2048 patches of 16^3 ({cells} cells), FP64",
            "cell_updates_per_s": cells * steps / el, "ms_per_step": el * 1e3 / steps,
            "kernel_avg_us": avg_s * 1e6, "bytes_per_cell": 64, "kernel_GBs": cells * 64 / avg_s / 1e9,
            "hbm_frac": cells * 64 / avg_s / 1e9 / HBM_PEAK_GBS, "nonfinite_units": st["nonfinite_units"]}


def newton_distribution(torch, pb, B, b, guess, net):
    """Newton iteration counts per cell on the batch's current state through
    the con2prim entry point with the same guess (outside any timed region):
    mean, p99, max, and the per-wave maximum (64 consecutive cells of a
    patch, the lanes of one wave of the con2prim pass), which sets a wave's
    cost"""
    import numpy as np
    K, c3 = int(b.p.size), int(b.p[0]) ** 3
    cons = B.current().view(K, 5, c3).permute(1, 0, 2).contiguous().view(5, -1)
    prim = torch.empty_like(cons)
    it = torch.empty(cons.shape[1], dtype=torch.int32, device=cons.device)
    pb.con2prim(cons, prim, guess=guess, mlp=net if guess == "learned" else None, iters=it)
    a = it.cpu().numpy().astype(np.int64)
    wave = a.reshape(-1, 64).max(axis=1)
    return {"cells": int(a.size), "mean": float(a.mean()), "p99": float(np.percentile(a, 99)), "max": int(a.max()),
            "per_wave_max_mean": float(wave.mean()), "per_wave_max_p99": float(np.percentile(wave, 99))}


def bench_srhd(torch, pb, I, steps, mlp_epochs, mlp_pairs, rounds=12, min_warmup_s=0.5):
    """SRHD on the configuration's i.i.d. state, for the plain, warm and
    learned con2prim guess.  Each repetition restores the initial state
    (a device copy, outside the events) and clears the counters, then runs
    either one step (the step on the configured state) or `steps` steps
    (the run from it, the state smoothing as it goes); the three guesses
    alternate repetition by repetition, so clock drift falls on all of them
    alike.  The warm start has no previous pressure in a run's first step
    and takes the plain guess there."""
    import numpy as np
    from paper_2608_19273_amd import mlp_train
    log("config-3 IC (SRHD, 2048 x 16^3)")
    b = I.config3()
    cells = b.total_cells
    res = {"workload": "3D SRHD Gamma 5/3, 2048 patches of 16^3, Rusanov FV, CFL 0.4, FP64; i.i.d. primitives "
                       "rho, eps log-uniform [1e-3,10], W uniform [1,10]; con2prim tol 1e-12, max 50 iterations",
           "timing": f"events around the step call; the initial state restored before every repetition; "
                     f"{rounds} rounds of (1 step, {steps} steps) per guess, the guesses interleaved"}
    log(f"training the guess network ({mlp_pairs} pairs, {mlp_epochs} epochs)")
    t0 = time.perf_counter()
    net, hist = mlp_train.train(n_pairs=mlp_pairs, epochs=mlp_epochs, batch=8192)
    torch.cuda.synchronize()
    res["mlp_training"] = {"seconds": time.perf_counter() - t0, "steps": hist["steps"],
                           "final_epoch_loss": hist["epoch_loss"][-1]}
    guesses = ("plain", "warm", "learned")
    Bs, tuned = {}, {}
    for g in guesses:
        B = pb.PatchBatch(b)
        tuned[g] = tune(B, "fv", cfl=0.4)   # measured for the first mode, then from the cache
        if g != "plain":
            B.set_c2p_guess(g, net if g == "learned" else None)
        Bs[g] = B
    ic = Bs["plain"].bufs[0].clone()
    dist_ic = {g: newton_distribution(torch, pb, Bs[g], b, g, net) for g in ("plain", "learned")}

    def rep(g, n):
        B = Bs[g]
        B.bufs[0].copy_(ic)
        B.reset()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        B.fv_rusanov_step(cfl=0.4, n_steps=n)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1)

    t0 = time.perf_counter()
    while time.perf_counter() - t0 < min_warmup_s:
        for g in guesses:
            rep(g, steps)
    t1 = {g: [] for g in guesses}
    tn = {g: [] for g in guesses}
    st1, stn = {}, {}
    for r in range(rounds):
        order = guesses[r % 3:] + guesses[:r % 3]
        for g in order:
            t1[g].append(rep(g, 1))
            st1[g] = Bs[g].stats()
        for g in order:
            tn[g].append(rep(g, steps))
            stn[g] = Bs[g].stats()
    for g in guesses:
        s1, sn = st1[g], stn[g]
        res[g] = {"step1_ms": float(np.mean(t1[g])), "step1_ms_min": float(np.min(t1[g])),
                  "step1_ms_median": float(np.median(t1[g])),
                  "run_ms_per_step": float(np.mean(tn[g])) / steps,
                  "run_ms_per_step_median": float(np.median(tn[g])) / steps, "run_steps": steps,
                  "cell_updates_per_s_step1": cells / (float(np.mean(t1[g])) * 1e-3),
                  "cell_updates_per_s_run": cells * steps / (float(np.mean(tn[g])) * 1e-3),
                  "newton_mean_step1": s1["c2p_iterations"] / max(s1["c2p_cells"], 1),
                  "newton_max_step1": s1["c2p_max_iterations"],
                  "newton_mean_run": sn["c2p_iterations"] / max(sn["c2p_cells"], 1),
                  "newton_max_run": sn["c2p_max_iterations"],
                  "c2p_failures": s1["c2p_failures"] + sn["c2p_failures"],
                  "fallbacks": s1["c2p_fallbacks"] + sn["c2p_fallbacks"], "autotune": tuned[g]}
        if g in dist_ic:
            res[g]["newton_distribution_initial_state"] = dist_ic[g]
            res[g]["newton_distribution_final_state"] = newton_distribution(torch, pb, Bs[g], b, g, net)
    # per-step times of one run from the initial state (one call per step)
    for g in ("plain", "learned"):
        B = Bs[g]
        B.bufs[0].copy_(ic)
        B.reset()
        per = []
        for s in range(steps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            B.fv_rusanov_step(cfl=0.4, n_steps=1)
            e1.record()
            torch.cuda.synchronize()
            per.append(e0.elapsed_time(e1))
        res[g]["per_step_ms"] = per
    for B in Bs.values():
        B.close()
    res["learned_over_plain_step1"] = res["plain"]["step1_ms"] / res["learned"]["step1_ms"]
    res["learned_over_plain_run"] = res["plain"]["run_ms_per_step"] / res["learned"]["run_ms_per_step"]
    net.close()
    return res


def warm_up(torch, B, step_fn, warmup, min_seconds, chunk=50):
    """W untimed steps, then further untimed steps until at least
    `min_seconds` of warm-up have passed: the first ~200 launches after an
    idle spell run about 15 % slower than the sustained rate (clock and power
    state ramp), which a short W does not cover.  Returns the extra steps."""
    t0 = time.perf_counter()
    if warmup > 0:
        step_fn(warmup)
    torch.cuda.synchronize()
    extra = 0
    while time.perf_counter() - t0 < min_seconds:
        step_fn(chunk)
        torch.cuda.synchronize()
        extra += chunk
    return extra


def compact(result):
    """The one-line summary the driver parses (a few hundred bytes per
    workload): headline, roofline, CPU baseline and one line per further
    workload; the full tables go to the detail file."""
    keep = ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
            "vs_baseline", "dtype", "data", "config", "nonfinite_units")
    out = {k: result[k] for k in keep if k in result}
    r = result["roofline"]
    out["roofline"] = {k: r[k] for k in ("bound", "achieved", "peak", "unit", "frac", "traffic", "kernel",
                                         "avg_launch_us", "attainable_copy_GBs", "frac_of_attainable")}
    out["warmup_extra_steps"] = result.get("warmup_extra_steps")
    if "cpu_baseline" in result:
        out["cpu_baseline"] = result["cpu_baseline"]
    wl = result.get("workloads", {})
    s = {}
    r3 = lambda v: None if v is None else float(f"{v:.4g}")
    if "euler3d_fp32_storage" in wl:
        w = wl["euler3d_fp32_storage"]
        s["euler3d_fp32"] = {"cell_updates_per_s": r3(w["cell_updates_per_s"]), "kernel_us": r3(w["kernel_avg_us"]),
                             "hbm_frac": r3(w["hbm_frac"])}
    if "euler2d_64x64_config0" in wl:
        w = wl["euler2d_64x64_config0"]
        s["euler2d_config0_us_per_step"] = {k: r3(v["us_per_step"]) for k, v in w.items()}
    if "advection_material_field" in wl:
        w = wl["advection_material_field"]
        s["adv_material_field"] = {"kernel_us": r3(w["kernel_avg_us"]), "hbm_frac": r3(w["hbm_frac"])}
    if "linsym58_fd4_rk4" in wl:
        w = wl["linsym58_fd4_rk4"]
        s["linsym58_fd4_rk4"] = {"ms_per_step": r3(w["ms_per_step"]), "stage_us": r3(w["stage_kernel_avg_us"]),
                                 "hbm_frac": r3(w["hbm_frac"]), "fp64_frac": r3(w["fp64_frac"]),
                                 "graph": w.get("use_graph")}
        if "cpu_oracle" in w:
            s["linsym58_fd4_rk4"]["cpu_oracle_cell_steps_per_s"] = r3(w["cpu_oracle"]["value"])
    if "euler3d_fd4_rk4" in wl:
        w = wl["euler3d_fd4_rk4"]
        s["euler3d_fd4_rk4"] = {"ms_per_step": r3(w["ms_per_step"]), "hbm_frac": r3(w["hbm_frac"]),
                                "nonfinite_units": w["nonfinite_units"]}
    if "srhd" in wl:
        w = wl["srhd"]
        s["srhd"] = {g: {"step1_ms": r3(w[g]["step1_ms"]), "run_ms_per_step": r3(w[g]["run_ms_per_step"]),
                         "newton_mean_step1": r3(w[g]["newton_mean_step1"]),
                         "newton_mean_run": r3(w[g]["newton_mean_run"]), "newton_max": w[g]["newton_max_step1"],
                         "failures": w[g]["c2p_failures"], "fallbacks": w[g]["fallbacks"]}
                     for g in ("plain", "warm", "learned")}
        s["srhd"]["learned_over_plain_step1"] = r3(w["learned_over_plain_step1"])
        s["srhd"]["learned_over_plain_run"] = r3(w["learned_over_plain_run"])
        s["srhd"]["run_steps"] = w["plain"]["run_steps"]
        s["srhd"]["mlp_training_s"] = r3(w["mlp_training"]["seconds"])
    if "k_sweep" in wl:
        rows = [row for v in wl["k_sweep"].values() for row in v]
        s["k_sweep"] = {"rows": len(rows), "invalid_rows": sum(1 for row in rows if not row.get("valid", True))}
    if "offload" in wl:
        s["offload_p16_K2048"] = {k: r3(v) for k, v in wl["offload"]["p16"][-1].items()
                                  if k in ("total_ns_per_cell", "compute_ns_per_cell")}
    if "cpu_oracle_multiprocess" in result:
        m = result["cpu_oracle_multiprocess"]
        s["cpu_oracle_multiprocess"] = {"value": r3(m["value"]), "unit": m["unit"], "cores": m["cores"]}
    if s:
        out["workloads"] = s
    out["detail_file"] = result.get("detail_file")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--min-warmup-seconds", type=float, default=0.5,
                    help="untimed warm-up steps continue until this much time has passed")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--cpu-workers", type=int, default=0,
                    help="processes of the multi-process oracle leg (0 = usable CPUs, at most 16)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--only-headline", action="store_true", help="skip the further workloads")
    ap.add_argument("--workloads", default="fp32,config0,advvar,linsym,fdeuler,srhd,ksweep,offload",
                    help="comma list of the further workloads to run")
    ap.add_argument("--mlp-epochs", type=int, default=20)
    ap.add_argument("--mlp-pairs", type=int, default=1 << 22)
    ap.add_argument("--tuning-file", default=os.path.join(ROOT, "paper_2608_19273_amd", "tuning_gfx950.txt"),
                    help="autotuner cache to start from (measured launch shapes per workload)")
    ap.add_argument("--retune", action="store_true", help="measure every workload's candidates again")
    ap.add_argument("--save-tuning", default=None, help="write the autotuner cache here at the end")
    ap.add_argument("--detail-out", default=os.path.join(ROOT, "gpurun_out", "bench_detail.json"),
                    help="file for the full result (every table); stdout gets the one-line summary")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "bench.py runs on one GPU; there is no multi-GPU path (--gpus must be 1)"}))
        sys.exit(2)

    import torch

    import paper_2608_19273_amd as pb
    from paper_2608_19273_amd import inputs as I

    global RETUNE, MIN_WARMUP_S
    RETUNE = args.retune
    MIN_WARMUP_S = args.min_warmup_seconds
    if not args.retune and os.path.exists(args.tuning_file):
        log(f"tuning cache: {pb.pb_autotune_cache_load(args.tuning_file)} entries from {args.tuning_file}")

    log("config-1 IC (3D Euler, 2048 x 16^3)")
    b1 = I.config1(seed=1)
    cells = b1.total_cells
    log("headline: 3D Euler FP64")
    h = bench_euler3d(torch, pb, b1, "fp64", args.steps, args.warmup)
    copy_gbs = attainable_copy(torch, pb)
    sha = kernel_source_sha(("pb_fv.hip", "pb_physics.h", "pb_common.h"))
    kernel = ("fv_step_dma_kernel<Euler<3>, double, true>" if h["tuning"]["fv_dma"]
              else "fv_step_kernel<Euler<3>, 3, double, true>")
    traffic = load_traffic("fv_euler3d_2048x16c_fp64_traffic.json", sha, kernel)
    achieved = h["kernel_GBs"]
    result = {
        "metric": METRIC,
        "value": h["cell_updates_per_s"],
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": h["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "3D Euler, Rusanov FV + explicit Euler, 2048 patches of 16^3 (8,388,608 cells), "
                               "halo 1, CFL 0.4, FP64 state, seeded Fourier-mode IC",
                   "patches": b1.K, "patch_cells": int(b1.p[0]) ** 3, "storage": "fp64"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": kernel, "avg_launch_us": h["kernel_avg_us"],
                     "avg_launch_timing": "HIP events: the first step launch's start to the last's end, "
                                          "over the launch count (the launches follow each other directly)",
                     "launches": h["launches"], "algorithmic_bytes_per_launch": cells * h["bytes_per_cell"],
                     "attainable_copy_GBs": copy_gbs, "frac_of_attainable": achieved / copy_gbs,
                     "kernel_source_sha": sha},
        "nonfinite_units": h["nonfinite_units"],
        "warmup_extra_steps": h["warmup_extra_steps"],
        "autotune": h["autotune"],
    }
    log(f"headline {h['cell_updates_per_s'] / 1e9:.2f} G cell-updates/s, kernel {h['kernel_avg_us']:.1f} us, "
        f"frac {achieved / HBM_PEAK_GBS:.3f}")
    if not args.only_headline:
        wl = {}
        want = set(args.workloads.split(","))
        if "fp32" in want:
            log("3D Euler FP32 storage")
            f32 = bench_euler3d(torch, pb, b1, "fp32", args.steps, args.warmup)
            f32["hbm_frac"] = f32["kernel_GBs"] / HBM_PEAK_GBS
            wl["euler3d_fp32_storage"] = f32
        del b1
        if "config0" in want:
            log("2D Euler entropy wave")
            wl["euler2d_64x64_config0"] = bench_config0(torch, pb, I, 10)
        if "advvar" in want:
            log("advection by a material-parameter velocity field")
            wl["advection_material_field"] = bench_adv_var(torch, pb, I, args.steps, args.warmup)
        if "linsym" in want:
            log("FD4 + KO6 + RK4, 58 unknowns")
            wl["linsym58_fd4_rk4"] = bench_fd(torch, pb, I, max(2, args.steps // 4), 1)
        if "fdeuler" in want:
            log("FD4 + KO6 + RK4, 3D Euler")
            wl["euler3d_fd4_rk4"] = bench_fd_euler(torch, pb, I, args.steps, 1)
        if "srhd" in want:
            log("SRHD plain / warm / learned con2prim")
            # 10 steps per guess (the configuration's step count): longer runs smooth
            # the i.i.d. initial state and change the Newton workload being compared
            wl["srhd"] = bench_srhd(torch, pb, I, min(10, args.steps), args.mlp_epochs, args.mlp_pairs)
        if "ksweep" in want:
            log("K sweep: runtime per cell against the batch size, p in {3, 6, 16}, FV and FD4")
            wl["k_sweep"] = bench_ksweep(torch, pb, I)
        if "offload" in want:
            log("offload mode: total runtime against kernel time")
            wl["offload"] = bench_offload(pb, I)
        result["workloads"] = wl
    if args.save_tuning:
        pb.pb_autotune_cache_save(args.save_tuning)
        log(f"tuning cache written to {args.save_tuning}")
    if not args.no_cpu:
        log("timing the CPU oracle")
        result["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
        wl = result.get("workloads", {})
        for kind, key in (("linsym", "linsym58_fd4_rk4"), ("srhd", "srhd")):
            if key in wl:
                log(f"timing the CPU oracle on a {kind} sample")
                wl[key]["cpu_oracle"] = cpu_oracle_sample(kind, 6.0)
        if "linsym58_fd4_rk4" in wl:
            workers = args.cpu_workers or min(16, cpu_info()["usable_cpus"])
            log(f"timing the multi-process oracle ({workers} processes)")
            result["cpu_oracle_multiprocess"] = cpu_oracle_multiprocess(workers, 5.0)
    try:
        os.makedirs(os.path.dirname(os.path.abspath(args.detail_out)), exist_ok=True)
        with open(args.detail_out, "w") as fh:
            json.dump(result, fh, indent=1)
        result["detail_file"] = os.path.relpath(args.detail_out, ROOT)
    except OSError as e:
        log(f"could not write {args.detail_out}: {e}")
    print(json.dumps(compact(result)), flush=True)


if __name__ == "__main__":
    main()
