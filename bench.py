#!/usr/bin/env python3
"""Throughput of the DEM contact pipeline on one MI355X.

Workload: the at-scale plain case -- 1,000,000 polydisperse spheres
(r ~ U[0.8, 1.2] mm, E = 5e6 Pa, nu = 0.25, rho = 2500 kg/m^3, e = 0.9,
mu = 0.5) in a settled bed on an 80 x 80 mm footprint, periodic in x and y,
wall at z = 0, dt = 1e-6 s, skin 0.1 r_max.  A step is one full pass of the
hot path: kick-drift, device-side rebuild check (binning + neighbour list with
history carry when needed), forces, kick.

Prints one JSON line: particle-steps/s (value), contact-pairs/s, the roofline
of the dominant kernel (timed with HIP events inside this run) and the CPU
oracle timed on a bounded sample of the same workload.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
    python bench.py --profile-pass     # short run for rocprofv3 counter passes
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "particle-steps/s and contact-pairs/s (FP64) vs HBM roofline; batched & adjoint vs plain"
PMC_FILE = os.path.join(ROOT, "profiles", "step_settled_bed_1e6_traffic.txt")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1705_03850_amd", "csrc", f) for f in ("dem_kernels.hip", "dem_core.h")]

# Algorithmic bytes (FP64 = 8 B, int32 = 4 B) of the fused step kernel k_step: every array element it
# must touch, counted once (neighbour re-reads are the cache's business):
#   per particle: packed position+radius, velocity+mass, spin+type read and written (96 + 96),
#                 (1/m, 1/I) read (16), displacement read and written (24 + 24),
#                 row length (4) and history mask (8) read                       = 268 B
#   per listed slot: its neighbour index (4 B)
#   per directed contact: its tangential history read and written (48 B)
#   per wall contact: the wall history read and written (48 B)
STEP_PER_PARTICLE, STEP_PER_SLOT, STEP_PER_CONTACT, STEP_PER_WALL = 268, 4, 48, 48


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash():
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(p, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_traffic():
    """HBM bytes per force launch from the committed counter summary, or None
    when the kernel sources changed since the counters were taken."""
    if not os.path.exists(PMC_FILE):
        return None
    vals = {}
    with open(PMC_FILE) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(system, steps):
    """The oracle as it stands, single thread, on `steps` steps of the same bed."""
    sys.path.insert(0, os.path.join(ROOT, "oracle"))
    import oracle as O

    o = O.Oracle(system)
    o.forces(False)
    t0 = time.perf_counter()
    o.step(steps)
    dt = time.perf_counter() - t0
    return {"value": system.n * steps / dt, "unit": "particle-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"{steps} steps of the same {system.n}-sphere bed after one force evaluation, "
                      f"1 thread, {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--chunk", type=int, default=64)
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--max-blocks", type=int, default=0, help="grid cap of the fused step kernel (0 = resident capacity)")
    ap.add_argument("--lanes", type=int, default=4, help="threads per particle in the force pass (4, 8, 16)")
    ap.add_argument("--timing-steps", type=int, default=300)
    ap.add_argument("--cpu-steps", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--profile-pass", action="store_true",
                    help="a few non-graph steps plus a 256 MiB device copy (counter calibration), no JSON")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this build runs on one GPU only; run bench.py with --gpus 1"}), flush=True)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1705_03850_amd import dem
    from paper_1705_03850_amd.inputs import workloads as W

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}), flush=True)
        sys.exit(1)
    footprint = 80e-3 * (args.n / 1e6) ** 0.5
    log(f"generating the settled bed of {args.n} spheres")
    t0 = time.perf_counter()
    bed = W.settled_bed(seed=2, n=args.n, footprint=footprint)
    log(f"bed ready in {time.perf_counter() - t0:.1f} s (height {bed.x[:, 2].max() * 1e3:.0f} mm)")

    g = dem.DemSystem(bed, k_max=32, block=args.block, use_graph=not args.no_graph, chunk=args.chunk)
    g.set_launch(args.lanes, args.max_blocks)
    g.prime()
    torch.cuda.synchronize()

    if args.profile_pass:
        g.set_step_options(False, args.chunk)
        g.step(args.timing_steps)
        torch.cuda.synchronize()
        nbytes = 256 << 20
        src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"profile pass done: {args.timing_steps} steps, 3 copies of {nbytes} bytes")
        return

    log(f"warmup {args.warmup} steps")
    g.step(args.warmup)
    torch.cuda.synchronize()
    s0 = g.stats()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    log(f"timing {args.steps} steps")
    ev0.record(g.stream)
    t0 = time.perf_counter()
    g.step(args.steps)
    ev1.record(g.stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    s1 = g.stats()
    steps = args.steps
    n = bed.n
    seconds = wall
    directed = s1["contacts"] - s0["contacts"]
    wall_contacts = s1["wall_contacts"] - s0["wall_contacts"]
    unordered_per_step = directed / 2.0 / steps
    builds = s1["builds"] - s0["builds"]

    # per-kernel durations with HIP events on the library's stream
    log(f"per-kernel timing over {args.timing_steps} steps")
    g.set_timing(True)
    t_s0 = g.stats()
    g.step(args.timing_steps)
    kt = g.kernel_times()
    t_s1 = g.stats()
    g.set_timing(False)
    tsteps = args.timing_steps
    slots = float(g.stats()["slots"])
    contacts_step = (t_s1["contacts"] - t_s0["contacts"]) / tsteps
    walls_step = (t_s1["wall_contacts"] - t_s0["wall_contacts"]) / tsteps
    bytes_step = (n * STEP_PER_PARTICLE + slots * STEP_PER_SLOT + contacts_step * STEP_PER_CONTACT
                  + walls_step * STEP_PER_WALL)
    kernels = {}
    for name in ("pack", "step", "last", "rebuild"):
        ms, cnt = kt[name]
        if cnt:
            kernels[name] = {"avg_us": ms / cnt * 1e3, "launches": cnt}
    kernels["step"]["alg_bytes"] = bytes_step
    kernels["step"]["GBps"] = bytes_step / (kernels["step"]["avg_us"] * 1e-6) / 1e9
    achieved = kernels["step"]["GBps"]
    traffic = read_traffic()
    roofline = {"bound": "hbm", "kernel": "k_step (fused forces + kick + kick-drift)",
                "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "alg_bytes_per_launch": round(bytes_step), "avg_launch_us": round(kernels["step"]["avg_us"], 2)}

    cpu = None
    if not args.no_cpu_baseline:
        log(f"CPU oracle baseline: {args.cpu_steps} steps")
        cpu = cpu_baseline(bed, args.cpu_steps)

    out = {
        "metric": METRIC,
        "value": n * steps / seconds,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": seconds / steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"settled polydisperse bed, {n} spheres, r U[0.8,1.2] mm, 80x80 mm periodic "
                               f"footprint, wall z=0, dt 1e-6 s, skin 0.1 r_max",
                   "particles": n, "parallelism": "1 GPU", "graph": not args.no_graph, "chunk": args.chunk},
        "contact_pairs_per_s": unordered_per_step * steps / seconds,
        "listed_slots": slots,
        "contacts_per_step": unordered_per_step,
        "wall_contacts_per_step": wall_contacts / steps,
        "list_builds": builds,
        "gpu_event_ms": gpu_ms,
        "roofline": roofline,
        "kernels": kernels,
        "cpu_baseline": cpu,
        "kernel_source": kernel_source_hash(),
        "device": torch.cuda.get_device_name(0),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
