#!/usr/bin/env python3
"""Throughput of the DEM contact pipeline on one MI355X.

Workload: the at-scale plain case -- 1,000,000 polydisperse spheres
(r ~ U[0.8, 1.2] mm, E = 5e6 Pa, nu = 0.25, rho = 2500 kg/m^3, e = 0.9,
mu = 0.5) in a settled bed on an 80 x 80 mm footprint, periodic in x and y,
wall at z = 0, dt = 1e-6 s, skin 0.1 r_max.  A step is one full pass of the
hot path: kick-drift, device-side rebuild check (binning + neighbour list with
history carry when needed), forces, kick.

Prints one JSON line: particle-steps/s (value), contact-pairs/s, the roofline
of the dominant kernel (timed with HIP events inside this run), forced
rebuilds, the small-workload latency, the 64-system and two-level batches
against plain stepping, the adjoint of the 200-step chute rollout (checkpoints
every 20 steps, windows recomputed; the kept mode beside it) against the plain
rollout, and the CPU oracle timed on a bounded sample of the same workload.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-suites]
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
# ... and of the neighbour build (dem_neighbors):
#   per particle: position+radius and id read (36), its previous row's length, mask and frame read (16),
#                 new length, mask and id written (16), displacement cleared (24)   = 92 B
#   per listed slot: new neighbour index written (4), previous index and its id read (8) = 12 B
#   per directed contact carried: tangential history read and written (48 B)
#   per cell: its start offset (4 B)
NBR_PER_PARTICLE, NBR_PER_SLOT, NBR_PER_CONTACT, NBR_PER_CELL = 92, 12, 48, 4


_T0 = time.perf_counter()


def log(msg):
    print(f"[bench {time.perf_counter() - _T0:7.1f} s] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash():
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(p, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_traffic(key="hbm_bytes_per_launch"):
    """HBM bytes per launch from the committed counter summary (force kernel by
    default; "nbr_hbm_bytes_per_launch" for the neighbour build), or None when
    the kernel sources changed since the counters were taken."""
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
        return float(vals[key])
    except (KeyError, ValueError):
        return None


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(system, steps, par_steps):
    """The oracle as it stands, single thread, on `steps` steps of the same bed
    (value), and its all-cores leg (the OpenMP gather form of the same step,
    bit-identical results) on `par_steps` further steps, with the threads it used."""
    sys.path.insert(0, os.path.join(ROOT, "oracle"))
    import oracle as O

    o = O.Oracle(system)
    o.forces(False)
    t0 = time.perf_counter()
    o.step(steps)
    dt = time.perf_counter() - t0
    threads, dtp = o.step_parallel(par_steps)
    host = f"{cpu_model()}, {os.cpu_count()} logical CPUs visible"
    return {"value": system.n * steps / dt, "unit": "particle-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"{steps} steps of the same {system.n}-sphere bed after one force evaluation, "
                      f"1 thread, {dt:.1f} s; host {host}",
            "all_cores": {"value": system.n * par_steps / dtp, "unit": "particle-steps/s", "cores": threads,
                          "kind": "oracle (OpenMP gather form, bit-identical to the serial oracle)",
                          "sample": f"{par_steps} further steps of the same bed, {threads} threads, "
                                    f"{dtp:.1f} s of step loop"}}


def copy_bandwidth(nbytes=1 << 30, reps=10):
    """Achievable HBM bandwidth: a plain device-to-device copy of `nbytes`
    (read + write counted), median of `reps` copies timed with events."""
    import torch

    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    ms = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        e1.synchronize()
        ms.append(e0.elapsed_time(e1))
    del src, dst
    ms.sort()
    return 2 * nbytes / (ms[len(ms) // 2] * 1e-3) / 1e9


def timed_steps(g, steps, warm):
    import torch

    g.step(warm)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.step(steps)
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def chute_controllers(g, cpl):
    """PI parameters on the fine level's transition layer and P parameters on
    the coarse spheres inside the fine region, for the two-level chute."""
    from paper_1705_03850_amd import dem

    pp = dem.PIParams()
    pp.grid = dem.make_grid(*cpl["pi_grid"], sys=1)
    for a in range(3):
        pp.nrm[a] = cpl["normal"][a]
    pp.face, pp.kp, pp.ki, pp.fade = cpl["face"], cpl["kp"], cpl["ki"], cpl["fade"]
    pp.interval = cpl["interval_steps"] * g.systems[1].dt
    qp = dem.PParams()
    qp.grid, qp.kp, qp.mass_flow = dem.make_grid(*cpl["p_grid"], sys=0), cpl["kp_coarse"], 1
    return pp, qp


def coupled_grouped_run(g, cpl, steps, group):
    """The same coupled chute stepped by dem_step_coupled: `group` intervals
    (coupling and steps, one captured graph per interval) per synchronisation.
    The first interval (graph capture) is left out of the timing."""
    import torch

    k = cpl["interval_steps"]
    pp, qp = chute_controllers(g, cpl)
    plan = g.coupling_plan(pp, 0, qp, 1, k, group=group)
    g.step_coupled(1, plan)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.step_coupled(steps // k, plan)
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def coupled_run(g, cpl, steps):
    """The two-level chute coupled (Sec. 2.3): every `interval_steps` steps the
    cell fields of both levels on the transition layer and on the grid inside
    the fine region, the PI controller on the fine spheres of the 10 mm shell and
    the P controller (mass flow) on the coarse spheres, then the steps.  The
    interval's coupling calls are captured once in a graph and replayed (they
    are asynchronous; the P controller reads no stress).  Returns (wall
    seconds, host seconds spent issuing the coupling)."""
    import torch

    from paper_1705_03850_amd import dem

    k = cpl["interval_steps"]
    pp, qp = chute_controllers(g, cpl)
    pi_f, pi_c = dem.make_grid(*cpl["pi_grid"], sys=1), dem.make_grid(*cpl["pi_grid"], sys=0)
    p_f, p_c = dem.make_grid(*cpl["p_grid"], sys=1), dem.make_grid(*cpl["p_grid"], sys=0)
    n_pi = pi_f.n[0] * pi_f.n[1] * pi_f.n[2]
    integral = torch.zeros(n_pi, dtype=torch.float64, device=g.device)
    u = torch.empty(n_pi, dtype=torch.float64, device=g.device)
    n_p = p_f.n[0] * p_f.n[1] * p_f.n[2]
    buf = [torch.empty((dem.NFIELDS, n), dtype=torch.float64, device=g.device) for n in (n_pi, n_pi, n_p, n_p)]
    t_ctl = 0.0
    # external forces switched on (all zero) before the capture, so that the
    # graph holds only the coupling
    g.set_external_force(torch.zeros((3, g.n), dtype=torch.float64, device=g.device))
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=g.stream):
        g.pi_control(pp, g.cell_fields(pi_f, out=buf[0]), g.cell_fields(pi_c, out=buf[1]), integral, u)
        g.p_control(qp, g.cell_fields(p_f, stress=False, out=buf[2]), g.cell_fields(p_c, stress=False, out=buf[3]))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    with torch.cuda.stream(g.stream):
        for _ in range(steps // k):
            tc = time.perf_counter()
            graph.replay()
            t_ctl += time.perf_counter() - tc
            g.step(k)
    torch.cuda.synchronize()
    return time.perf_counter() - t0, t_ctl


def exchange_events(two, cpl, chunk, events=12, ncand=4096, interval=15):
    """Insertion and deletion events on the fine level of the two-level chute
    (Sec. 2.3): every `interval` steps one dem_exchange call on the fine system
    (5e5 spheres, 65,536 free slots) with `ncand` candidates in a 5 mm slab
    across its top face z_f over 4 x 2 boundary cells (seeded inflow fields,
    budgets of up to 60 spheres per cell; spheres above z_f removed, among them
    those the previous event inserted above the face).  Wall time of each
    synchronising call (removal, SSI, insertion, the system's list rebuild and
    force pass), of a call that changes nothing, and the plain forced rebuild
    of the context for scale."""
    import numpy as np
    import torch

    from paper_1705_03850_amd import dem
    from paper_1705_03850_amd.inputs import workloads as W

    fine = two[1]
    zf = -cpl["face"]
    g = dem.DemSystem(two, use_graph=True, chunk=chunk, capacity=[None, fine.n + 65536])
    g.prime()
    g.step(64)
    wall, ins, rem = [], [], []
    for k in range(events):
        ev = W.exchange_inputs(fine, zf + 4e-3, ncand, seed=100 + k, cells=(4, 2), budget_spheres=60.0,
                               depth=5e-3)
        budget = torch.from_numpy(ev["budget"]).to(g.device)
        p = dem.ExchangeParams()
        for a in range(3):
            p.nrm[a] = ev["nrm"][a]
        p.face, p.slab, p.interval, p.ncell = -zf, ev["slab"], interval * fine.dt, ev["ncell"]
        fields = torch.from_numpy(ev["fields"]).to(g.device)
        cand = [torch.from_numpy(np.ascontiguousarray(a)).to(g.device)
                for a in (ev["cand_x"], ev["cand_r"], ev["cand_type"], ev["cand_cell"])]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, i, r = g.exchange(1, p, fields, budget, *cand)
        wall.append(time.perf_counter() - t0)
        ins.append(i)
        rem.append(r)
        g.step(interval)
    # an event that changes nothing (no candidate, nothing to remove): the call's floor
    p.face = -1.0
    empty = torch.zeros(8, dtype=torch.float64, device=g.device)
    noop = []
    for _ in range(5):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.exchange(1, p, fields, empty)
        noop.append(time.perf_counter() - t0)
    torch.cuda.synchronize()
    t_steps = time.perf_counter()
    g.step(64 * 4)
    torch.cuda.synchronize()
    t_steps = (time.perf_counter() - t_steps) / 256
    # the plain forced rebuild of the whole context, for scale
    reb = []
    for _ in range(5):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.build_list()
        g.forces(False)
        torch.cuda.synchronize()
        reb.append(time.perf_counter() - t0)
    w = sorted(wall[2:])
    return {"events": events, "candidates": ncand, "interval_steps": interval,
            "event_ms_median": 1e3 * w[len(w) // 2], "event_ms_max": 1e3 * max(wall[2:]),
            "noop_event_ms_median": 1e3 * sorted(noop)[2],
            "inserted_mean": float(np.mean(ins)), "removed_mean": float(np.mean(rem)),
            "live_fine_after": g.live(1), "step_ms": 1e3 * t_steps,
            "rebuild_and_forces_ms_median": 1e3 * sorted(reb)[2],
            "event_vs_interval_steps": w[len(w) // 2] / (interval * t_steps)}


def batch_suite(args, emit=True):
    """Batched against plain on the same GPU (one JSON line).

    64 systems (N log-uniform in [5e3, 2e5], alpha in {1, 2, 4, 8}, dt = alpha 1e-6 s):
      batched    -- all systems in one context: one launch per step for all of them, graph replay;
      sequential -- the same systems, each in its own context with the library's default
                    launch shape and skin (plain dem_step as a user runs it), one after another;
      equal N    -- one plain bed with the same total particle count (defaults too).
    Multi-rate: the same batch with every system stepping its own dt once every alpha substeps
    (all levels over the same simulated time), against the single-rate batch.
    Two-level chute (2e5 spheres alpha = 4 + 5e5 spheres alpha = 1): one 2-system batch against the two
    systems one after another, and coupled (fields and controllers every 15 steps).  Launch shape, skin
    and cell come from the autotuner."""
    import torch

    from paper_1705_03850_amd import autotune, dem
    from paper_1705_03850_amd.inputs import workloads as W

    steps = args.steps if args.steps != 10000 else 2000
    log("generating 64 batch systems")
    systems = W.batch_systems()
    ntot = sum(s.n for s in systems)
    log(f"{len(systems)} systems, {ntot} particles; autotuning")
    if args.no_autotune:
        choice = {"skin_factor": 0.1, "cell_factor": 1.0, "block": 256, "lanes": 4}
    else:
        choice = autotune.autotune(systems, steps=128, long_steps=1024, log=log)
    kw = autotune.apply(systems, choice)
    g = dem.DemSystem(systems, use_graph=True, chunk=args.chunk, **kw)
    g.prime()
    t_batch = timed_steps(g, steps, 64)
    builds_batch = g.stats()["builds"]
    del g
    torch.cuda.empty_cache()
    # multi-rate: every system steps with its own dt = alpha 1e-6 s once every alpha
    # substeps, so all levels advance over the same simulated time (steps * 1e-6 s);
    # against the single-rate batch above, which steps every system every substep
    log("multi-rate batch")
    gm = dem.DemSystem(systems, use_graph=True, chunk=args.chunk, **kw)
    gm.set_multirate(True)
    gm.prime()
    nsub = steps - steps % 8
    t_mr = timed_steps(gm, nsub, 64)
    work_mr = sum(s.n * (nsub // int(round(s.dt / 1e-6))) for s in systems)
    builds_mr = gm.stats()["builds"]
    del gm
    torch.cuda.empty_cache()
    log("sequential plain contexts")
    t_seq = 0.0
    for s in systems:
        gk = dem.DemSystem(s, use_graph=True, chunk=args.chunk)
        gk.prime()
        t_seq += timed_steps(gk, steps, 64)
        del gk
    torch.cuda.empty_cache()
    log("equal-N plain system")
    big = W.tiled_bed(ntot)
    gb = dem.DemSystem(big, use_graph=True, chunk=args.chunk)
    gb.prime()
    t_big = timed_steps(gb, steps, 64)
    del gb
    torch.cuda.empty_cache()
    log("two-level chute")
    two = W.chute_two_level()
    n2 = sum(s.n for s in two)
    g2 = dem.DemSystem(two, use_graph=True, chunk=args.chunk)
    g2.prime()
    steps2 = 5000 if args.steps == 10000 else args.steps
    t_two = timed_steps(g2, steps2, 64)
    builds_two = g2.stats()["builds"]
    del g2
    t_two_seq = 0.0
    for s in two:
        gk = dem.DemSystem(s, use_graph=True, chunk=args.chunk)
        gk.prime()
        t_two_seq += timed_steps(gk, steps2, 64)
        del gk
    log("two-level chute, coupled")
    cpl = W.chute_coupling(*two)
    g2c = dem.DemSystem(two, use_graph=True, chunk=8)
    g2c.prime()
    steps_c = steps2 - steps2 % cpl["interval_steps"]
    t_cpl, t_ctl = coupled_run(g2c, cpl, steps_c)
    del g2c
    group = 8
    g2g = dem.DemSystem(two, use_graph=True, chunk=8)
    g2g.prime()
    t_grp = coupled_grouped_run(g2g, cpl, steps_c, group)
    del g2g
    log("two-level chute, insertion events")
    exch = exchange_events(two, cpl, args.chunk)
    out = {
        "suite": "batch", "unit": "particle-steps/s", "dtype": "f64", "data": "synthetic",
        "batch64": {"systems": len(systems), "particles": ntot, "steps": steps,
                    "batched": ntot * steps / t_batch, "sequential_plain": ntot * steps / t_seq,
                    "equal_n_plain": big.n * steps / t_big, "equal_n_particles": big.n,
                    "batched_vs_sequential": t_seq / t_batch,
                    "batched_vs_equal_n": (ntot / t_batch) / (big.n / t_big),
                    "list_builds_batched": builds_batch, "autotune": {k: choice[k] for k in
                                                                       ("lanes", "block", "skin_factor", "cell_factor")},
                    "multirate": {"substeps": nsub, "particle_steps": work_mr,
                                  "particle_steps_per_s": work_mr / t_mr,
                                  "work_fraction": work_mr / (ntot * nsub),
                                  "simulated_time_speedup_vs_single_rate": (t_batch / steps) / (t_mr / nsub),
                                  "list_builds": builds_mr}},
        "two_level_chute": {"particles": n2, "steps": steps2, "batched": n2 * steps2 / t_two,
                            "sequential_plain": n2 * steps2 / t_two_seq, "batched_vs_sequential": t_two_seq / t_two,
                            "list_builds_batched": builds_two,
                            "coupled": {"steps": steps_c, "interval_steps": cpl["interval_steps"],
                                        "particle_steps_per_s": n2 * steps_c / t_cpl,
                                        "coupled_vs_batched": (n2 * steps_c / t_cpl) / (n2 * steps2 / t_two),
                                        "coupling_issue_host_s": t_ctl,
                                        "grouped": {"group": group, "particle_steps_per_s": n2 * steps_c / t_grp,
                                                    "vs_batched": (n2 * steps_c / t_grp) / (n2 * steps2 / t_two)},
                                        "transition_cells": list(cpl["pi_grid"][2]),
                                        "fine_region_cells": list(cpl["p_grid"][2])},
                            "exchange": exch},
        "device": torch.cuda.get_device_name(0),
    }
    if emit:
        print(json.dumps(out), flush=True)
    return out


def silo_run(label, r, dt, fill, settle_s, discharge_s, sample_s, chunk):
    """One silo (Sec. 3, the paper's shape and material table): spheres of
    radius r on a lattice filling the silo to `fill` of its height, settled
    with the orifice closed for settle_s, then discharged for discharge_s.
    Every sample_s one dem_exchange call removes the spheres more than 1 cm
    below the orifice; their mass over sample_s is the discharge rate."""
    import math

    import numpy as np
    import torch

    from paper_1705_03850_amd import dem
    from paper_1705_03850_amd.inputs import workloads as W

    s = W.silo_system(scale=1.0, r=r, fill=fill, dt=dt, mat=W.MAT_SILO, mu_wall=W.MU_WALL_SILO)
    log(f"silo {label}: {s.n} spheres of d = {2e3 * r:.1f} mm")
    g = dem.DemSystem(s, surfaces=s.meta["surfaces"], capacity=s.n, use_graph=True, chunk=chunk)
    g.prime()
    m = 4.0 / 3.0 * math.pi * W.MAT_SILO.rho * r ** 3
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    nset = int(round(settle_s / dt))
    g.step(nset)
    torch.cuda.synchronize()
    t_settle = time.perf_counter() - t0
    g.set_surfaces(0, W.silo_surfaces(1.0, open_orifice=True, mu_wall=W.MU_WALL_SILO))
    p = dem.ExchangeParams()
    p.nrm[2] = -1.0
    p.face = -1e9                       # no boundary face: removal at the outlet only
    p.slab, p.interval, p.ncell = 1.0, 0.0, 1
    p.out_nrm[2] = 1.0
    p.out_face = -0.01                  # 1 cm below the orifice
    fields = torch.zeros((16, 1), dtype=torch.float64, device=g.device)
    budget = torch.zeros(1, dtype=torch.float64, device=g.device)
    per = int(round(sample_s / dt))
    rates, work = [], 0
    t1 = time.perf_counter()
    for k in range(int(round(discharge_s / sample_s))):
        live = g.live(0)
        g.step(per)
        work += live * per
        _, _, rem = g.exchange(0, p, fields, budget)
        rates.append(rem * m / sample_s)
        if (k + 1) % 10 == 0:
            log(f"silo {label}: {(k + 1) * sample_s:.2f} s discharged, {g.live(0)} spheres left")
    torch.cuda.synchronize()
    t_dis = time.perf_counter() - t1
    st = g.stats()
    rates = np.array(rates)
    steady = rates[int(0.2 / sample_s):] if len(rates) > int(0.3 / sample_s) else rates
    out = {"spheres": s.n, "d_mm": 2e3 * r, "dt": dt, "settle_steps": nset,
           "discharge_steps": per * len(rates), "sample_s": sample_s,
           "rate_kg_s_mean": float(steady.mean()), "rate_kg_s_std": float(steady.std()),
           "rate_window_s": [0.2, discharge_s], "remaining": g.live(0),
           "discharged_kg": float(rates.sum() * sample_s),
           "settle_wall_s": t_settle, "discharge_wall_s": t_dis,
           "particle_steps_per_s_discharge": work / t_dis,
           "particle_steps_per_s_settle": s.n * nset / t_settle,
           "list_builds": st["builds"], "rates_kg_s": [round(float(q), 4) for q in rates]}
    log(f"silo {label}: {out['rate_kg_s_mean']:.3f} +- {out['rate_kg_s_std']:.3f} kg/s, "
        f"settle {t_settle:.1f} s, discharge {t_dis:.1f} s")
    return out


def mlcg_silo_run(settle_s, discharge_s, chunk, interval=15, exchange_every=10, sample_s=0.01, multirate=False,
                  stepper="coupled", group=5):
    """The multi-level silo (Sec. 2.3 on the silo of Sec. 3, Table 2's MLCG
    rows): the coarse level (alpha = 2, d = 5.6 mm) fills the silo as in the
    coarse-grain run; the fine level (d = 2.8 mm) fills its lower quarter
    (z < 10 cm), the fine region.  On a grid of 2 cm cubes over the region
    (8 x 8 in plan, five layers) every `interval` steps: the cell fields of
    both levels; the PI controller on the fine spheres of the top layer (the
    transition layer, boundary face z = 10 cm); the P controller in mass-flow
    mode on the coarse spheres of the four layers below.  Every
    `exchange_every` intervals an insertion event on the fine level: the
    budget of each 2 x 2 cm boundary cell grows by the coarse inflow through
    the face (the coarse fields of the 2 cm slab above it, averaged over the
    couplings since the last event, so that the inserted spheres move with
    the Favre-averaged velocity of the period), candidates are
    drawn in the top centimetre of the region and fine spheres above the face
    are removed.  Both levels discharge through the orifice; each level's
    rate is its mass removed 1 cm below the orifice per 10 ms.  With
    `multirate` the coarse level steps at 2 dt in one multi-rate schedule
    (Sec. 3: the time step may grow with the coarse-grain factor) and
    `interval` counts fine substeps (even, so that both levels meet).
    stepper "coupled": dem_step_coupled runs `group` intervals (coupling and
    steps) per synchronisation; "calls": per interval the coupling calls
    replayed as one graph, then dem_step."""
    import math

    import numpy as np
    import torch

    from paper_1705_03850_amd import dem
    from paper_1705_03850_amd.inputs import workloads as W

    dt = 1e-6
    mat, muw = W.MAT_SILO, W.MU_WALL_SILO
    if multirate and interval % 2:
        raise ValueError("a multi-rate coupling interval must be even")
    coarse = W.silo_system(scale=1.0, r=2.8e-3, fill=0.53, dt=2 * dt if multirate else dt, mat=mat, mu_wall=muw,
                           seed=9)
    coarse.alpha = 2.0
    fine = W.silo_system(scale=1.0, r=1.4e-3, fill=0.25, dt=dt, mat=mat, mu_wall=muw, seed=10)
    log(f"multi-level silo: {coarse.n} coarse spheres (d = 5.6 mm), {fine.n} fine (d = 2.8 mm) below z = 10 cm")
    closed = W.silo_surfaces(1.0, mu_wall=muw)
    g = dem.DemSystem([coarse, fine], surfaces=[closed, closed], capacity=[coarse.n, fine.n + 40_000],
                      use_graph=True, chunk=chunk)
    if multirate:
        g.set_multirate(True)
    g.prime()
    zf, h = 0.10, 0.02
    pi_grid = dem.make_grid((-0.08, -0.08, zf - h), (h, h, h), (8, 8, 1), sys=1)
    pi_grid_c = dem.make_grid((-0.08, -0.08, zf - h), (h, h, h), (8, 8, 1), sys=0)
    p_grid_f = dem.make_grid((-0.08, -0.08, 0.0), (h, h, h), (8, 8, 4), sys=1)
    p_grid_c = dem.make_grid((-0.08, -0.08, 0.0), (h, h, h), (8, 8, 4), sys=0)
    in_grid_c = dem.make_grid((-0.08, -0.08, zf), (h, h, h), (8, 8, 1), sys=0)
    pp = dem.PIParams()
    pp.grid = pi_grid
    pp.nrm[2] = -1.0
    pp.face, pp.kp, pp.ki, pp.fade, pp.interval = -zf, 1.0, 200.0, 1.5, interval * dt
    qp = dem.PParams()
    qp.grid, qp.kp, qp.mass_flow = p_grid_c, 2000.0, 1
    integral = torch.zeros(64, dtype=torch.float64, device=g.device)
    ex = dem.ExchangeParams()
    ex.nrm[2] = -1.0
    ex.face, ex.slab, ex.interval, ex.ncell = -zf, h, exchange_every * interval * dt, 64
    budget = torch.zeros(64, dtype=torch.float64, device=g.device)
    out = dem.ExchangeParams()
    out.nrm[2] = -1.0
    out.face, out.slab, out.interval, out.ncell = -1e9, 1.0, 0.0, 1
    out.out_nrm[2] = 1.0
    out.out_face = -0.01
    zero_f = torch.zeros((16, 1), dtype=torch.float64, device=g.device)
    zero_b = torch.zeros(1, dtype=torch.float64, device=g.device)
    rng = np.random.default_rng(12)
    rf = 1.4e-3
    mf = 4.0 / 3.0 * math.pi * mat.rho * rf ** 3
    mc = 4.0 / 3.0 * math.pi * mat.rho * (2.0 * rf) ** 3

    def candidates(per_cell=12, depth=0.01):
        cell = np.repeat(np.arange(64), per_cell)
        k = cell.size
        x = -0.08 + (cell % 8 + rng.uniform(0.0, 1.0, k)) * h
        y = -0.08 + (cell // 8 + rng.uniform(0.0, 1.0, k)) * h
        z = zf - depth * rng.uniform(0.0, 1.0, k)
        inside = np.hypot(x, y) <= W.silo_radius_at(z) - 1.05 * rf / (0.2 / math.hypot(0.115, 0.2))
        c = [np.column_stack([x, y, z])[inside], np.full(int(inside.sum()), rf), np.zeros(int(inside.sum()), np.int32),
             cell[inside].astype(np.int32)]
        return [torch.from_numpy(np.ascontiguousarray(a)).to(g.device) for a in c]

    # the loop runs on the library's stream with its buffers allocated once;
    # the P controller and the insertion budget read no stress
    buf = {k: torch.zeros((dem.NFIELDS, 64 * n), dtype=torch.float64, device=g.device)
           for k, n in (("pi", 1), ("pi_c", 1), ("p", 4), ("p_c", 4), ("in_c", 1))}
    u = torch.empty(64, dtype=torch.float64, device=g.device)
    in_sum = torch.zeros((dem.NFIELDS, 64), dtype=torch.float64, device=g.device)

    def interval_coupling():
        g.pi_control(pp, g.cell_fields(pi_grid, out=buf["pi"]), g.cell_fields(pi_grid_c, out=buf["pi_c"]),
                     integral, u)
        g.p_control(qp, g.cell_fields(p_grid_f, stress=False, out=buf["p"]),
                    g.cell_fields(p_grid_c, stress=False, out=buf["p_c"]))
        # the coarse level on the boundary cells, summed at every coupling
        # between insertion events: their mean is the Favre average over the
        # period (momentum over mass) and the mean inflow
        in_sum.add_(g.cell_fields(in_grid_c, stress=False, out=buf["in_c"]))

    inserted = removed_top = 0
    t_cpl = t_ex = 0.0
    # the interval's coupling calls captured once in a graph that every
    # interval replays: the calls read everything that changes (positions,
    # binning, live counts, list buffer) from the device; external forces
    # switched on (all zero) first, so that the graph holds only the coupling
    g.set_external_force(torch.zeros((3, g.n), dtype=torch.float64, device=g.device))
    torch.cuda.synchronize()
    if stepper == "calls":
        cpl_graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(cpl_graph, stream=g.stream):
            interval_coupling()

    plan = g.coupling_plan(pp, 0, qp, 1, interval, group=group, integral=integral, sum_grid=in_grid_c)

    def insertion_event():
        nonlocal inserted, removed_top, t_ex
        te = time.perf_counter()
        acc = plan.buffers["sum"] if stepper == "coupled" else in_sum
        fields = acc / exchange_every
        acc.zero_()
        _, i, r = g.exchange(1, ex, fields, budget, *candidates())
        inserted += i
        removed_top += r
        t_ex += time.perf_counter() - te

    def run_coupled(seconds, sampling):
        # blocks of whole insertion periods; a rate sample at the first block
        # end at least sample_s after the last one, over the time elapsed
        nonlocal t_cpl
        rates_f, rates_c = [], []
        per_sample = int(round(sample_s / (interval * dt)))
        n_int = int(round(seconds / (interval * dt)))
        k = last = 0
        next_log = 5 * per_sample
        while k < n_int:
            nb = min(exchange_every - k % exchange_every, n_int - k)
            tc = time.perf_counter()
            g.step_coupled(nb, plan)
            t_cpl += time.perf_counter() - tc
            k += nb
            if k % exchange_every == 0:
                insertion_event()
            if sampling and k - last >= per_sample:
                _, _, rf_ = g.exchange(1, out, zero_f, zero_b)
                _, _, rc_ = g.exchange(0, out, zero_f, zero_b)
                rates_f.append(rf_ * mf / ((k - last) * interval * dt))
                rates_c.append(rc_ * mc / ((k - last) * interval * dt))
                last = k
            if k >= next_log:
                next_log += 5 * per_sample
                log(f"multi-level silo: {k * interval * dt:.2f} s of {seconds:.2f} s"
                    f"{' (discharge)' if sampling else ' (settling)'}; fine {g.live(1)}, coarse {g.live(0)}, "
                    f"inserted {inserted}")
        return np.array(rates_f), np.array(rates_c)

    def run(seconds, sampling):
        if stepper == "coupled":
            return run_coupled(seconds, sampling)
        nonlocal t_cpl
        rates_f, rates_c = [], []
        per_sample = int(round(sample_s / (interval * dt)))
        n_int = int(round(seconds / (interval * dt)))
        for k in range(n_int):
            tc = time.perf_counter()
            cpl_graph.replay()
            t_cpl += time.perf_counter() - tc
            g.step(interval)
            if (k + 1) % exchange_every == 0:
                insertion_event()
            if sampling and (k + 1) % per_sample == 0:
                _, _, rf_ = g.exchange(1, out, zero_f, zero_b)
                _, _, rc_ = g.exchange(0, out, zero_f, zero_b)
                rates_f.append(rf_ * mf / (per_sample * interval * dt))
                rates_c.append(rc_ * mc / (per_sample * interval * dt))
            if (k + 1) % (5 * per_sample) == 0:
                log(f"multi-level silo: {(k + 1) * interval * dt:.2f} s of {seconds:.2f} s"
                    f"{' (discharge)' if sampling else ' (settling)'}; fine {g.live(1)}, coarse {g.live(0)}, "
                    f"inserted {inserted}")
        return np.array(rates_f), np.array(rates_c)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    with torch.cuda.stream(g.stream):
        run(settle_s, False)
    torch.cuda.synchronize()
    t_settle = time.perf_counter() - t0
    opened = W.silo_surfaces(1.0, open_orifice=True, mu_wall=muw)
    g.set_surfaces(0, opened)
    g.set_surfaces(1, opened)
    t1 = time.perf_counter()
    with torch.cuda.stream(g.stream):
        rates_f, rates_c = run(discharge_s, True)
    torch.cuda.synchronize()
    t_dis = time.perf_counter() - t1
    skip = int(0.2 / sample_s)
    sf, sc = rates_f[skip:], rates_c[skip:]
    res = {"coarse_spheres": coarse.n, "fine_spheres_start": fine.n, "fine_live_end": g.live(1),
           "coarse_live_end": g.live(0), "interval_steps": interval, "exchange_every_intervals": exchange_every,
           "inserted": inserted, "removed_above_face": removed_top,
           "rate_fine_kg_s_mean": float(sf.mean()), "rate_fine_kg_s_std": float(sf.std()),
           "rate_coarse_kg_s_mean": float(sc.mean()), "rate_coarse_kg_s_std": float(sc.std()),
           "settle_wall_s": t_settle, "discharge_wall_s": t_dis, "stepper": stepper,
           "group": group if stepper == "coupled" else 1,
           "coupled_steps_wall_s" if stepper == "coupled" else "coupling_wall_s": t_cpl, "exchange_wall_s": t_ex,
           "rates_fine_kg_s": [round(float(q), 4) for q in rates_f],
           "rates_coarse_kg_s": [round(float(q), 4) for q in rates_c]}
    log(f"multi-level silo: fine {res['rate_fine_kg_s_mean']:.3f} +- {res['rate_fine_kg_s_std']:.3f} kg/s, coarse "
        f"{res['rate_coarse_kg_s_mean']:.3f} +- {res['rate_coarse_kg_s_std']:.3f} kg/s, settle {t_settle:.1f} s, "
        f"discharge {t_dis:.1f} s")
    return res


def silo_suite(args):
    """The paper's silo discharge (Sec. 3, Table 2): the reference (d = 2.8 mm)
    and the coarse-grain model (alpha = 2, d = 5.6 mm, same dt), each filled
    from a lattice to about 187,504 reference spheres' worth, settled 0.2 s,
    discharged 1.0 s; discharge rates sampled at 100 Hz 1 cm below the orifice.
    The paper reports 0.400 and 0.315 kg/s (its fill is poured, ours starts
    from a lattice).  With --silo-mlcg also the multi-level silo (0.390 and
    0.391 kg/s in the paper)."""
    import torch

    settle = args.silo_settle
    line = {"suite": "silo", "metric": "silo discharge rate (kg/s) and particle-steps/s", "dtype": "f64",
            "data": "synthetic",
            "paper": {"reference": 0.400, "cg_alpha2": 0.315, "cg_over_reference": 0.315 / 0.400,
                      "mlcg_fine": 0.390, "mlcg_coarse": 0.391},
            "device": torch.cuda.get_device_name(0)}
    if not (args.silo_mlcg_only or args.silo_mlcg_multirate_only):
        ref = silo_run("reference", 1.4e-3, 1e-6, 0.525, settle, args.silo_discharge, 0.01, args.chunk)
        cg = silo_run("CG alpha=2", 2.8e-3, 1e-6, 0.53, settle, args.silo_discharge, 0.01, args.chunk)
        line.update({"reference": ref, "cg_alpha2": cg,
                     "cg_over_reference": cg["rate_kg_s_mean"] / ref["rate_kg_s_mean"]})
    stepper = "calls" if args.silo_mlcg_calls else "coupled"
    if args.silo_mlcg or args.silo_mlcg_only:
        line["mlcg"] = mlcg_silo_run(settle, args.silo_discharge, 16, stepper=stepper)
    if args.silo_mlcg_multirate or args.silo_mlcg_multirate_only:
        line["mlcg_multirate"] = dict(mlcg_silo_run(settle, args.silo_discharge, 16, interval=16, multirate=True,
                                                    stepper=stepper), coarse_dt=2e-6, fine_dt=1e-6)
    print(json.dumps(line), flush=True)


def adjoint_suite(args, emit=True):
    """Adjoint against plain on the chute calibration workload (one JSON line).

    50,000 spheres, two types 50/50 (r ~ U[0.9, 1.1] mm), 30-degree periodic
    chute, 200 steps, checkpoints every 20 steps.  Loss: mean squared difference
    of the 20-bin mass-flux profile from the oracle's profile at a perturbed
    parameter set (tests/golden/chute_flux_target.json).
      plain    -- dem_step over the 200 steps (graph replay), after one force evaluation;
      adjoint  -- DemRollout forward (windows + checkpoints) and loss.backward()
                  (recompute of every window + reverse sweep + parameter gradient);
                  with --keep the forward stores every step's inputs and the
                  backward recomputes nothing.
    Reports (forward + backward) / plain, the parts, and the device memory."""
    import numpy as np
    import torch

    from paper_1705_03850_amd import dem
    from paper_1705_03850_amd import rollout as R
    from paper_1705_03850_amd.inputs import workloads as W

    with open(os.path.join(ROOT, "tests", "golden", "chute_flux_target.json")) as fh:
        tgt = json.load(fh)
    steps, window, reps = tgt["steps"], args.window, 3
    log("generating the 50,000-sphere chute")
    s = W.chute_adjoint()
    H0, Lx, Ly = s.meta["H0"], s.hi[0] - s.lo[0], s.hi[1] - s.lo[1]
    target = torch.tensor(tgt["target_flux"], dtype=torch.float64, device="cuda")
    t_plain = []
    g = dem.DemSystem(s, use_graph=True, chunk=20)
    for _ in range(reps + 1):
        g.load_state()
        g.reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.prime()
        g.step(steps)
        torch.cuda.synchronize()
        t_plain.append(time.perf_counter() - t0)
    plain_builds = g.stats()["builds"]
    del g
    torch.cuda.empty_cache()
    torch.cuda.reset_peak_memory_stats()
    g = dem.DemSystem(s)
    # checkpoints sized for the longest neighbour row (with a margin for the
    # rows of later builds) and for the windows the rollout needs
    kslots, max_windows = args.kslots, args.max_windows
    if kslots < 0:
        g.build_list()
        lo, _ = g.export_neighbors()
        kslots = min(int(np.bincount(lo).max()) + 4, 32)
    if max_windows < 0:
        max_windows = -(-steps // window) + 3
    adj = g.adjoint(steps, window=window, keep=args.keep, kslots=kslots, max_windows=max_windows)
    if args.adj_lanes:
        adj.set_lanes(args.adj_lanes)
    t_fwd, t_bwd = [], []
    for _ in range(reps + 1):
        g.load_state()
        g.reset()
        theta = R.theta_of(s.materials).requires_grad_(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, v, w = R.rollout(theta, adj)
        flux = R.mass_flux_profile(x, v, R.masses(g), H0, Lx, Ly)
        loss = ((flux - target) ** 2).mean()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        loss.backward()
        torch.cuda.synchronize()
        t_bwd.append(time.perf_counter() - t1)
        t_fwd.append(t1 - t0)
    info = adj.info()
    tp, tf, tb = (float(np.median(t[1:])) for t in (t_plain, t_fwd, t_bwd))
    out = {
        "suite": "adjoint", "workload": "chute_adjoint(seed=5, n=50000), 200 steps, flux loss in 20 bins",
        "n": s.n, "steps": steps, "window": window, "keep": bool(args.keep), "lanes": args.adj_lanes or "default",
        "kslots": kslots or 32, "max_windows": info["max_windows"],
        "dtype": "f64", "data": "synthetic",
        "plain_forward_s": tp, "adjoint_forward_s": tf, "backward_s": tb,
        "adjoint_vs_plain": (tf + tb) / tp, "backward_vs_plain": tb / tp,
        "plain_particle_steps_per_s": s.n * steps / tp,
        "windows": info["windows"], "rebuilds": info["rebuilds"], "plain_list_builds": plain_builds,
        "adjoint_workspace_bytes": info["bytes"], "context_workspace_bytes": g.ws_bytes,
        "peak_torch_bytes": torch.cuda.max_memory_allocated(),
        "loss": float(loss.detach().cpu()), "grad": {"E": theta.grad[0].tolist(), "e": theta.grad[1].tolist(),
                                                     "mu": theta.grad[2].tolist()},
        "device": torch.cuda.get_device_name(0),
    }
    if emit:
        print(json.dumps(out), flush=True)
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--chunk", type=int, default=64)
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--max-blocks", type=int, default=0, help="grid cap of the fused step kernel (0 = resident capacity)")
    ap.add_argument("--lanes", type=int, default=0,
                    help="threads per particle in the force pass (4, 8, 16; 0: the library default)")
    ap.add_argument("--timing-steps", type=int, default=300)
    ap.add_argument("--cpu-steps", type=int, default=4)
    ap.add_argument("--cpu-par-steps", type=int, default=8, help="steps of the oracle's all-cores leg")
    ap.add_argument("--rebuilds", type=int, default=10, help="forced rebuilds (dem_bin + dem_neighbors) after the timing")
    ap.add_argument("--small-steps", type=int, default=1000, help="steps of the 2000-sphere workload timed for latency")
    ap.add_argument("--no-suites", action="store_true", help="leave the batch and adjoint comparisons out of the line")
    ap.add_argument("--rebuild-every", type=int, default=50, help="steps between forced rebuilds")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--window", type=int, default=20, help="adjoint suite: steps per checkpoint window")
    ap.add_argument("--keep", action="store_true", help="adjoint suite: store every step's inputs (no recompute)")
    ap.add_argument("--kslots", type=int, default=-1,
                    help="adjoint suite: history slots per particle in the checkpoints (-1: longest row + 4, 0: k_max)")
    ap.add_argument("--max-windows", type=int, default=-1,
                    help="adjoint suite: checkpoint windows (-1: ceil(steps / window) + 3, 0: the library's default)")
    ap.add_argument("--adj-lanes", type=int, default=0, help="adjoint suite: threads per particle (0: library default)")
    ap.add_argument("--silo-settle", type=float, default=0.2, help="silo suite: settling time (s)")
    ap.add_argument("--silo-discharge", type=float, default=1.0, help="silo suite: discharge time (s)")
    ap.add_argument("--silo-mlcg", action="store_true", help="silo suite: also the multi-level silo")
    ap.add_argument("--silo-mlcg-only", action="store_true", help="silo suite: the multi-level silo only")
    ap.add_argument("--silo-mlcg-multirate", action="store_true",
                    help="silo suite: also the multi-level silo with the coarse level at 2 dt (multi-rate)")
    ap.add_argument("--silo-mlcg-calls", action="store_true",
                    help="silo suite: multi-level runs by per-interval calls (coupling graph + dem_step) instead of "
                         "dem_step_coupled")
    ap.add_argument("--silo-mlcg-multirate-only", action="store_true",
                    help="silo suite: the multi-rate multi-level silo only")
    ap.add_argument("--suite", choices=("plain", "batch", "adjoint", "silo"), default="plain",
                    help="plain: the 1e6-sphere bed (default); batch: 64-system and two-level batches vs plain")
    ap.add_argument("--no-autotune", action="store_true", help="batch suite: default launch shape and skin")
    ap.add_argument("--profile-pass", action="store_true",
                    help="a few non-graph steps, three list rebuilds and a 256 MiB device copy (counter "
                         "calibration), no JSON")
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
    if args.suite == "adjoint":
        adjoint_suite(args)
        return
    if args.suite == "batch":
        batch_suite(args)
        return
    if args.suite == "silo":
        silo_suite(args)
        return
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
        for _ in range(3):                   # neighbour builds with history carry
            g.bin()
            g.neighbors()
        torch.cuda.synchronize()
        nbytes = 256 << 20
        src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"profile pass done: {args.timing_steps} steps, 3 rebuilds, 3 copies of {nbytes} bytes")
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
    copy_gbs = copy_bandwidth()
    roofline = {"bound": "hbm", "kernel": "k_step (fused forces + kick + kick-drift)",
                "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "alg_bytes_per_launch": round(bytes_step), "avg_launch_us": round(kernels["step"]["avg_us"], 2),
                "copy_GBps": round(copy_gbs, 1), "frac_of_copy": round(achieved / copy_gbs, 4)}

    # forced rebuilds: dem_bin and dem_neighbors every `rebuild_every` steps,
    # each call timed with events on the library's stream
    forced = None
    if args.rebuilds > 0:
        every = args.rebuild_every
        log(f"{args.rebuilds} forced rebuilds, one every {every} steps")
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(3 * args.rebuilds)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for r in range(args.rebuilds):
            g.step(every)
            evs[3 * r].record(g.stream)
            g.bin()
            evs[3 * r + 1].record(g.stream)
            g.neighbors()
            evs[3 * r + 2].record(g.stream)
        torch.cuda.synchronize()
        wall_r = time.perf_counter() - t0
        bin_ms = sorted(evs[3 * r].elapsed_time(evs[3 * r + 1]) for r in range(args.rebuilds))
        nbr_ms = sorted(evs[3 * r + 1].elapsed_time(evs[3 * r + 2]) for r in range(args.rebuilds))
        nbr_med = nbr_ms[len(nbr_ms) // 2]
        h = 2.0 * float(bed.r.max()) + float(bed.skin)         # default cell edge: the cut-off
        ncell = 1
        for ax in range(3):
            ncell *= max(1, int((bed.hi[ax] - bed.lo[ax]) / (h * (1.0 + 1e-9))))
        nbr_bytes = (n * NBR_PER_PARTICLE + slots * NBR_PER_SLOT + contacts_step * NBR_PER_CONTACT
                     + ncell * NBR_PER_CELL)
        forced = {"every": every, "calls": args.rebuilds,
                  "particle_steps_per_s": n * every * args.rebuilds / wall_r,
                  "bin_ms_median": bin_ms[len(bin_ms) // 2], "neighbors_ms_median": nbr_med,
                  "neighbors_alg_bytes": round(nbr_bytes),
                  "neighbors_GBps": round(nbr_bytes / (nbr_med * 1e-3) / 1e9, 1),
                  "neighbors_frac": round(nbr_bytes / (nbr_med * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                  "neighbors_traffic": read_traffic("nbr_hbm_bytes_per_launch")}

    # the small correctness workload: only its latency per step means anything
    # (its state and lists fit in L2)
    small = None
    if args.small_steps > 0:
        fcc = W.plain_fcc()
        gs = dem.DemSystem(fcc, use_graph=True, chunk=64)
        gs.prime()
        gs.step(64)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(gs.stream)
        gs.step(args.small_steps)
        e1.record(gs.stream)
        torch.cuda.synchronize()
        small = {"workload": f"{fcc.n} spheres on a jittered FCC subset, 20x20 mm periodic, dt 1e-6 s",
                 "steps": args.small_steps, "ms_per_step": e0.elapsed_time(e1) / args.small_steps}
        del gs

    # the metric's other two parts, compact: the 64-system batch and the
    # two-level chute against plain stepping (library defaults, no tuner), and
    # the adjoint of the 200-step chute rollout against the plain rollout
    batched = adjoint = None
    if not args.no_suites:
        import copy
        del g
        torch.cuda.empty_cache()
        ab = copy.copy(args)
        ab.no_autotune, ab.steps = True, 10000      # the suite's own step counts (2000 and 5000)
        b = batch_suite(ab, emit=False)
        batched = {"launch": "library defaults, graph replay",
                   "batch64": {k: b["batch64"][k] for k in ("systems", "particles", "steps", "batched",
                                                            "sequential_plain", "equal_n_plain",
                                                            "batched_vs_sequential", "batched_vs_equal_n",
                                                            "multirate")},
                   "two_level_chute": {k: b["two_level_chute"][k] for k in ("particles", "steps", "batched",
                                                                           "sequential_plain",
                                                                           "batched_vs_sequential", "coupled",
                                                                           "exchange")}}
        keys = ("workload", "steps", "window", "keep", "kslots", "windows", "max_windows", "plain_forward_s",
                "adjoint_forward_s", "backward_s", "adjoint_vs_plain", "adjoint_workspace_bytes",
                "context_workspace_bytes", "peak_torch_bytes")
        # the headline: checkpoints every 20 steps, each window recomputed by the
        # backward (memory bounded by the window); the kept mode (every step's
        # inputs stored, nothing recomputed) is reported beside it
        aa = copy.copy(args)
        aa.keep, aa.window = False, 20
        a_ = adjoint_suite(aa, emit=False)
        adjoint = {k: a_[k] for k in keys}
        torch.cuda.empty_cache()
        ak = copy.copy(args)
        ak.keep, ak.window = True, 20
        k_ = adjoint_suite(ak, emit=False)
        adjoint["kept_mode"] = {k: k_[k] for k in keys if k not in ("workload", "steps", "window")}
        torch.cuda.empty_cache()

    cpu = None
    if not args.no_cpu_baseline:
        log(f"CPU oracle baseline: {args.cpu_steps} steps")
        cpu = cpu_baseline(bed, args.cpu_steps, args.cpu_par_steps)

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
        "listed_pairs_per_s": slots / 2.0 * steps / seconds,
        "listed_slots": slots,
        "contacts_per_step": unordered_per_step,
        "wall_contacts_per_step": wall_contacts / steps,
        "list_builds": builds,
        "gpu_event_ms": gpu_ms,
        "roofline": roofline,
        "kernels": kernels,
        "forced_rebuild": forced,
        "small_latency": small,
        "batched_vs_plain": batched,
        "adjoint_vs_plain": adjoint,
        "cpu_baseline": cpu,
        "kernel_source": kernel_source_hash(),
        "device": torch.cuda.get_device_name(0),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
