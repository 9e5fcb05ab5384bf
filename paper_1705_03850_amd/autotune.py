"""Launch-shape and neighbour-list autotuner for a batch of DEM systems.

Chooses, by timing short runs on the GPU:
  * threads per particle in the force pass (lanes) and threads per block,
  * the neighbour-list skin (as a factor of each system's largest radius),
  * the cell edge (as a factor of each system's cut-off 2 r_max + skin).
None of these changes the results (rows are summed in neighbour-id order and
the history follows ids; bit-for-bit equality is tested), so the tuner only
trades list length against rebuild frequency and occupancy.  The choice can
be written to a JSON file and reused.
"""
from __future__ import annotations

import json
import time

from . import dem


def _time_run(systems, steps, skin_f, cell_f, block, lanes, use_graph=True, chunk=32):
    import torch

    skins = [skin_f * float(s.r.max()) for s in systems]
    cells = [cell_f * (2.0 * float(s.r.max()) + sk) for s, sk in zip(systems, skins)]
    g = dem.DemSystem(systems, block=block, lanes=lanes, skin=skins, cell=cells, use_graph=use_graph, chunk=chunk)
    g.prime()
    g.step(chunk)  # warm: graph capture, caches
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.step(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    builds = g.stats()["builds"]
    del g
    return dt / steps, builds


def autotune(systems, steps: int = 128, long_steps: int = 1024, out_json: str | None = None, log=print,
             reps: int = 2, margin: float = 0.02) -> dict:
    """Coordinate search.  The launch shape (lanes, block) is timed over `steps`
    steps; skin and cell are timed over `long_steps` steps, long enough for the
    list rebuilds they cause to show up in the time per step.  Every candidate
    is timed `reps` times, the candidates interleaved, and keeps its best time;
    a candidate replaces the current value only when it is faster by more than
    `margin` (timing noise of a few per cent otherwise flips the choice from
    run to run)."""
    best = {"skin_factor": 0.1, "cell_factor": 1.0, "block": 256, "lanes": 4}
    tried = []

    def run(nsteps, **kw):
        cfg = dict(best, **kw)
        try:
            sec, builds = _time_run(systems, nsteps, cfg["skin_factor"], cfg["cell_factor"], cfg["block"],
                                    cfg["lanes"])
        except dem.DemError as e:  # e.g. a cell too large for a small periodic box
            if log:
                log(f"autotune {cfg} rejected: {e}")
            return float("inf")
        tried.append(dict(cfg, steps=nsteps, ms_per_step=sec * 1e3, builds=builds))
        if log:
            log(f"autotune {cfg} over {nsteps} steps -> {sec * 1e3:.3f} ms/step ({builds} builds)")
        return sec

    for nsteps, key, values in ((steps, "lanes", (4, 8)), (steps, "block", (128, 256)),
                                (long_steps, "skin_factor", (0.1, 0.05, 0.2, 0.3)),
                                (long_steps, "cell_factor", (1.0, 1.25))):
        times = {}
        for _ in range(max(1, reps)):
            for v in values:
                times[v] = min(times.get(v, float("inf")), run(nsteps, **{key: v}))
        cand = min(times, key=times.get)
        if times[cand] < times[best[key]] * (1.0 - margin):
            best[key] = cand
    cur = min(t["ms_per_step"] for t in tried if all(t[k] == best[k] for k in best))
    result = dict(best, ms_per_step=cur, steps=steps, long_steps=long_steps, tried=tried)
    if out_json:
        with open(out_json, "w") as fh:
            json.dump(result, fh, indent=1)
    return result


def apply(systems, choice: dict):
    """Per-system skin and cell lists for DemSystem from a tuner choice."""
    skins = [choice["skin_factor"] * float(s.r.max()) for s in systems]
    cells = [choice["cell_factor"] * (2.0 * float(s.r.max()) + sk) for s, sk in zip(systems, skins)]
    return dict(skin=skins, cell=cells, block=choice["block"], lanes=choice["lanes"])
