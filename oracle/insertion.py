"""Insertion and deletion of fine spheres at the boundary of the fine region
(multi-level coarse-grain model, Sec. 2.3), written out plainly with numpy.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check of the entry module
and the CPU-baseline leg of the benchmark may import this module; the GPU
library never imports or links it and shares nothing with it.

The paper measures, per cell of the fine region's boundary surface, the mass
flow, velocity and size distribution of the coarse particles, Favre-averages
the velocity over a coupling interval, and inserts fine particles cell by cell
by simple sequential inhibition (SSI), as ensembles that keep the local size
distribution.  Readings where it is silent (also in the repository's design
notes):
  S-1 inflow: per boundary cell, a slab of height h on the coarse side of the
      face with inward unit normal n: the mass flow into the fine region is
      max(0, n . P) / h, P the cell's momentum sum (the coarse cell fields);
      each interval T adds it times T to the cell's mass budget, which carries
      over between intervals;
  S-2 candidates (positions in the cell's insertion slab inside the fine
      region, radii from the cell's coarse radii divided by the coarse-grain
      factor, types) are drawn by the caller from a seeded generator and
      passed in, in one global order;
  S-3 SSI: candidate k is accepted iff its mass (4/3) pi rho r^3 is at most
      its cell's remaining budget and its sphere overlaps no sphere of the
      fine system and no candidate accepted before it:
      d^2 < (r_k + r_j)^2, d^2 = (dx dx + dy dy) + dz dz with the minimum
      image on periodic axes; an accepted candidate takes its mass from the
      budget;
  S-4 inserted spheres move with their cell's Favre velocity, do not spin,
      and take the ids after the system's largest;
  S-5 deletion: a fine sphere whose centre lies on the outer side of the
      region's plane, x . n < d (evaluated as (x nx + y ny) + z nz), is
      removed, and its history with it.
"""
from __future__ import annotations

import math

import numpy as np


def min_image(d: float, L: float, periodic: int) -> float:
    if not periodic:
        return d
    if d > 0.5 * L:
        return d - L
    if d < -0.5 * L:
        return d + L
    return d


def overlaps(xa, ra, xb, rb, box_L, periodic) -> bool:
    dx = min_image(xa[0] - xb[0], box_L[0], periodic[0])
    dy = min_image(xa[1] - xb[1], box_L[1], periodic[1])
    dz = min_image(xa[2] - xb[2], box_L[2], periodic[2])
    d2 = dx * dx + dy * dy + dz * dz
    s = ra + rb
    return d2 < s * s


def overlaps_many(xa, ra, xb, rb, box_L, periodic) -> np.ndarray:
    """overlaps() of one sphere against many (the same arithmetic, elementwise)."""
    d = []
    for a in range(3):
        v = xa[a] - xb[:, a]
        if periodic[a]:
            h = 0.5 * box_L[a]
            v = np.where(v > h, v - box_L[a], np.where(v < -h, v + box_L[a], v))
        d.append(v)
    d2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2]
    s = ra + rb
    return d2 < s * s


def sphere_mass(r: float, rho: float) -> float:
    return 4.0 / 3.0 * math.pi * rho * r * r * r


def inflow_budget(budget, momentum, normal, slab_height, interval):
    """S-1: budget + max(0, n . P) / h * T per cell (momentum: (ncell, 3))."""
    n = np.asarray(normal, float)
    flow = momentum[:, 0] * n[0] + momentum[:, 1] * n[1] + momentum[:, 2] * n[2]
    return np.asarray(budget, float) + np.maximum(flow, 0.0) / slab_height * interval


def ssi_accept(existing_x, existing_r, cand_x, cand_r, cand_rho, cand_cell, budget, box_L, periodic):
    """S-3, candidate by candidate in the given order.  Returns (accepted
    flags, remaining budget); brute force over every existing sphere."""
    budget = np.array(budget, float)
    acc = np.zeros(len(cand_x), np.int32)
    taken = []
    for k in range(len(cand_x)):
        m = sphere_mass(float(cand_r[k]), float(cand_rho[k]))
        c = int(cand_cell[k])
        if not m <= budget[c]:
            continue
        if len(existing_x) and np.any(overlaps_many(cand_x[k], cand_r[k], existing_x, existing_r, box_L, periodic)):
            continue
        if any(overlaps(cand_x[k], cand_r[k], cand_x[a], cand_r[a], box_L, periodic) for a in taken):
            continue
        acc[k] = 1
        taken.append(k)
        budget[c] -= m
    return acc, budget


def outside(x, normal, d):
    """S-5: centres on the outer side of the plane x . n < d."""
    n = np.asarray(normal, float)
    return (x[:, 0] * n[0] + x[:, 1] * n[1] + x[:, 2] * n[2]) < d


def favre_velocity(mass, momentum):
    """S-4: the mass-weighted mean velocity P / M of each cell; zero in a cell
    that holds no mass."""
    mass = np.asarray(mass, float)
    out = np.zeros((len(mass), 3))
    nz = mass > 0
    out[nz] = momentum[nz] / mass[nz, None]
    return out


def exchange(system, orc, normal, d, cand_x, cand_r, cand_type, cand_cell, budget, cell_mass, cell_mom,
             id_base, fext=None, outlet=None, surfaces=None):
    """One insertion-and-deletion event of the fine system (S-1 .. S-5, with
    the budget already topped up by inflow_budget).  Deletion first (S-5),
    then SSI against the kept spheres (S-3), the accepted candidates appended
    in candidate order with ids id_base, id_base + 1, ... and their cell's
    Favre velocity (S-4); the pair and wall history of the kept spheres is
    carried by id.  `outlet` (normal, offset): a second half-space whose
    outer side is removed too (a silo's outlet).  Returns (new system, new oracle, accepted flags, budget,
    kept mask, external forces of the new system)."""
    import oracle as O

    st = orc.state()
    keep = ~outside(st["x"], normal, d)
    if outlet is not None:                       # a second bounding half-space (normal, offset)
        keep &= ~outside(st["x"], outlet[0], outlet[1])
    xk = st["x"][keep]
    rk = system.r[keep]
    box_L = [system.hi[a] - system.lo[a] for a in range(3)]
    rho = np.array([system.materials[int(t)].rho for t in cand_type])
    acc, budget = ssi_accept(xk, rk, cand_x, cand_r, rho, cand_cell, budget, box_L, system.periodic)
    a = acc.astype(bool)
    na = int(a.sum())
    vf = favre_velocity(cell_mass, cell_mom)
    new = system.copy()
    new.x = np.concatenate([xk, cand_x[a]])
    new.v = np.concatenate([st["v"][keep], vf[np.asarray(cand_cell)[a]]])
    new.w = np.concatenate([st["w"][keep], np.zeros((na, 3))])
    new.r = np.concatenate([rk, np.asarray(cand_r, float)[a]])
    new.type = np.concatenate([system.type[keep], np.asarray(cand_type, np.int32)[a]]).astype(np.int32)
    new.id = np.concatenate([system.id[keep], id_base + np.arange(na)]).astype(np.int32)
    o2 = O.Oracle(new, lib_path=getattr(orc, "lib_path", None))
    kept_ids = set(int(i) for i in system.id[keep])
    lo, hi, xi = orc.history()
    sel = np.array([int(p) in kept_ids and int(q) in kept_ids for p, q in zip(lo, hi)], bool)
    o2.set_history(lo[sel], hi[sel], xi[sel])
    wid, wxi = orc.wall_history()
    wsel = np.array([int(p) in kept_ids for p in wid], bool)
    o2.set_wall_history(wid[wsel], wxi[wsel])
    if surfaces is not None:                     # static wall surfaces and their history
        o2.set_surfaces(surfaces)
        sid, sk, sxi = orc.surface_history()
        ssel = np.array([int(p) in kept_ids for p in sid], bool)
        o2.set_surface_history(sid[ssel], sk[ssel], sxi[ssel])
    f2 = None
    if fext is not None:
        f2 = np.concatenate([np.asarray(fext, float)[keep], np.zeros((na, 3))])
        o2.set_external(f2)
    return new, o2, acc, budget, keep, f2
