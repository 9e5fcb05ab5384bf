"""Cell fields and coupling controllers of the multi-level coarse-grain model,
written out plainly with numpy.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check of the entry module
and the CPU-baseline leg of the benchmark may import this module; the GPU
library never imports or links it and shares nothing with it.

What it computes (Queteschiner et al., CFD2017, Sec. 2.3):
  * per hexahedral cell: the granular stress of Eq. (7), the volume fraction,
    the Favre-averaged (mass-weighted) velocity and the maximum particle
    velocity (the Eulerian properties of the transition layer and of the grid
    inside the fine region);
  * the PI controller on the fine particles of the transition layer: process
    variable the fine normal stress, setpoint the coarse one, output a
    correcting force, limited so that a particle does not exceed the coarse
    cell's maximum velocity, fading out 3/2 fine diameters from the boundary;
  * the P controller on the coarse particles inside the fine region: velocity
    or mass flow, where the mass-flow target is the fine velocity times the
    volume-fraction mismatch.

Readings where the paper is silent (also listed in the repository's design
notes):
  F-1 cells are the boxes of a regular grid (corner lo, edges h, counts n; cell
      (a, b, c) has index (c n1 + b) n0 + a); a sphere belongs to the cell that
      contains its centre, spheres outside the grid to none;
  F-2 in Eq. (7) V is the cell volume; the contact part sums over the spheres i
      of the cell and their contacts j the term 1/2 d_ij (x) f_ij, component
      (a, b) = d_a f_b, with d_ij = x_i - x_j (minimum image) and f_ij the
      force on i; wall contacts are not pairs and do not enter; the forces are
      those of the current state with the stored history, not advanced (a
      force evaluation without history update); the kinetic part uses the
      fluctuation v' = v - u about the cell's Favre velocity u;
  F-3 volume fraction = sum over the cell's spheres of (4/3) pi r^3, divided by
      the cell volume; maximum velocity = max |v| over the cell's spheres;
  F-4 PI controller, per transition cell with inward unit normal n (pointing
      into the fine region): error e = s* - s, where s = n . sigma . n of the
      fine cell and s* the coarse setpoint; integral I += e T (T the coupling
      interval); output u = kp e + ki I (a stress);
  F-5 force on a fine sphere of the cell: F = u (pi r^2) w n with the fade
      w = 1 - s / (k 2 r) for 0 <= s < k 2 r, 1 for s < 0 and 0 beyond, where
      s = x . n - face is the depth below the boundary face and k = 3/2; then
      limited along n: for F > 0 to at most m (vmax - v.n) / dt, for F < 0 to
      at least m (-vmax - v.n) / dt, and never reversed (0 if the sphere is
      already faster than vmax), vmax the coarse cell's maximum velocity;
  F-6 P controller, per cell of the grid inside the fine region, when both the
      fine and the coarse cell hold mass: target = u_f (velocity mode) or
      u_f phi_f / phi_c (mass-flow mode); force on each coarse sphere of the
      cell F = kp m (target - u_c) with u_c the coarse Favre velocity.
"""
from __future__ import annotations

import math

import numpy as np


def cell_index(x: np.ndarray, lo, h, n) -> np.ndarray:
    """Cell of each centre (F-1), -1 outside the grid."""
    lo = np.asarray(lo, float); h = np.asarray(h, float); n = np.asarray(n, int)
    c = np.floor((x - lo) / h).astype(np.int64)
    inside = np.all((c >= 0) & (c < n), axis=1)
    idx = (c[:, 2] * n[1] + c[:, 1]) * n[0] + c[:, 0]
    return np.where(inside, idx, -1)


def cell_fields(system, orc, lo, h, n) -> dict:
    """Eq. (7) and the other cell fields of the oracle's current state.

    Returns count, mass, momentum (ncell, 3), solids volume, vmax, favre
    (ncell, 3; zero where the cell is empty), phi and stress (ncell, 3, 3):
    contact + kinetic parts over the cell volume (F-2, F-3)."""
    st = orc.state()
    x, v = st["x"], st["v"]
    m, _ = orc.mass()
    r = np.asarray(system.r, float)
    ncell = int(np.prod(n))
    vcell = float(np.prod(h))
    c = cell_index(x, lo, h, n)
    inn = c >= 0
    count = np.zeros(ncell)
    mass = np.zeros(ncell)
    mom = np.zeros((ncell, 3))
    vol = np.zeros(ncell)
    vmax = np.zeros(ncell)
    np.add.at(count, c[inn], 1.0)
    np.add.at(mass, c[inn], m[inn])
    np.add.at(mom, c[inn], m[inn, None] * v[inn])
    np.add.at(vol, c[inn], 4.0 / 3.0 * math.pi * r[inn] ** 3)
    np.maximum.at(vmax, c[inn], np.sqrt(np.sum(v[inn] ** 2, axis=1)))
    favre = np.zeros((ncell, 3))
    full = mass > 0
    favre[full] = mom[full] / mass[full, None]
    # kinetic part: fluctuations about the cell's Favre velocity
    kin = np.zeros((ncell, 3, 3))
    vp = v[inn] - favre[c[inn]]
    np.add.at(kin, c[inn], m[inn, None, None] * vp[:, :, None] * vp[:, None, :])
    # contact part: every contact counted from both spheres with 1/2 d (x) f
    lo_id, hi_id, d, f = orc.pair_forces()
    pos = {int(q): k for k, q in enumerate(system.id)}
    ia = np.array([pos[int(q)] for q in lo_id], dtype=np.int64)
    ib = np.array([pos[int(q)] for q in hi_id], dtype=np.int64)
    con = np.zeros((ncell, 3, 3))
    if len(ia):
        term = 0.5 * d[:, :, None] * f[:, None, :]        # the same for both spheres: (-d) (x) (-f)
        for side in (ia, ib):
            cs = c[side]
            ok = cs >= 0
            np.add.at(con, cs[ok], term[ok])
    stress = (con + kin) / vcell
    return dict(count=count, mass=mass, momentum=mom, volume=vol, vmax=vmax, favre=favre, phi=vol / vcell,
                stress=stress, contact_stress=con / vcell, kinetic_stress=kin / vcell)


def normal_stress(stress: np.ndarray, normal) -> np.ndarray:
    """n . sigma . n per cell."""
    nn = np.asarray(normal, float)
    return np.einsum("a,cab,b->c", nn, stress, nn)


def pi_update(setpoint, measured, integral, kp, ki, interval):
    """One discrete PI update per cell (F-4): returns (u, new integral)."""
    e = np.asarray(setpoint, float) - np.asarray(measured, float)
    integral = np.asarray(integral, float) + e * interval
    return kp * e + ki * integral, integral


def pi_forces(x, v, r, m, dt, lo, h, n, normal, face, fade, u, vmax):
    """Correcting forces on the fine spheres of the transition cells (F-5),
    (N, 3); spheres outside the cells get zero."""
    nn = np.asarray(normal, float)
    c = cell_index(x, lo, h, n)
    F = np.zeros((len(x), 3))
    for i in np.nonzero(c >= 0)[0]:
        depth = float(x[i] @ nn) - face
        reach = fade * 2.0 * r[i]
        if depth < 0.0:
            w = 1.0
        elif depth < reach:
            w = 1.0 - depth / reach
        else:
            continue
        mag = u[c[i]] * math.pi * r[i] ** 2 * w
        vn = float(v[i] @ nn)
        vm = vmax[c[i]]
        if mag > 0.0:
            mag = min(mag, max(0.0, m[i] * (vm - vn) / dt))
        elif mag < 0.0:
            mag = max(mag, min(0.0, m[i] * (-vm - vn) / dt))
        F[i] = mag * nn
    return F


def p_forces(x, m, lo, h, n, fine, coarse, kp, mass_flow: bool):
    """Correcting forces on the coarse spheres of the grid inside the fine
    region (F-6), (N, 3); `fine` and `coarse` are cell_fields of the same grid
    in the two systems."""
    c = cell_index(x, lo, h, n)
    ok = (fine["mass"] > 0) & (coarse["mass"] > 0)
    target = fine["favre"].copy()
    if mass_flow:
        ratio = np.zeros_like(fine["volume"])
        ratio[ok] = fine["volume"][ok] / coarse["volume"][ok]
        target = target * ratio[:, None]
    F = np.zeros((len(x), 3))
    for i in np.nonzero(c >= 0)[0]:
        if ok[c[i]]:
            F[i] = kp * m[i] * (target[c[i]] - coarse["favre"][c[i]])
    return F
