"""Pins of the oracle's coupling fields and controllers (Sec. 2.3, Eq. 7).

  * Eq. (7) contact part: a uniformly compressed FCC crystal at rest carries
    the isotropic pressure p = 2 sqrt(2) f_n / d^2 (lattice sums: twelve
    neighbours at distance d, sum of n n over them = 4 I, 4 spheres per cubic
    cell of edge a = sqrt(2) d), with the Hertz force f_n = (4/3) E* sqrt(R)
    delta^(3/2); its volume fraction is 16 pi r^3 / (3 a^3).
  * Eq. (7) kinetic part and the Favre average: a contact-free lattice of two
    sphere sizes drifting at U with fluctuations that cancel in the
    mass-weighted mean but not in the plain mean: the Favre velocity is U and
    the kinetic stress is the fluctuation's sum of m w w / V.
  * the P controller: the forces of a cell, divided by the cell's mass, give
    kp (target - u_c) (a dead-beat gain kp = 1/dt moves the Favre velocity to
    the target in one unit of time); mass-flow mode scales the fine velocity
    by the volume-fraction mismatch.
  * the PI controller: the force acts along the inward normal, fades to zero
    3/2 diameters below the boundary face and never accelerates a sphere past
    the coarse cell's maximum velocity.
"""
import math

import numpy as np
import pytest

import coupling as C
import oracle as O
from paper_1705_03850_amd.inputs.workloads import MAT_A, System
from systems import e_star, mat, sphere_mass

TAU = 4                        # cubic FCC cells per edge of the crystal


def fcc_crystal(r=1e-3, delta=1e-6, cells=TAU, v=None, w=None, m=None, shift=0.25):
    """A periodic FCC crystal of spheres of radius r whose 12 nearest
    neighbours overlap by delta; sites shifted by `shift` a off the box faces."""
    d = 2 * r - delta
    a = math.sqrt(2.0) * d
    base = np.array([[0, 0, 0], [0.5, 0.5, 0], [0.5, 0, 0.5], [0, 0.5, 0.5]])
    sites = []
    for i in range(cells):
        for j in range(cells):
            for k in range(cells):
                sites.append(base + np.array([i, j, k]) + shift)
    x = np.concatenate(sites) * a
    nsph = len(x)
    L = cells * a
    return System(x=x, v=np.zeros((nsph, 3)) if v is None else v, w=np.zeros((nsph, 3)) if w is None else w,
                  r=np.full(nsph, r), type=np.zeros(nsph, np.int32), id=np.arange(nsph, dtype=np.int32),
                  materials=[m or MAT_A], lo=(0.0, 0.0, 0.0), hi=(L, L, L), periodic=(1, 1, 1), wall_z0=0,
                  g=(0.0, 0.0, 0.0), dt=1e-6, skin=0.1e-3, steps=0, name="fcc_crystal"), a, d


def check_fcc_pressure(fields_fn=C.cell_fields):
    s, a, d = fcc_crystal()
    o = O.Oracle(s)
    L = s.hi[0]
    n = (2, 2, 2)
    h = (L / 2,) * 3
    f = fields_fn(s, o, s.lo, h, n)
    m = MAT_A
    R = 0.5e-3
    delta = 1e-6
    fn = 4.0 / 3.0 * e_star(m, m) * math.sqrt(R) * delta ** 1.5
    p = 2.0 * math.sqrt(2.0) * fn / d ** 2
    assert np.all(f["count"] == 4 * (TAU // 2) ** 3)
    for c in range(8):
        np.testing.assert_allclose(f["stress"][c], p * np.eye(3), rtol=0, atol=1e-12 * p)
    np.testing.assert_allclose(f["phi"], 16 * math.pi * 1e-9 / (3 * a ** 3), rtol=1e-13)
    assert np.all(f["vmax"] == 0.0)
    return p


def test_fcc_crystal_pressure_and_volume_fraction():
    check_fcc_pressure()


def drifting_gas(U=(0.3, -0.2, 0.1), c=0.05):
    """Contact-free simple cubic lattice (spacing 3 mm) of alternating radii 0.5
    and 0.8 mm.  Sphere k moves at U + w_k with w_k = +c x^ (small spheres) or
    -c (m_small / m_large) x^ (large spheres), so that sum m w = 0 per pair of
    neighbours along x while the plain mean of w is not zero."""
    sp = 3e-3
    nx, ny, nz = 8, 4, 4
    g = np.stack(np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij"), -1).reshape(-1, 3)
    x = (g + 0.5) * sp
    small = (g[:, 0] % 2) == 0
    r = np.where(small, 0.5e-3, 0.8e-3)
    ms, ml = sphere_mass(0.5e-3, MAT_A.rho), sphere_mass(0.8e-3, MAT_A.rho)
    wx = np.where(small, c, -c * ms / ml)
    v = np.tile(np.array(U), (len(x), 1))
    v[:, 0] += wx
    s = System(x=x, v=v, w=np.zeros_like(v), r=r, type=np.zeros(len(x), np.int32), id=np.arange(len(x), dtype=np.int32),
               materials=[MAT_A], lo=(0.0, 0.0, 0.0), hi=(nx * sp, ny * sp, nz * sp), periodic=(1, 1, 1),
               wall_z0=0, g=(0.0, 0.0, 0.0), dt=1e-6, skin=0.1e-3, steps=0, name="drifting_gas")
    return s, np.array(U), wx, ms, ml


def test_favre_velocity_and_kinetic_stress():
    s, U, wx, ms, ml = drifting_gas()
    o = O.Oracle(s)
    L = np.array(s.hi)
    n = (2, 1, 1)                                 # each cell: 4 x 4 x 4 spheres, half small, half large
    f = C.cell_fields(s, o, s.lo, L / np.array(n), n)
    V = float(np.prod(L / np.array(n)))
    for cell in range(2):
        np.testing.assert_allclose(f["favre"][cell], U, rtol=0, atol=1e-15)
        kxx = 32 * (ms * 0.05 ** 2 + ml * (0.05 * ms / ml) ** 2) / V
        expect = np.zeros((3, 3))
        expect[0, 0] = kxx
        np.testing.assert_allclose(f["stress"][cell], expect, rtol=0, atol=1e-12 * kxx)
        np.testing.assert_allclose(f["vmax"][cell], np.linalg.norm(U + np.array([0.05, 0, 0])), rtol=1e-15)
        vol = 32 * 4.0 / 3.0 * math.pi * (0.5e-3 ** 3 + 0.8e-3 ** 3)
        np.testing.assert_allclose(f["phi"][cell], vol / V, rtol=1e-14)
    # the plain mean would not remove the fluctuation: this pins the mass weighting
    assert abs(np.mean(wx)) > 1e-3


def test_contact_stress_split_between_cells():
    """A single pair in contact across a cell face: each cell gets half of
    d (x) f, so the sum over the two cells times their volume is d (x) f (Eq. 7
    counts a contact once in total)."""
    r = 1e-3
    x = np.array([[5e-3 - r + 1e-6, 5e-3, 5e-3], [5e-3 + r - 1e-6, 5.02e-3, 5.01e-3]])
    s = System(x=x, v=np.array([[0.01, 0.02, 0.0], [-0.01, 0.0, 0.03]]), w=np.array([[0, 0, 50.0], [10.0, 0, 0]]),
               r=np.array([r, r]), type=np.zeros(2, np.int32), id=np.array([0, 1], np.int32), materials=[mat()],
               lo=(0.0, 0.0, 0.0), hi=(10e-3, 10e-3, 10e-3), periodic=(0, 0, 0), wall_z0=0, g=(0.0, 0.0, 0.0),
               dt=1e-6, skin=0.1e-3, steps=0, name="pair_across_face")
    o = O.Oracle(s)
    o.set_history(np.array([0]), np.array([1]), np.array([[0.0, 1e-7, -2e-7]]))
    f = C.cell_fields(s, o, (0.0, 0.0, 0.0), (5e-3, 10e-3, 10e-3), (2, 1, 1))
    lo, hi, d, fo = o.pair_forces()
    assert len(lo) == 1
    V = 5e-3 * 10e-3 * 10e-3
    dxf = d[0][:, None] * fo[0][None, :]
    np.testing.assert_allclose(f["contact_stress"][0] * V, 0.5 * dxf, rtol=1e-15, atol=0)
    np.testing.assert_allclose(f["contact_stress"][1] * V, 0.5 * dxf, rtol=1e-15, atol=0)
    assert abs(dxf[0, 1] - dxf[1, 0]) > 1e-3 * abs(dxf[0, 0])     # tangential force: not symmetric


def test_p_controller_moves_favre_velocity():
    rng = np.random.default_rng(3)
    N = 400
    x = rng.uniform(0, 1, (N, 3)) * np.array([0.1, 0.05, 0.05])
    m = rng.uniform(1e-5, 3e-5, N)
    lo, h, n = (0.0, 0.0, 0.0), (0.025, 0.025, 0.025), (4, 2, 2)
    fine = dict(mass=rng.uniform(1, 2, 16), volume=rng.uniform(1e-6, 2e-6, 16), favre=rng.normal(size=(16, 3)))
    coarse = dict(mass=rng.uniform(1, 2, 16), volume=rng.uniform(1e-6, 2e-6, 16), favre=rng.normal(size=(16, 3)))
    fine["mass"][5] = 0.0                          # no fine mass: no correction there
    c = C.cell_index(x, lo, h, n)
    for mass_flow in (False, True):
        kp = 123.0
        F = C.p_forces(x, m, lo, h, n, fine, coarse, kp, mass_flow)
        for cell in range(16):
            sel = c == cell
            if not sel.any():
                continue
            dv = F[sel].sum(axis=0) / m[sel].sum()
            if cell == 5:
                assert np.all(F[sel] == 0.0)
                continue
            target = fine["favre"][cell] * (fine["volume"][cell] / coarse["volume"][cell] if mass_flow else 1.0)
            np.testing.assert_allclose(dv, kp * (target - coarse["favre"][cell]), rtol=1e-12)
        assert np.all(F[c < 0] == 0.0)


def test_pi_controller_direction_fade_and_velocity_limit():
    rng = np.random.default_rng(4)
    N = 3000
    lo, h, n = (0.0, 0.0, 0.09), (0.02, 0.02, 0.01), (3, 2, 1)      # one layer below the face z = 0.1
    x = np.column_stack([rng.uniform(0, 0.06, N), rng.uniform(0, 0.04, N), rng.uniform(0.085, 0.1005, N)])
    r = rng.uniform(0.8e-3, 1.2e-3, N)
    m = 4 / 3 * np.pi * 2500 * r ** 3
    v = rng.normal(0, 0.05, (N, 3))
    normal, face, fade, dt = (0.0, 0.0, -1.0), -0.1, 1.5, 1e-6     # inward normal -z: depth = 0.1 - z
    u, integral = C.pi_update(np.full(6, 500.0), np.full(6, 200.0), np.zeros(6), 2.0, 1e3, 15 * dt)
    np.testing.assert_allclose(u, 2.0 * 300 + 1e3 * 300 * 15 * dt)
    np.testing.assert_allclose(integral, 300 * 15 * dt)
    vmax = np.full(6, 0.08)
    F = C.pi_forces(x, v, r, m, dt, lo, h, n, normal, face, fade, u, vmax)
    depth = 0.1 - x[:, 2]
    assert np.all(F[:, :2] == 0.0)
    assert np.all(F[:, 2] <= 0.0)                                     # pushed into the fine region (-z)
    far = depth >= 3.0 * r
    assert np.all(F[far] == 0.0) and (far & (C.cell_index(x, lo, h, n) >= 0)).any()
    vn_new = -v[:, 2] + dt * (-F[:, 2]) / m                          # velocity along the inward normal
    slow = -v[:, 2] <= vmax[0]
    assert np.all(vn_new[slow] <= vmax[0] * (1 + 1e-12))
    assert np.all(F[~slow] == 0.0)
    # below the limit the force is u pi r^2 (1 - depth / 3 r)
    c = C.cell_index(x, lo, h, n)
    free = (c >= 0) & (depth > 0) & (depth < 3 * r)
    raw = u[0] * np.pi * r ** 2 * (1 - depth / (3 * r))
    unl = free & (vn_new < vmax[0] * (1 - 1e-9))
    assert unl.sum() > 100
    np.testing.assert_allclose(-F[unl, 2], raw[unl], rtol=1e-14)
