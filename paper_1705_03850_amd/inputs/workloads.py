"""Seeded synthetic workloads for the DEM contact pipeline.

This module only *places* particles and draws their sizes, velocities and
types; it contains no contact mechanics and no time stepping.  Both the CPU
oracle and the GPU library are fed from here, so neither side generates its
own inputs.

Workloads (all lengths in metres, SI units throughout):

* ``plain_fcc``      -- 2,000 monodisperse spheres (r = 1 mm) on a jittered FCC
                        subset in a 20 x 20 mm footprint periodic in x and y,
                        wall at z = 0, vertical gravity (the small plain case).
* ``settled_bed``    -- N polydisperse spheres, r ~ U[0.8, 1.2] mm, deposited
                        by the geometric drop-and-roll construction on an
                        80 x 80 mm periodic footprint, then compacted
                        vertically (the at-scale plain case, N = 1e6).
* ``chute_two_level``-- a coarse (alpha = 4) and a fine (alpha = 1) bed on a
                        30 degree chute, as one two-system batch.
* ``batch_systems``  -- 64 independent deposited beds with log-uniform
                        particle counts and coarse-grain factors in {1,2,4,8}.
* ``chute_adjoint``  -- 50,000 spheres of two material types on a 30 degree
                        chute with a sheared initial velocity profile.

The material sets are the ones the workloads are quoted with: E = 5e6 Pa,
nu = 0.25, rho = 2500 kg/m^3, e = 0.9, mu = 0.5 (and a second type with
E = 1e7 Pa, e = 0.7, mu = 0.3 for the two-type chute).  The coarse-grain rule
of the paper (Sec. 2.2) keeps E, nu, rho, e and mu fixed and scales only the
radius, so a coarse system differs from a fine one only in r.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = os.path.join(_HERE, "libdeposit.so")

G0 = 9.81


@dataclass
class Material:
    E: float
    nu: float
    rho: float
    e: float
    mu: float


MAT_A = Material(E=5e6, nu=0.25, rho=2500.0, e=0.9, mu=0.5)
MAT_B = Material(E=1e7, nu=0.25, rho=2500.0, e=0.7, mu=0.3)


@dataclass
class System:
    """One DEM system: particle arrays (row i = one particle) plus its setup."""

    x: np.ndarray          # (n, 3) float64 positions
    v: np.ndarray          # (n, 3) float64 velocities
    w: np.ndarray          # (n, 3) float64 angular velocities
    r: np.ndarray          # (n,)   float64 radii
    type: np.ndarray       # (n,)   int32 material index
    id: np.ndarray         # (n,)   int32 particle id (unique within the system)
    materials: list        # [Material]
    lo: tuple              # box lower corner
    hi: tuple              # box upper corner (z: top of the binning grid)
    periodic: tuple        # (px, py, pz) 0/1
    wall_z0: int           # flat wall at z = 0
    g: tuple               # gravity vector
    dt: float
    skin: float
    steps: int
    name: str = ""
    alpha: float = 1.0
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.r.shape[0])

    def copy(self) -> "System":
        return System(self.x.copy(), self.v.copy(), self.w.copy(), self.r.copy(), self.type.copy(),
                      self.id.copy(), list(self.materials), tuple(self.lo), tuple(self.hi),
                      tuple(self.periodic), self.wall_z0, tuple(self.g), self.dt, self.skin, self.steps,
                      self.name, self.alpha, dict(self.meta))


def _deposit_lib():
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(os.path.join(_HERE, "deposit.c")):
        build_deposit()
    lib = ctypes.CDLL(_LIB)
    dp = ctypes.POINTER(ctypes.c_double)
    lib.deposit.argtypes = [ctypes.c_int, dp, dp, dp, dp, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                            dp, dp, dp]
    lib.deposit.restype = ctypes.c_int
    return lib


def build_deposit() -> str:
    """Compile the deposition helper in place (plain gcc, no GPU code)."""
    src = os.path.join(_HERE, "deposit.c")
    tmp = _LIB + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", src, "-o", tmp, "-lm"])
    os.replace(tmp, _LIB)
    return _LIB


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def deposit(r: np.ndarray, Lx: float, Ly: float, rng: np.random.Generator, zcap: float | None = None):
    """Drop-and-roll deposition of spheres with radii ``r`` (in that order).

    Returns (n, 3) centres.  Random drop points and tie-break azimuths come from
    ``rng``; the geometry itself is deterministic.
    """
    r = np.ascontiguousarray(r, dtype=np.float64)
    n = r.shape[0]
    dx = rng.uniform(0.0, Lx, n)
    dy = rng.uniform(0.0, Ly, n)
    az = rng.uniform(0.0, 2.0 * math.pi, n)
    if zcap is None:
        zcap = 1.3 * float(np.sum(4.0 / 3.0 * math.pi * r ** 3)) / (0.55 * Lx * Ly) + 4.0 * float(r.max())
    x = np.empty(n); y = np.empty(n); z = np.empty(n)
    lib = _deposit_lib()
    stuck = lib.deposit(n, _ptr(r), _ptr(dx), _ptr(dy), _ptr(az), Lx, Ly, float(zcap), _ptr(x), _ptr(y), _ptr(z))
    return np.stack([x, y, z], axis=1), int(stuck)


def compact(z: np.ndarray, strain_bottom: float) -> np.ndarray:
    """Vertical compaction z -> z - int_0^z eps(s) ds with eps(s) = eps_b (1 - s/H)^(2/3).

    A heuristic stand-in for the load a settled bed carries: the strain is
    largest at the floor and vanishes at the free surface (H = max z).
    """
    H = float(z.max())
    if H <= 0.0 or strain_bottom == 0.0:
        return z.copy()
    # int_0^z (1 - s/H)^(2/3) ds = (3H/5) (1 - (1 - z/H)^(5/3))
    u = np.clip(1.0 - z / H, 0.0, 1.0)
    return z - strain_bottom * 0.6 * H * (1.0 - u ** (5.0 / 3.0))


# ----------------------------------------------------------------------------
# Workload 1: 2,000 spheres, jittered FCC subset
# ----------------------------------------------------------------------------

def plain_fcc(seed: int = 1, e: float | None = None, mu: float | None = None) -> System:
    """2,000 spheres, r = 1 mm, in a 20 x 20 mm footprint periodic in x/y.

    2,000 random non-overlapping spheres at packing fraction pi/6 cannot be
    produced by random sequential insertion (its jamming limit is ~0.38), so
    the positions are a seeded subset of an FCC lattice: lattice constant
    a = 20/7 mm (7 x 7 cubic cells span the footprint exactly; nearest
    neighbours at 2.0203 mm), 21 close-packed-direction planes at
    z = 1.01 mm + k a/2 (2,058 sites), 2,000 sites chosen at random, each
    coordinate jittered by U(-5, 5) um.  Velocities N(0, 0.1 m/s) per component
    with the mean removed; zero spin.
    """
    rng = np.random.default_rng(seed)
    a = 20e-3 / 7.0
    sites = []
    for k in range(21):
        z = 1.01e-3 + k * a / 2.0
        offs = [(0.0, 0.0), (0.5, 0.5)] if k % 2 == 0 else [(0.5, 0.0), (0.0, 0.5)]
        for cy in range(7):
            for cx in range(7):
                for ox, oy in offs:
                    sites.append(((cx + ox) * a, (cy + oy) * a, z))
    sites = np.asarray(sites, dtype=np.float64)
    pick = rng.choice(sites.shape[0], 2000, replace=False)
    x = sites[pick] + rng.uniform(-5e-6, 5e-6, (2000, 3))
    x[:, 0] = np.mod(x[:, 0], 20e-3)
    x[:, 1] = np.mod(x[:, 1], 20e-3)
    v = rng.normal(0.0, 0.1, (2000, 3))
    v -= v.mean(axis=0)
    mat = Material(MAT_A.E, MAT_A.nu, MAT_A.rho, MAT_A.e if e is None else e, MAT_A.mu if mu is None else mu)
    return System(x=x, v=v, w=np.zeros((2000, 3)), r=np.full(2000, 1e-3), type=np.zeros(2000, np.int32),
                  id=np.arange(2000, dtype=np.int32), materials=[mat], lo=(0.0, 0.0, 0.0),
                  hi=(20e-3, 20e-3, 60e-3), periodic=(1, 1, 0), wall_z0=1, g=(0.0, 0.0, -G0), dt=1e-6,
                  skin=0.1e-3, steps=1000, name="plain_fcc_2000")


# ----------------------------------------------------------------------------
# Workload 2: settled polydisperse bed
# ----------------------------------------------------------------------------

def bed(n: int, r: np.ndarray, Lx: float, Ly: float, rng: np.random.Generator, overlap_frac: float = 2.5e-4,
        strain_bottom: float = 0.02):
    """Deposit ``n`` spheres, then shrink all gaps slightly and compact vertically.

    Deposition uses radii r (1 - overlap_frac) so that every touching pair of
    the construction overlaps by overlap_frac (r_i + r_j) at the true radii;
    the vertical compaction adds the depth-dependent strain.
    """
    pos, stuck = deposit(r * (1.0 - overlap_frac), Lx, Ly, rng)
    pos[:, 2] = compact(pos[:, 2], strain_bottom)
    return pos, stuck


def _cache_path(name: str) -> str | None:
    d = os.environ.get("DEM_INPUT_CACHE", "/tmp/dem_input_cache")
    try:
        os.makedirs(d, exist_ok=True)
    except OSError:
        return None
    src = open(os.path.join(_HERE, "deposit.c"), "rb").read() + open(os.path.abspath(__file__), "rb").read()
    import hashlib
    tag = hashlib.sha256(src).hexdigest()[:16]
    return os.path.join(d, f"{name}_{tag}.npz")


def settled_bed(seed: int = 2, n: int = 1_000_000, footprint: float = 80e-3, cache: bool = True) -> System:
    """N spheres, r ~ U[0.8, 1.2] mm, on a periodic square footprint, settled by deposition.

    Deposition of 1e6 spheres takes ~20 s, so the result is kept in a cache
    file keyed by the arguments and a hash of the generator sources."""
    path = _cache_path(f"bed_{seed}_{n}_{footprint!r}") if cache else None
    if path and os.path.exists(path):
        with np.load(path, allow_pickle=False) as z:
            pos, r, ids, stuck = z["x"], z["r"], z["id"], int(z["stuck"])
        return _bed_system(pos, r, ids, footprint, n, stuck)
    pos, r, ids, stuck = _settled_bed_arrays(seed, n, footprint)
    if path:
        tmp = path + f".{os.getpid()}.tmp.npz"
        np.savez(tmp, x=pos, r=r, id=ids, stuck=stuck)
        os.replace(tmp, path)
    return _bed_system(pos, r, ids, footprint, n, stuck)


def _bed_system(pos, r, ids, footprint, n, stuck):
    rmax = 1.2e-3
    top = float(pos[:, 2].max()) + 4.0 * rmax
    return System(x=pos, v=np.zeros((n, 3)), w=np.zeros((n, 3)), r=r, type=np.zeros(n, np.int32), id=ids,
                  materials=[MAT_A], lo=(0.0, 0.0, 0.0), hi=(footprint, footprint, top), periodic=(1, 1, 0),
                  wall_z0=1, g=(0.0, 0.0, -G0), dt=1e-6, skin=0.1 * rmax, steps=10_000,
                  name=f"settled_bed_{n}", meta={"deposit_stuck": stuck})


def _settled_bed_arrays(seed, n, footprint):
    rng = np.random.default_rng(seed)
    r = rng.uniform(0.8e-3, 1.2e-3, n)
    pos, stuck = bed(n, r, footprint, footprint, rng)
    order = np.argsort(pos[:, 2], kind="stable")  # ids follow height, like a filled bed
    pos = pos[order]; r = r[order]
    # shuffle the storage order so that no code can rely on input sorting
    perm = rng.permutation(n)
    pos = pos[perm]; r = r[perm]
    ids = perm.astype(np.int32)
    return pos, r, ids, stuck


# ----------------------------------------------------------------------------
# Chutes and batches
# ----------------------------------------------------------------------------

def chute_gravity(angle_deg: float = 30.0):
    a = math.radians(angle_deg)
    return (G0 * math.sin(a), 0.0, -G0 * math.cos(a))


def tiled_bed(n_total: int, seed: int = 6) -> System:
    """A settled bed of about n_total spheres made of a periodic bed of
    n_total/4 spheres repeated 2 x 2 in x and y (exact, since the tile is
    periodic); used as one plain system of the same size as a batch."""
    n = max(1, int(round(n_total / 4)))
    fp = 80e-3 * math.sqrt(n / 1e6)
    tile = settled_bed(seed=seed, n=n, footprint=fp)
    xs, rs, ids = [], [], []
    for k, (ox, oy) in enumerate(((0, 0), (1, 0), (0, 1), (1, 1))):
        xs.append(tile.x + np.array([ox * fp, oy * fp, 0.0]))
        rs.append(tile.r)
        ids.append(tile.id.astype(np.int64) + k * n)
    x = np.concatenate(xs); r = np.concatenate(rs); idv = np.concatenate(ids).astype(np.int32)
    m = x.shape[0]
    return System(x=x, v=np.zeros((m, 3)), w=np.zeros((m, 3)), r=r, type=np.zeros(m, np.int32), id=idv,
                  materials=[MAT_A], lo=(0.0, 0.0, 0.0), hi=(2 * fp, 2 * fp, tile.hi[2]), periodic=(1, 1, 0),
                  wall_z0=1, g=(0.0, 0.0, -G0), dt=1e-6, skin=tile.skin, steps=2000, name=f"tiled_bed_{m}")


def _system_from_bed(pos, r, types, materials, Lx, Ly, g, dt, skin, steps, name, alpha, v=None, rng=None):
    n = r.shape[0]
    rmax = float(r.max())
    top = float(pos[:, 2].max()) + 4.0 * rmax
    return System(x=pos, v=np.zeros((n, 3)) if v is None else v, w=np.zeros((n, 3)), r=r, type=types,
                  id=np.arange(n, dtype=np.int32), materials=materials, lo=(0.0, 0.0, 0.0), hi=(Lx, Ly, top),
                  periodic=(1, 1, 0), wall_z0=1, g=g, dt=dt, skin=skin, steps=steps, name=name, alpha=alpha)


def chute_two_level(seed: int = 3, n_fine: int = 500_000, n_coarse: int = 200_000):
    """Two systems of one batch on a periodic 30 degree chute (Sec. 2.3: a fine
    region embedded in a coarse-grain domain):

    * coarse: n_coarse spheres of r = 4 mm (alpha = 4), 1000 x 400 mm footprint;
    * fine:   n_fine spheres of r = 1 mm, 200 x 100 mm footprint.

    Footprints scale with sqrt(n) for smaller test sizes.  The fine particles
    within 10 mm of the fine bed's top face form the coupling shell; their
    indices are in ``meta['shell']`` (the shell receives an external-force array
    that stays zero until the coupling controllers exist).  Both use dt = 1e-6 s.
    """
    ss = np.random.SeedSequence(seed)
    kids = ss.spawn(2)
    g = chute_gravity(30.0)
    Lc = (1000e-3 * math.sqrt(n_coarse / 200_000), 400e-3 * math.sqrt(n_coarse / 200_000))
    Lf = (200e-3 * math.sqrt(n_fine / 500_000), 100e-3 * math.sqrt(n_fine / 500_000))
    jobs = [(n_coarse, (4.0, 0.0), Lc[0], Lc[1], 0.01, kids[0]), (n_fine, (1.0, 0.0), Lf[0], Lf[1], 0.01, kids[1])]
    (pc, rc, _), (pf, rf, _) = _cached_beds(f"chute{seed}", jobs)
    coarse = _system_from_bed(pc, rc, np.zeros(n_coarse, np.int32), [MAT_A], Lc[0], Lc[1], g, 1e-6,
                              0.1 * 4e-3, 5000, "chute_coarse", 4.0)
    fine = _system_from_bed(pf, rf, np.zeros(n_fine, np.int32), [MAT_A], Lf[0], Lf[1], g, 1e-6, 0.1e-3, 5000,
                            "chute_fine", 1.0)
    fine.meta["shell"] = np.nonzero(pf[:, 2] > pf[:, 2].max() - 10e-3)[0].astype(np.int64)
    return [coarse, fine]


def chute_coupling(coarse: System, fine: System, shell: float = 10e-3, interval_steps: int = 15) -> dict:
    """Coupling geometry of the two-level chute (plain numbers, no physics).

    The fine region is the fine bed's footprint at the origin of the coarse
    chute, from the floor to its initial top z_f.  The transition layer is the
    shell of thickness `shell` below z_f, one layer of cells of about 50 mm
    (the paper's cells are three to ten coarse diameters); the boundary face is
    z = z_f with the normal -z into the fine region.  The coarse spheres inside
    the fine region below the shell are corrected on cells of the same footprint
    and about 35 mm height.  Coupling every `interval_steps` fine steps (the
    paper updates its controller every 15 steps)."""
    Lx, Ly = fine.hi[0] - fine.lo[0], fine.hi[1] - fine.lo[1]
    zf = float(fine.x[:, 2].max())
    nx, ny = max(1, int(round(Lx / 50e-3))), max(1, int(round(Ly / 50e-3)))
    hx, hy = Lx / nx, Ly / ny
    nz = max(1, int(round((zf - shell) / 35e-3)))
    return {"pi_grid": ((0.0, 0.0, zf - shell), (hx, hy, shell), (nx, ny, 1)),
            "p_grid": ((0.0, 0.0, 0.0), (hx, hy, (zf - shell) / nz), (nx, ny, nz)),
            "normal": (0.0, 0.0, -1.0), "face": -zf, "fade": 1.5, "kp": 1.0, "ki": 200.0, "kp_coarse": 2000.0,
            "interval_steps": interval_steps}


def _deposit_job(args):
    """Worker: one bed from its own seed (used to build batches in parallel)."""
    n, r_args, Lx, Ly, strain, child = args
    rng = np.random.default_rng(child)
    alpha, p = r_args
    r = alpha * 1e-3 * rng.uniform(1.0 - p, 1.0 + p, n)
    pos, stuck = bed(n, r, Lx, Ly, rng, strain_bottom=strain)
    return pos, r, stuck


def _cached_beds(tag: str, jobs, workers: int | None = None):
    """Run deposition jobs (in worker processes), caching each result on disk."""
    out = [None] * len(jobs)
    todo = []
    paths = []
    for k, job in enumerate(jobs):
        path = _cache_path(f"{tag}_{k}_{job[0]}_{job[1]!r}_{job[2]!r}_{job[3]!r}_{job[4]!r}_{job[5].entropy}_{job[5].spawn_key}")
        paths.append(path)
        if path and os.path.exists(path):
            with np.load(path, allow_pickle=False) as z:
                out[k] = (z["x"], z["r"], int(z["stuck"]))
        else:
            todo.append(k)
    if todo:
        nw = workers or min(16, os.cpu_count() or 1, len(todo))
        if nw > 1:
            import concurrent.futures as cf
            import multiprocessing as mp
            with cf.ProcessPoolExecutor(max_workers=nw, mp_context=mp.get_context("fork")) as ex:
                res = list(ex.map(_deposit_job, [jobs[k] for k in todo]))
        else:
            res = [_deposit_job(jobs[k]) for k in todo]
        for k, rr in zip(todo, res):
            out[k] = rr
            if paths[k]:
                tmp = paths[k] + f".{os.getpid()}.tmp.npz"
                np.savez(tmp, x=rr[0], r=rr[1], stuck=rr[2])
                os.replace(tmp, paths[k])
    return out


def batch_systems(seed: int = 4, count: int = 64, n_lo: int = 5_000, n_hi: int = 200_000,
                  dt_scaled: bool = True, scale: float = 1.0):
    """``count`` independent beds: N log-uniform in [n_lo, n_hi], alpha in {1,2,4,8},
    r = alpha U[1-p, 1+p] mm with p ~ U(0, 0.2), footprint aspect U(1, 4), bed
    depth about 20 alpha mm; dt = alpha * 1e-6 s when ``dt_scaled`` (Sec. 3: the
    time step may grow with the particle size).  ``scale`` multiplies every N
    (for small test batches).  The per-system draws come from ``seed``; each bed
    is deposited from its own child seed, so beds can be built in parallel."""
    ss = np.random.SeedSequence(seed)
    rng = np.random.default_rng(ss)
    children = ss.spawn(count)
    params = []
    for s in range(count):
        n = max(8, int(round(scale * math.exp(rng.uniform(math.log(n_lo), math.log(n_hi))))))
        alpha = float(rng.choice([1, 2, 4, 8]))
        p = rng.uniform(0.0, 0.2)
        aspect = rng.uniform(1.0, 4.0)
        depth = 20e-3 * alpha
        mean_r3 = (alpha * 1e-3) ** 3 * (1.0 + p * p)          # E[r^3] for r = alpha U[1-p, 1+p]
        area = n * 4.0 / 3.0 * math.pi * mean_r3 / (0.58 * depth)
        Lx = math.sqrt(area * aspect)
        Ly = area / Lx
        rmax = alpha * 1e-3 * (1.0 + p)
        cut = 2.0 * rmax * 1.1
        Lx = max(Lx, 3.0 * cut); Ly = max(Ly, 3.0 * cut)
        params.append((n, alpha, p, Lx, Ly))
    jobs = [(n, (alpha, p), Lx, Ly, 0.005, children[k]) for k, (n, alpha, p, Lx, Ly) in enumerate(params)]
    beds = _cached_beds(f"batch{seed}", jobs)
    systems = []
    for k, ((n, alpha, p, Lx, Ly), (pos, r, _)) in enumerate(zip(params, beds)):
        dt = alpha * 1e-6 if dt_scaled else 1e-6
        rmax = float(r.max())
        systems.append(_system_from_bed(pos, r, np.zeros(n, np.int32), [MAT_A], Lx, Ly, (0.0, 0.0, -G0), dt,
                                        0.1 * rmax, 2000, f"batch_{k}", alpha))
    return systems


def chute_adjoint(seed: int = 5, n: int = 50_000, Lx: float = 100e-3, Ly: float = 50e-3) -> System:
    """Two-type chute (50/50 by seeded draw), r ~ U[0.9, 1.1] mm, 30 degrees.

    The initial velocity is a synthetic sheared flow profile
    v_x(z) = U (1 - (1 - z/H)^(3/2)) with U = 0.2 m/s plus N(0, 0.01 m/s) noise.
    """
    rng = np.random.default_rng(seed)
    r = rng.uniform(0.9e-3, 1.1e-3, n)
    pos, _ = bed(n, r, Lx, Ly, rng, strain_bottom=0.005)
    types = (rng.uniform(size=n) < 0.5).astype(np.int32)
    H = float(pos[:, 2].max())
    v = rng.normal(0.0, 0.01, (n, 3))
    v[:, 0] += 0.2 * (1.0 - np.clip(1.0 - pos[:, 2] / H, 0.0, 1.0) ** 1.5)
    sysm = _system_from_bed(pos, r, types, [MAT_A, MAT_B], Lx, Ly, chute_gravity(30.0), 1e-6, 0.1 * 1.1e-3,
                            200, "chute_adjoint", 1.0, v=v)
    sysm.meta["H0"] = H
    return sysm


# ----------------------------------------------------------------------------
# Insertion events at the boundary of a fine region
# ----------------------------------------------------------------------------

NFIELD_ROWS = 16          # rows of a cell-fields array: count, mass, momentum (3), volume, ...
ROW_MASS, ROW_MOM = 1, 2


def exchange_inputs(system: System, zf: float, ncand: int, seed: int, cells=(2, 2), slab: float = 4e-3,
                    depth: float = 3e-3, interval: float = 15e-6, inflow_mass: float = 2e-3,
                    inflow_speed: float = 0.4, budget_spheres: float = 1.0) -> dict:
    """Inputs of one insertion event of a fine bed whose region is z <= zf
    (boundary face z = zf, normal -z into the region): a grid of cells x cells
    boundary cells over the footprint; the coarse level's fields on them (mass
    inflow_mass * U[0.5, 1.5] per cell, momentum of that mass moving at
    inflow_speed * U[0.5, 1.5] downwards plus N(0, 0.1 inflow_speed) sideways;
    one cell in four flows outwards); the starting budget (U[0, 1] sphere
    masses, times budget_spheres); ncand candidates uniform in the slab zf - depth < z < zf of a
    uniformly drawn cell, radii uniform over the system's radius range, type 0."""
    rng = np.random.default_rng(seed)
    nx, ny = cells
    ncell = nx * ny
    Lx, Ly = system.hi[0] - system.lo[0], system.hi[1] - system.lo[1]
    fields = np.zeros((NFIELD_ROWS, ncell))
    mass = inflow_mass * rng.uniform(0.5, 1.5, ncell)
    speed = inflow_speed * rng.uniform(0.5, 1.5, ncell)
    sign = np.where(np.arange(ncell) % 4 == 3, 1.0, -1.0)
    fields[ROW_MASS] = mass
    fields[ROW_MOM] = mass * rng.normal(0.0, 0.1 * inflow_speed, ncell)
    fields[ROW_MOM + 1] = mass * rng.normal(0.0, 0.1 * inflow_speed, ncell)
    fields[ROW_MOM + 2] = mass * speed * sign
    rmin, rmax = float(system.r.min()), float(system.r.max())
    rho = system.materials[0].rho
    m_sphere = 4.0 / 3.0 * math.pi * rho * ((rmin + rmax) / 2) ** 3
    budget = rng.uniform(0.0, 1.0, ncell) * m_sphere * budget_spheres
    cell = rng.integers(0, ncell, ncand)
    cx, cy = cell % nx, cell // nx
    x = np.column_stack([(cx + rng.uniform(0.0, 1.0, ncand)) * Lx / nx + system.lo[0],
                         (cy + rng.uniform(0.0, 1.0, ncand)) * Ly / ny + system.lo[1],
                         zf - depth * rng.uniform(0.0, 1.0, ncand)])
    for a in range(2):                       # keep positions inside [lo, hi) on the periodic axes
        L = system.hi[a] - system.lo[a]
        x[:, a] = np.where(x[:, a] >= system.hi[a], x[:, a] - L, x[:, a])
    r = rng.uniform(rmin, rmax, ncand)
    return {"nrm": (0.0, 0.0, -1.0), "face": -zf, "slab": slab, "interval": interval, "ncell": ncell,
            "fields": fields, "budget": budget, "cand_x": x, "cand_r": r,
            "cand_type": np.zeros(ncand, np.int32), "cand_cell": cell.astype(np.int32)}


# ----------------------------------------------------------------------------
# Silo (Sec. 3: filling and discharge)
# ----------------------------------------------------------------------------

SURF_CYLINDER, SURF_CONE, SURF_DISK, SURF_RING = 1, 2, 3, 4


MAT_SILO = Material(E=2.5e7, nu=0.25, rho=1000.0, e=0.5, mu=0.2)   # the paper's silo table
MU_WALL_SILO = 0.175                                                 # its particle-wall friction


def silo_surfaces(scale: float = 1.0, open_orifice: bool = False, mu_wall: float = -1.0) -> list:
    """Wall surfaces of the paper's silo scaled by `scale`: 40 cm high, the top
    half a cylinder of 27 cm diameter, the lower half a cone narrowing to a
    4 cm orifice at z = 0, closed by a plug (a disk) until the orifice opens;
    the opened orifice's rim is an edge (a ring).  Records (kind, enabled,
    axis x, axis y, z0, z1, r0, r1, mu), axis through the origin; mu the
    particle-wall friction (< 0: the particle's own)."""
    R, Ro, Hc, H = 0.135 * scale, 0.02 * scale, 0.20 * scale, 0.40 * scale
    return [(SURF_CONE, 1, 0.0, 0.0, 0.0, Hc, Ro, R, mu_wall),
            (SURF_CYLINDER, 1, 0.0, 0.0, Hc, H, R, 0.0, mu_wall),
            (SURF_DISK, 0 if open_orifice else 1, 0.0, 0.0, 0.0, 0.0, Ro, 0.0, mu_wall),
            (SURF_RING, 1 if open_orifice else 0, 0.0, 0.0, 0.0, 0.0, Ro, 0.0, mu_wall)]


def silo_radius_at(z: np.ndarray, scale: float = 1.0) -> np.ndarray:
    """Inner radius of the silo at height z (cone below half height, cylinder above)."""
    R, Ro, Hc = 0.135 * scale, 0.02 * scale, 0.20 * scale
    return np.where(z < Hc, Ro + (R - Ro) * np.clip(z, 0.0, Hc) / Hc, R)


def silo_system(scale: float = 1.0, r: float = 1.4e-3, spread: float = 0.0, fill: float = 1.0, seed: int = 9,
                speed: float = 0.0, mat: Material = MAT_A, dt: float = 1e-6, mu_wall: float = -1.0) -> System:
    """Spheres of radius r (uniform in r (1 +- spread)) on a jittered cubic
    lattice (spacing 2.1 r_max) filling the silo from the plug up to the
    fraction `fill` of its height, each at least 1.05 r_max inside the walls;
    velocities N(0, speed) per component.  Open box around the silo (no
    periodic axis, no flat wall), gravity -z; the grid reaches 5 cm (scaled)
    below the orifice, where discharged spheres are removed.  The paper's
    reference silo holds 187,504 spheres of 2.8 mm diameter (r = 1.4 mm)."""
    rng = np.random.default_rng(seed)
    R, H = 0.135 * scale, 0.40 * scale
    rmax = r * (1.0 + spread)
    a = 2.1 * rmax
    zs = np.arange(1.05 * rmax, H * fill - rmax, a)
    xs = np.arange(-R, R + a / 2, a)
    X, Y, Z = np.meshgrid(xs, xs, zs, indexing="ij")
    pos = np.column_stack([X.ravel(), Y.ravel(), Z.ravel()])
    rho = np.hypot(pos[:, 0], pos[:, 1])
    # perpendicular clearance from the cone's slanted side: (R(z) - rho) cos(theta)
    cos_t = 0.2 / math.hypot(0.115, 0.2)
    clear = np.where(pos[:, 2] < 0.20 * scale, 1.05 * rmax / cos_t, 1.05 * rmax)
    inside = rho <= silo_radius_at(pos[:, 2], scale) - clear
    pos = pos[inside]
    pos += rng.uniform(-0.02 * rmax, 0.02 * rmax, pos.shape)
    n = pos.shape[0]
    radii = r * (1.0 + spread * rng.uniform(-1.0, 1.0, n))
    v = rng.normal(0.0, speed, (n, 3)) if speed > 0 else np.zeros((n, 3))
    lo = (-R - 4 * rmax, -R - 4 * rmax, -0.05 * scale)
    hi = (R + 4 * rmax, R + 4 * rmax, H + 4 * rmax)
    s = System(x=pos, v=v, w=np.zeros((n, 3)), r=radii, type=np.zeros(n, np.int32), id=np.arange(n, dtype=np.int32),
               materials=[mat], lo=lo, hi=hi, periodic=(0, 0, 0), wall_z0=0, g=(0.0, 0.0, -G0), dt=dt,
               skin=0.1 * rmax, steps=0, name=f"silo_{n}", alpha=1.0)
    s.meta["surfaces"] = silo_surfaces(scale, mu_wall=mu_wall)
    s.meta["mu_wall"] = mu_wall
    s.meta["scale"] = scale
    return s
