"""ctypes binding of the FP64 CPU oracle (``dem_oracle.cpp``).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check of the entry
module and the CPU-baseline leg of the benchmark may import this module.  The
GPU library neither imports nor links it, and nothing here is shared with it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dem_oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)


class OrcConfig(ctypes.Structure):
    _fields_ = [("ntypes", ctypes.c_int),
                ("E", ctypes.c_double * 4), ("nu", ctypes.c_double * 4), ("rho", ctypes.c_double * 4),
                ("e", ctypes.c_double * 4), ("mu", ctypes.c_double * 4),
                ("dt", ctypes.c_double), ("g", ctypes.c_double * 3),
                ("lo", ctypes.c_double * 3), ("hi", ctypes.c_double * 3),
                ("periodic", ctypes.c_int * 3), ("wall_z0", ctypes.c_int)]


def compile_to(src: str, out: str) -> str:
    """g++ with the oracle's flags (no FMA contraction, no -march)."""
    tmp = out + ".tmp"
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", src,
                           "-o", tmp])
    os.replace(tmp, out)
    return out


def build(force: bool = False) -> str:
    """Compile the oracle (only when the source is newer than the library)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        compile_to(_SRC, _LIB)
    return _LIB


_libs = {}


def lib(path: str | None = None):
    """The oracle library (default: the one built from dem_oracle.cpp).  Tests
    of the pins themselves may load a modified copy compiled elsewhere."""
    key = path or _LIB
    if key not in _libs:
        L = ctypes.CDLL(build() if path is None else path)
        vp = ctypes.c_void_p
        L.orc_new.restype = vp
        L.orc_new.argtypes = [ctypes.POINTER(OrcConfig), ctypes.c_int, _dp, _dp, _dp, _dp, _ip, _ip]
        L.orc_tan_new.restype = vp
        L.orc_tan_new.argtypes = L.orc_new.argtypes
        for name in ("orc_free", "orc_tan_free"):
            getattr(L, name).argtypes = [vp]
        L.orc_get.argtypes = [vp, _dp, _dp, _dp, _dp, _dp]
        L.orc_set.argtypes = [vp, _dp, _dp, _dp, _dp, _dp]
        L.orc_get_mass.argtypes = [vp, _dp, _dp]
        L.orc_forces.argtypes = [vp, ctypes.c_int]
        L.orc_step.argtypes = [vp, ctypes.c_int]
        L.orc_kick.argtypes = [vp]
        L.orc_drift.argtypes = [vp]
        L.orc_history.restype = ctypes.c_long
        L.orc_history.argtypes = [vp, _ip, _ip, _dp, ctypes.c_long]
        L.orc_set_history.argtypes = [vp, ctypes.c_long, _ip, _ip, _dp]
        L.orc_wall_history.restype = ctypes.c_long
        L.orc_wall_history.argtypes = [vp, _ip, _dp, ctypes.c_long]
        L.orc_set_wall_history.argtypes = [vp, ctypes.c_long, _ip, _dp]
        L.orc_pairs.restype = ctypes.c_long
        L.orc_pairs.argtypes = [vp, ctypes.c_double, ctypes.c_int, _ip, _ip, ctypes.c_long]
        L.orc_records.restype = ctypes.c_long
        L.orc_records.argtypes = [vp, _ip, _ip, _dp, _dp, _dp, _dp, _dp, ctypes.c_long]
        L.orc_step_parallel.restype = ctypes.c_int
        L.orc_step_parallel.argtypes = [vp, ctypes.c_int, _dp]
        L.orc_set_external.argtypes = [vp, _dp]
        L.orc_set_surfaces.argtypes = [vp, ctypes.c_int, _dp]
        L.orc_surface_contact.restype = ctypes.c_int
        L.orc_surface_contact.argtypes = [_dp, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                          _dp]
        L.orc_surface_history.restype = ctypes.c_long
        L.orc_surface_history.argtypes = [vp, _ip, _ip, _dp, ctypes.c_long]
        L.orc_set_surface_history.argtypes = [vp, ctypes.c_long, _ip, _ip, _dp]
        L.orc_pair_forces.restype = ctypes.c_long
        L.orc_pair_forces.argtypes = [vp, _ip, _ip, _dp, _dp, ctypes.c_long]
        L.orc_tan_forces.argtypes = [vp, ctypes.c_int]
        L.orc_tan_step.argtypes = [vp, ctypes.c_int]
        L.orc_tan_get.argtypes = [vp, _dp, _dp, _dp, _dp]
        L.orc_tan_get_ext.argtypes = [vp, ctypes.c_int, _dp, _dp]
        L.orc_tan_seed_state.argtypes = [vp, ctypes.c_int, _dp, _dp, _dp]
        _libs[key] = L
    return _libs[key]


def _d(a):
    return None if a is None else a.ctypes.data_as(_dp)


def _i(a):
    return None if a is None else a.ctypes.data_as(_ip)


def make_config(system) -> OrcConfig:
    """Oracle configuration from a workload ``System`` (materials, box, dt, gravity)."""
    c = OrcConfig()
    mats = system.materials
    c.ntypes = len(mats)
    for t, m in enumerate(mats):
        c.E[t] = m.E; c.nu[t] = m.nu; c.rho[t] = m.rho; c.e[t] = m.e; c.mu[t] = m.mu
    c.dt = system.dt
    for d in range(3):
        c.g[d] = system.g[d]; c.lo[d] = system.lo[d]; c.hi[d] = system.hi[d]
        c.periodic[d] = int(system.periodic[d])
    c.wall_z0 = int(system.wall_z0)
    return c


class Oracle:
    """One simulated system in the oracle; arrays are (n, 3) in input order."""

    def __init__(self, system, tangent: bool = False, lib_path: str | None = None):
        self.L = lib(lib_path)
        self.n = system.n
        self.tangent = tangent
        self.cfg = make_config(system)
        arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (system.x, system.v, system.w, system.r)]
        ty = np.ascontiguousarray(system.type, dtype=np.int32)
        ids = np.ascontiguousarray(system.id, dtype=np.int32)
        new = self.L.orc_tan_new if tangent else self.L.orc_new
        self.h = new(ctypes.byref(self.cfg), self.n, *[_d(a) for a in arrs], _i(ty), _i(ids))
        self.ids = ids.copy()

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            (self.L.orc_tan_free if self.tangent else self.L.orc_free)(h)
            self.h = None

    # ---- double-precision handle
    def state(self):
        out = {k: np.empty((self.n, 3)) for k in ("x", "v", "w", "f", "t")}
        self.L.orc_get(self.h, *[_d(out[k]) for k in ("x", "v", "w", "f", "t")])
        return out

    def set_state(self, x=None, v=None, w=None, f=None, t=None):
        a = [None if q is None else np.ascontiguousarray(q, dtype=np.float64) for q in (x, v, w, f, t)]
        self.L.orc_set(self.h, *[_d(q) for q in a])

    def mass(self):
        m = np.empty(self.n); inertia = np.empty(self.n)
        self.L.orc_get_mass(self.h, _d(m), _d(inertia))
        return m, inertia

    def forces(self, update_history: bool = False):
        self.L.orc_forces(self.h, int(update_history))

    def step(self, nsteps: int = 1):
        self.L.orc_step(self.h, int(nsteps))

    def step_parallel(self, nsteps: int = 1):
        """The same steps on all host cores (OpenMP gather form, for timing);
        returns (threads used, seconds of the step loop)."""
        sec = ctypes.c_double(0.0)
        th = int(self.L.orc_step_parallel(self.h, int(nsteps), ctypes.byref(sec)))
        if th < 0:
            raise ValueError("the all-cores form takes no wall surfaces")
        return th, sec.value

    def kick(self):
        self.L.orc_kick(self.h)

    def drift(self):
        self.L.orc_drift(self.h)

    def integrate_vjp(self, phase: int, xb, vb, wb) -> dict:
        """Reverse mode of one half of the velocity-Verlet step (Eq. (1)-(2)):
        phase 0 is kick() then drift() (v' = v + dt/2 f/m, w' = w + dt/2 t/I,
        x' = x + dt v' wrapped into the box), phase 1 is kick().  Given the
        adjoints of the outputs x', v', w' ((n, 3) in input order), returns
        those of the inputs x, v, w, f, t.  Written from the map itself: it is
        linear in its inputs and the wrap is a shift by a box length, so
        x_in = x', v_in = v' + dt x' (phase 0) or v' (phase 1), w_in = w',
        f_in = dt/2 v_in / m, t_in = dt/2 w' / I."""
        m, inertia = self.mass()
        dt = self.cfg.dt
        xb, vb, wb = (np.asarray(q, dtype=np.float64) for q in (xb, vb, wb))
        uv = vb + dt * xb if phase == 0 else vb.copy()
        return {"x": xb.copy(), "v": uv, "w": wb.copy(), "f": 0.5 * dt * uv / m[:, None],
                "t": 0.5 * dt * wb / inertia[:, None]}

    def history(self):
        """Unordered pair history: (id_lo, id_hi, xi (k,3)) with xi seen from id_lo."""
        k = self.L.orc_history(self.h, None, None, None, 0)
        lo = np.empty(k, np.int32); hi = np.empty(k, np.int32); xi = np.empty((k, 3))
        self.L.orc_history(self.h, _i(lo), _i(hi), _d(xi), k)
        return lo, hi, xi

    def set_history(self, lo, hi, xi):
        lo = np.ascontiguousarray(lo, np.int32); hi = np.ascontiguousarray(hi, np.int32)
        xi = np.ascontiguousarray(xi, np.float64)
        self.L.orc_set_history(self.h, lo.shape[0], _i(lo), _i(hi), _d(xi))

    def wall_history(self):
        k = self.L.orc_wall_history(self.h, None, None, 0)
        ids = np.empty(k, np.int32); xi = np.empty((k, 3))
        self.L.orc_wall_history(self.h, _i(ids), _d(xi), k)
        return ids, xi

    def set_wall_history(self, ids, xi):
        ids = np.ascontiguousarray(ids, np.int32); xi = np.ascontiguousarray(xi, np.float64)
        self.L.orc_set_wall_history(self.h, ids.shape[0], _i(ids), _d(xi))

    def pairs(self, extra: float = 0.0, brute: bool = False):
        """Unordered id pairs (lo < hi, ascending) with d^2 < (r_i + r_j + extra)^2."""
        k = self.L.orc_pairs(self.h, float(extra), int(brute), None, None, 0)
        lo = np.empty(k, np.int32); hi = np.empty(k, np.int32)
        self.L.orc_pairs(self.h, float(extra), int(brute), _i(lo), _i(hi), k)
        return lo, hi

    def records(self):
        """Contacts of the last force evaluation: ids (hi = -1: wall), |f_n|, |F_ij|,
        |F_t|, the Coulomb cap mu |f_n| and the normal part |F_t . n|."""
        k = self.L.orc_records(self.h, None, None, None, None, None, None, None, 0)
        lo = np.empty(k, np.int32); hi = np.empty(k, np.int32)
        fn, fm, ftm, cap, ftn = (np.empty(k) for _ in range(5))
        self.L.orc_records(self.h, _i(lo), _i(hi), _d(fn), _d(fm), _d(ftm), _d(cap), _d(ftn), k)
        return dict(lo=lo, hi=hi, fn=fn, fmag=fm, ftmag=ftm, cap=cap, ftn=ftn)

    def set_surfaces(self, surfaces):
        """Static wall surfaces: records (kind, enabled, cx, cy, z0, z1, r0, r1[, mu])
        (kinds 1 cylinder, 2 cone, 3 disk, 4 ring; mu < 0 or absent: the particle's friction)."""
        d = np.ascontiguousarray(_surface_records(surfaces))
        self.L.orc_set_surfaces(self.h, d.shape[0], _d(d))

    def surface_history(self):
        k = self.L.orc_surface_history(self.h, None, None, None, 0)
        ids = np.empty(k, np.int32); ks = np.empty(k, np.int32); xi = np.empty((k, 3))
        self.L.orc_surface_history(self.h, _i(ids), _i(ks), _d(xi), k)
        return ids, ks, xi

    def set_surface_history(self, ids, ks, xi):
        ids = np.ascontiguousarray(ids, np.int32); ks = np.ascontiguousarray(ks, np.int32)
        xi = np.ascontiguousarray(xi, np.float64).reshape(-1, 3)
        self.L.orc_set_surface_history(self.h, ids.shape[0], _i(ids), _i(ks), _d(xi))

    def set_external(self, f=None):
        """External force per particle ((n,3), input order), added after the wall
        term at every force evaluation; None removes it."""
        a = None if f is None else np.ascontiguousarray(f, dtype=np.float64).reshape(self.n, 3)
        self._fext = a
        self.L.orc_set_external(self.h, _d(a))

    def pair_forces(self):
        """Contact forces of the current state (no history update): ids lo < hi,
        branch vectors d = x_lo - x_hi (k,3) and forces on lo (k,3)."""
        k = self.L.orc_pair_forces(self.h, None, None, None, None, 0)
        lo = np.empty(k, np.int32); hi = np.empty(k, np.int32); d = np.empty((k, 3)); f = np.empty((k, 3))
        self.L.orc_pair_forces(self.h, _i(lo), _i(hi), _d(d), _d(f), k)
        return lo, hi, d, f

    # ---- forward-mode handle
    def tan_forces(self, update_history: bool = False):
        self.L.orc_tan_forces(self.h, int(update_history))

    def tan_step(self, nsteps: int = 1):
        self.L.orc_tan_step(self.h, int(nsteps))

    def tan_state(self):
        """Values (n,3) and tangents (n,3,6) of x and v; directions E0, E1, e0, e1, mu0, mu1."""
        xv = np.empty((self.n, 3)); vv = np.empty((self.n, 3))
        xt = np.empty((self.n, 3, 6)); vt = np.empty((self.n, 3, 6))
        self.L.orc_tan_get(self.h, _d(xv), _d(xt), _d(vv), _d(vt))
        return xv, xt, vv, vt

    def tan_seed_state(self, k: int, dx=None, dv=None, dw=None):
        """Make tangent direction k the derivative along an initial-state
        perturbation (dx, dv, dw: (n,3) in input order) instead of a parameter."""
        a = [None if q is None else np.ascontiguousarray(q, dtype=np.float64) for q in (dx, dv, dw)]
        self.L.orc_tan_seed_state(self.h, int(k), *[_d(q) for q in a])

    def tan_vector(self, name: str):
        """Value (n,3) and tangent (n,3,6) of one of x, v, w, f, t."""
        which = ("x", "v", "w", "f", "t").index(name)
        val = np.empty((self.n, 3)); tan = np.empty((self.n, 3, 6))
        self.L.orc_tan_get_ext(self.h, which, _d(val), _d(tan))
        return val, tan


def _surface_records(surfaces):
    rows = [list(map(float, q)) + ([] if len(q) > 8 else [-1.0]) for q in surfaces]
    return np.asarray(rows, np.float64).reshape(-1, 9)


def surface_contact(record, x, y, z, r, lib_path: str | None = None):
    """The oracle's contact geometry of one sphere with one surface record:
    (distance, normal) or None when not in contact."""
    d = np.ascontiguousarray(_surface_records([record]).reshape(9))
    out = np.zeros(4)
    if not lib(lib_path).orc_surface_contact(_d(d), float(x), float(y), float(z), float(r), _d(out)):
        return None
    return float(out[0]), out[1:].copy()
