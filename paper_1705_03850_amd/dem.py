"""ctypes binding of libdem.so (include/dem.h).

Argument marshalling only: every step of the DEM pipeline runs in the HIP
kernels of ``libdem.so``.  PyTorch provides the device memory (particle
arrays and the one workspace buffer) and the stream.  Loading fails loudly
when the library has not been built; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdem.so")

DEM_OK, DEM_ERR_ARG, DEM_ERR_CAPACITY, DEM_ERR_DOMAIN, DEM_ERR_NONFINITE, DEM_ERR_HIP, DEM_ERR_STATE = range(7)
ERROR_NAMES = {1: "DEM_ERR_ARG", 2: "DEM_ERR_CAPACITY", 3: "DEM_ERR_DOMAIN", 4: "DEM_ERR_NONFINITE",
               5: "DEM_ERR_HIP", 6: "DEM_ERR_STATE"}
MAX_TYPES = 4


class DemError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


class Material(ctypes.Structure):
    _fields_ = [("E", ctypes.c_double), ("nu", ctypes.c_double), ("rho", ctypes.c_double),
                ("e", ctypes.c_double), ("mu", ctypes.c_double)]


class Config(ctypes.Structure):
    _fields_ = [("ntypes", ctypes.c_int32), ("mat", Material * MAX_TYPES), ("dt", ctypes.c_double),
                ("g", ctypes.c_double * 3), ("lo", ctypes.c_double * 3), ("hi", ctypes.c_double * 3),
                ("periodic", ctypes.c_int32 * 3), ("wall_z0", ctypes.c_int32), ("skin", ctypes.c_double),
                ("cell", ctypes.c_double), ("r_max", ctypes.c_double), ("n", ctypes.c_int64),
                ("k_max", ctypes.c_int32), ("block", ctypes.c_int32), ("n_max", ctypes.c_int64),
                ("n_surf", ctypes.c_int32), ("pad", ctypes.c_int32)]


class Surface(ctypes.Structure):
    """dem_surface: kind (1 cylinder, 2 cone, 3 disk, 4 ring), enabled, axis (x, y),
    heights z0, z1, radii r0, r1 and the contact friction mu (< 0: the particle's)."""
    _fields_ = [("kind", ctypes.c_int32), ("enabled", ctypes.c_int32), ("axis", ctypes.c_double * 2),
                ("z0", ctypes.c_double), ("z1", ctypes.c_double), ("r0", ctypes.c_double), ("r1", ctypes.c_double),
                ("mu", ctypes.c_double)]


def make_surfaces(records):
    """dem_surface array from records (kind, enabled, cx, cy, z0, z1, r0, r1[, mu])."""
    arr = (Surface * max(1, len(records)))()
    for k, q in enumerate(records):
        arr[k].kind, arr[k].enabled = int(q[0]), int(q[1])
        arr[k].axis[0], arr[k].axis[1] = float(q[2]), float(q[3])
        arr[k].z0, arr[k].z1, arr[k].r0, arr[k].r1 = float(q[4]), float(q[5]), float(q[6]), float(q[7])
        arr[k].mu = float(q[8]) if len(q) > 8 else -1.0
    return arr


class State(ctypes.Structure):
    _fields_ = [(k, ctypes.c_void_p) for k in ("x", "v", "w", "f", "t", "r", "type", "id")]


class Grid(ctypes.Structure):
    """dem_grid: cells (lo, h, n) in the coordinates of system `sys`."""
    _fields_ = [("lo", ctypes.c_double * 3), ("h", ctypes.c_double * 3), ("n", ctypes.c_int32 * 3),
                ("sys", ctypes.c_int32)]


class PIParams(ctypes.Structure):
    _fields_ = [("grid", Grid), ("nrm", ctypes.c_double * 3), ("face", ctypes.c_double), ("kp", ctypes.c_double),
                ("ki", ctypes.c_double), ("interval", ctypes.c_double), ("fade", ctypes.c_double)]


class PParams(ctypes.Structure):
    _fields_ = [("grid", Grid), ("kp", ctypes.c_double), ("mass_flow", ctypes.c_int32)]


class CouplingPlan(ctypes.Structure):
    """dem_coupling_plan: one coupling interval (fields, PI and P controllers,
    an optional running sum of fields) repeated by dem_step_coupled."""
    _fields_ = [("pi", PIParams), ("pi_setpoint_sys", ctypes.c_int32), ("p_target_sys", ctypes.c_int32),
                ("p", PParams), ("pi_fine", ctypes.c_void_p), ("pi_coarse", ctypes.c_void_p),
                ("p_fine", ctypes.c_void_p), ("p_coarse", ctypes.c_void_p), ("integral", ctypes.c_void_p),
                ("u", ctypes.c_void_p), ("sum_grid", Grid), ("sum", ctypes.c_void_p), ("sum_tmp", ctypes.c_void_p),
                ("interval_steps", ctypes.c_int64), ("group", ctypes.c_int32), ("pad", ctypes.c_int32)]


class ExchangeParams(ctypes.Structure):
    """dem_exchange_params: boundary face (region x . nrm >= face), inflow slab
    and interval, number of boundary cells, an optional outlet half-space
    (region also x . out_nrm >= out_face; out_nrm = 0: none)."""
    _fields_ = [("nrm", ctypes.c_double * 3), ("face", ctypes.c_double), ("slab", ctypes.c_double),
                ("interval", ctypes.c_double), ("ncell", ctypes.c_int64), ("out_nrm", ctypes.c_double * 3),
                ("out_face", ctypes.c_double)]


# rows of a fields array (dem.h: DEM_F_*)
F_COUNT, F_MASS, F_MOM, F_VOLUME, F_VMAX, F_STRESS, NFIELDS = 0, 1, 2, 5, 6, 7, 16


def make_grid(lo, h, n, sys: int = 0) -> Grid:
    g = Grid()
    for a in range(3):
        g.lo[a], g.h[a], g.n[a] = float(lo[a]), float(h[a]), int(n[a])
    g.sys = int(sys)
    return g


_lib = None
_SYMBOLS = ["dem_workspace_size", "dem_batch_workspace_size", "dem_init", "dem_batch_init", "dem_init_noalloc",
            "dem_reset", "dem_bin",
            "dem_neighbors", "dem_forces", "dem_integrate", "dem_step", "dem_declare_forces", "dem_set_step_options", "dem_set_launch", "dem_check",
            "dem_stats", "dem_set_timing", "dem_kernel_times", "dem_export_neighbors", "dem_export_contacts", "dem_export_wall", "dem_import_history",
            "dem_last_error", "dem_destroy", "dem_set_materials", "dem_adjoint_workspace_size", "dem_adjoint_init",
            "dem_rollout_forward", "dem_rollout_backward", "dem_forces_vjp", "dem_integrate_vjp", "dem_adjoint_set_lanes", "dem_adjoint_info",
            "dem_adjoint_destroy", "dem_cell_fields", "dem_cell_mass_fields", "dem_pi_control", "dem_p_control", "dem_set_external_force",
            "dem_set_multirate", "dem_exchange", "dem_live_count", "dem_set_surfaces", "dem_export_surface_history",
            "dem_import_surface_history", "dem_step_coupled"]


def load(path: str = LIB_PATH):
    """Load libdem.so and declare its C signatures (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run __graft_entry__.build() or paper_1705_03850_amd/build.py")
    try:
        # the library must bind to the HIP runtime that PyTorch loads (it ships its own):
        # load PyTorch first so that the runtime is already resolved
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(path)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    P = ctypes.POINTER
    ip, dp = P(i32), P(ctypes.c_double)
    L.dem_workspace_size.argtypes = [P(Config), P(ctypes.c_size_t)]
    L.dem_batch_workspace_size.argtypes = [i32, P(Config), P(ctypes.c_size_t)]
    L.dem_init.argtypes = [P(vp), P(Config), vp, ctypes.c_size_t, vp]
    L.dem_batch_init.argtypes = [P(vp), i32, P(Config), vp, ctypes.c_size_t, vp]
    L.dem_init_noalloc.argtypes = [P(vp), P(Config), vp]
    for name in ("dem_reset", "dem_bin", "dem_neighbors"):
        getattr(L, name).argtypes = [vp, P(State)]
    L.dem_forces.argtypes = [vp, P(State), ctypes.c_int]
    L.dem_integrate.argtypes = [vp, P(State), ctypes.c_int]
    L.dem_step.argtypes = [vp, P(State), i64]
    L.dem_declare_forces.argtypes = [vp]
    L.dem_set_step_options.argtypes = [vp, ctypes.c_int, i32]
    L.dem_set_multirate.argtypes = [vp, ctypes.c_int]
    L.dem_set_launch.argtypes = [vp, i32, i32]
    L.dem_check.argtypes = [vp, P(i64)]
    L.dem_stats.argtypes = [vp, P(i64)]
    L.dem_set_timing.argtypes = [vp, ctypes.c_int]
    L.dem_kernel_times.argtypes = [vp, P(ctypes.c_double), P(i64)]
    L.dem_export_neighbors.argtypes = [vp, P(State), ip, ip, i64, P(i64)]
    L.dem_export_contacts.argtypes = [vp, P(State), ip, ip, dp, i64, P(i64)]
    L.dem_export_wall.argtypes = [vp, P(State), ip, dp, i64, P(i64)]
    L.dem_import_history.argtypes = [vp, P(State), i64, ip, ip, dp, i64, ip, dp]
    L.dem_last_error.argtypes = [vp]
    L.dem_last_error.restype = ctypes.c_char_p
    L.dem_destroy.argtypes = [vp]
    L.dem_set_materials.argtypes = [vp, i32, P(Material), i32]
    L.dem_adjoint_workspace_size.argtypes = [vp, i64, i32, i32, i32, i32, P(ctypes.c_size_t)]
    L.dem_adjoint_init.argtypes = [vp, i64, i32, i32, i32, i32, vp, ctypes.c_size_t, P(vp)]
    L.dem_rollout_forward.argtypes = [vp, P(State)]
    L.dem_rollout_backward.argtypes = [vp, P(State), vp, vp, vp, vp, vp, vp, vp, dp]
    L.dem_forces_vjp.argtypes = [vp, P(State), vp, vp, vp, vp, vp, dp]
    L.dem_integrate_vjp.argtypes = [vp, P(State), ctypes.c_int, vp, vp, vp, vp, vp, vp, vp, vp]
    L.dem_adjoint_set_lanes.argtypes = [vp, i32]
    L.dem_adjoint_info.argtypes = [vp, P(i64)]
    L.dem_adjoint_destroy.argtypes = [vp]
    L.dem_cell_fields.argtypes = [vp, P(State), P(Grid), vp]
    L.dem_cell_mass_fields.argtypes = [vp, P(State), P(Grid), vp]
    L.dem_pi_control.argtypes = [vp, P(State), P(PIParams), vp, vp, vp, vp]
    L.dem_p_control.argtypes = [vp, P(State), P(PParams), vp, vp]
    L.dem_set_external_force.argtypes = [vp, P(State), vp]
    L.dem_exchange.argtypes = [vp, P(State), i32, P(ExchangeParams), vp, vp, i64, vp, vp, vp, vp, vp, P(i64)]
    L.dem_live_count.argtypes = [vp, i32, P(i64)]
    L.dem_set_surfaces.argtypes = [vp, i32, i32, P(Surface)]
    L.dem_export_surface_history.argtypes = [vp, P(State), vp, vp, vp, i64, P(i64)]
    L.dem_step_coupled.argtypes = [vp, P(State), i64, P(CouplingPlan)]
    L.dem_import_surface_history.argtypes = [vp, P(State), i64, vp, vp, vp]
    for name in _SYMBOLS:
        if name != "dem_last_error":
            getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def symbols():
    return list(_SYMBOLS)


def make_config(system, k_max: int = 32, block: int = 0, cell: float = 0.0, skin: float | None = None,
                n_max: int = 0, n_surf: int = 0) -> Config:
    """dem_config of one workload system (inputs.workloads.System)."""
    c = Config()
    mats = system.materials
    if not 1 <= len(mats) <= MAX_TYPES:
        raise ValueError("1..4 material types")
    c.ntypes = len(mats)
    for t, m in enumerate(mats):
        c.mat[t].E, c.mat[t].nu, c.mat[t].rho, c.mat[t].e, c.mat[t].mu = m.E, m.nu, m.rho, m.e, m.mu
    c.dt = system.dt
    for a in range(3):
        c.g[a] = system.g[a]
        c.lo[a] = system.lo[a]
        c.hi[a] = system.hi[a]
        c.periodic[a] = int(system.periodic[a])
    c.wall_z0 = int(system.wall_z0)
    c.skin = system.skin if skin is None else skin
    c.cell = cell
    c.r_max = float(np.max(system.r)) if system.n else 1e-3
    c.n = system.n
    c.k_max = k_max
    c.block = block
    c.n_max = int(n_max)
    c.n_surf = int(n_surf)
    return c


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _i32p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class DemSystem:
    """Particles of one or several systems on the GPU plus a libdem context.

    ``systems``: one ``System`` or a list (a batch; the systems are concatenated
    and ids are made unique by adding each system's slot offset).
    ``capacity``: particle slots per system (one number or a list; default:
    the system's count), room for spheres inserted by ``exchange``.
    ``surfaces``: static wall surfaces per system (a list of records (kind,
    enabled, cx, cy, z0, z1, r0, r1) for one system, or a list of such lists);
    the system's surfaces can be changed later with ``set_surfaces``.
    """

    def __init__(self, systems, k_max: int = 32, block: int = 0, cell=0.0, skin=None, device: str = "cuda",
                 use_graph: bool = False, chunk: int = 64, lanes: int = 0, max_blocks: int = 0,
                 static_workspace: bool = False, capacity=None, surfaces=None):
        import torch

        self.torch = torch
        self.L = load()
        if not isinstance(systems, (list, tuple)):
            systems = [systems]
        self.systems = list(systems)
        self.nsys = len(self.systems)
        cells = cell if isinstance(cell, (list, tuple)) else [cell] * self.nsys
        skins = skin if isinstance(skin, (list, tuple)) else [skin] * self.nsys
        caps = capacity if isinstance(capacity, (list, tuple)) else [capacity] * self.nsys
        self.live_counts = [s.n for s in self.systems]
        self.counts = [s.n if caps[k] is None else int(caps[k]) for k, s in enumerate(self.systems)]
        if surfaces is None:
            surfs = [None] * self.nsys
        elif self.nsys == 1 and (len(surfaces) == 0 or not isinstance(surfaces[0][0], (list, tuple))):
            surfs = [surfaces]
        else:
            surfs = list(surfaces)
        self.cfgs = (Config * self.nsys)(*[make_config(s, k_max, block, cells[k], skins[k], self.counts[k],
                                                       len(surfs[k]) if surfs[k] else 0)
                                          for k, s in enumerate(self.systems)])
        self.offsets = np.concatenate([[0], np.cumsum(self.counts)]).astype(np.int64)
        self.n = int(self.offsets[-1])
        self.id_offset = np.repeat(self.offsets[:-1], self.live_counts).astype(np.int64)
        self.device = torch.device(device)
        # a stream of our own (default priority): graph capture needs a non-default stream
        self.stream = torch.cuda.Stream(self.device)
        ws = ctypes.c_size_t()
        self._rc(self.L.dem_batch_workspace_size(self.nsys, self.cfgs, ctypes.byref(ws)))
        self.ws_bytes = ws.value
        self.ctx = ctypes.c_void_p()
        if static_workspace:
            # dem_init_noalloc: the library's static device array is the workspace
            if self.nsys != 1:
                raise ValueError("static_workspace takes one system")
            self.workspace = None
            with torch.cuda.device(self.device):
                self._rc(self.L.dem_init_noalloc(ctypes.byref(self.ctx), self.cfgs,
                                                 ctypes.c_void_p(self.stream.cuda_stream)))
        else:
            self.workspace = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
            base = self.workspace.data_ptr()
            self.ws_ptr = (base + 255) // 256 * 256
            self._rc(self.L.dem_batch_init(ctypes.byref(self.ctx), self.nsys, self.cfgs, ctypes.c_void_p(self.ws_ptr),
                                           ctypes.c_size_t(self.ws_bytes), ctypes.c_void_p(self.stream.cuda_stream)))
        f64 = dict(dtype=torch.float64, device=self.device)
        self.x = torch.empty((3, self.n), **f64)
        self.v = torch.empty((3, self.n), **f64)
        self.w = torch.empty((3, self.n), **f64)
        self.f = torch.zeros((3, self.n), **f64)
        self.t = torch.zeros((3, self.n), **f64)
        self.r = torch.empty(self.n, **f64)
        self.type = torch.empty(self.n, dtype=torch.int32, device=self.device)
        self.id = torch.empty(self.n, dtype=torch.int32, device=self.device)
        self.load_state()
        self._state = State(*[_ptr(t) for t in (self.x, self.v, self.w, self.f, self.t, self.r, self.type, self.id)])
        self._rc(self.L.dem_set_step_options(self.ctx, int(use_graph), int(chunk)))
        self._rc(self.L.dem_set_launch(self.ctx, int(lanes), int(max_blocks)))
        self.reset()
        self.surfaces = [[] for _ in range(self.nsys)]
        for k, sf in enumerate(surfs):
            if sf:
                self.set_surfaces(k, sf)

    def set_surfaces(self, sys: int, records):
        """Static wall surfaces of system `sys` (dem_set_surfaces)."""
        self._rc(self.L.dem_set_surfaces(self.ctx, int(sys), len(records), make_surfaces(records)))
        self.surfaces[int(sys)] = [tuple(r) for r in records]

    def export_surface_history(self):
        """(id, surface index, xi (k, 3)) of every stored surface history (the
        surface contacts of the last force evaluation)."""
        cnt = ctypes.c_int64()
        self._rc(self.L.dem_export_surface_history(self.ctx, self._state, None, None, None, 0, ctypes.byref(cnt)))
        a = np.empty(cnt.value, np.int32); k = np.empty(cnt.value, np.int32); xi = np.empty((cnt.value, 3))
        self._rc(self.L.dem_export_surface_history(self.ctx, self._state, _i32p(a), _i32p(k), _dp(xi), cnt.value,
                                                   ctypes.byref(cnt)))
        return a, k, xi

    def import_surface_history(self, ids, surf, xi):
        ids = np.ascontiguousarray(ids, np.int32); surf = np.ascontiguousarray(surf, np.int32)
        xi = np.ascontiguousarray(xi, np.float64).reshape(-1, 3)
        self._rc(self.L.dem_import_surface_history(self.ctx, self._state, len(ids), _i32p(ids), _i32p(surf), _dp(xi)))

    # ------------------------------------------------------------ helpers
    def _rc(self, rc):
        if rc != DEM_OK:
            msg = self.L.dem_last_error(getattr(self, "ctx", None) or None)
            raise DemError(rc, (msg or b"").decode())

    def close(self):
        """Destroy the context now (a static-workspace context releases the array)."""
        ctx = getattr(self, "ctx", None)
        if ctx is not None and ctx.value:
            try:
                self.torch.cuda.synchronize(self.device)
            except Exception:
                pass
            self.L.dem_destroy(ctx)
        self.ctx = None

    def __del__(self):
        self.close()

    def live_index(self):
        """Slots of the live particles, system by system."""
        return np.concatenate([np.arange(self.offsets[k], self.offsets[k] + self.live_counts[k])
                               for k in range(self.nsys)]).astype(np.int64)

    def load_state(self, x=None, v=None, w=None, f=None, t=None):
        """Copy host arrays ((n,3) rows in system order, ids from the systems) to
        the device (the systems' own particles: before any exchange)."""
        torch = self.torch
        cat = lambda k: np.concatenate([getattr(s, k) for s in self.systems])  # noqa: E731
        slots = self.live_index()
        dense = len(slots) == self.n
        idx = None if dense else torch.from_numpy(slots).to(self.device)

        def put(dst, host):
            src = torch.from_numpy(np.ascontiguousarray(host)).to(self.device)
            if dense:
                dst.copy_(src)
            else:
                dst[..., idx] = src

        x = cat("x") if x is None else x
        v = cat("v") if v is None else v
        w = cat("w") if w is None else w
        if not dense:
            for a in (self.x, self.v, self.w, self.f, self.t):
                a.zero_()
            self.r.fill_(1.0)
            self.type.zero_()
            self.id.fill_(-1)
        put(self.x, np.asarray(x, np.float64).T)
        put(self.v, np.asarray(v, np.float64).T)
        put(self.w, np.asarray(w, np.float64).T)
        if f is not None:
            put(self.f, np.asarray(f, np.float64).T)
        if t is not None:
            put(self.t, np.asarray(t, np.float64).T)
        put(self.r, cat("r").astype(np.float64))
        put(self.type, cat("type").astype(np.int32))
        gid = cat("id").astype(np.int64) + self.id_offset
        put(self.id, gid.astype(np.int32))
        torch.cuda.synchronize(self.device)

    @property
    def state(self):
        return self._state

    # ------------------------------------------------------------ the ABI
    def reset(self):
        self._rc(self.L.dem_reset(self.ctx, self._state))

    def bin(self):
        self._rc(self.L.dem_bin(self.ctx, self._state))

    def neighbors(self):
        self._rc(self.L.dem_neighbors(self.ctx, self._state))

    def build_list(self):
        self.bin()
        self.neighbors()

    def forces(self, update_history: bool = False):
        self._rc(self.L.dem_forces(self.ctx, self._state, int(update_history)))

    def integrate(self, phase: int):
        self._rc(self.L.dem_integrate(self.ctx, self._state, int(phase)))

    def integrate_vjp(self, phase: int, xb, vb, wb) -> dict:
        """Reverse of integrate(phase) (dem_integrate_vjp): the adjoints of its
        outputs x, v, w ((3, n) device, current order) -> the adjoints of its
        inputs x, v, w, f, t (a dict of new (3, n) device tensors)."""
        t = self.torch
        xb, vb, wb = (q.to(t.float64).contiguous() for q in (xb, vb, wb))
        out = {k: t.empty((3, self.n), dtype=t.float64, device=self.device) for k in ("x", "v", "w", "f", "t")}
        self._enter(xb, vb, wb, *out.values())
        self._rc(self.L.dem_integrate_vjp(self.ctx, self._state, int(phase), _ptr(xb), _ptr(vb), _ptr(wb),
                                          *[_ptr(out[k]) for k in ("x", "v", "w", "f", "t")]))
        self._leave()
        return out

    def step(self, nsteps: int):
        self._rc(self.L.dem_step(self.ctx, self._state, int(nsteps)))

    def declare_forces(self):
        """State that f and t hold the forces of the current state (e.g. loaded
        with load_state), so that step() may start from them."""
        self._rc(self.L.dem_declare_forces(self.ctx))

    def set_multirate(self, enable: bool = True):
        """Each system of the batch steps with its own dt every dt / dt_min
        substeps; step(n) then counts substeps of dt_min (dem_set_multirate)."""
        self._rc(self.L.dem_set_multirate(self.ctx, int(enable)))

    def set_step_options(self, use_graph: bool, chunk: int = 64):
        self._rc(self.L.dem_set_step_options(self.ctx, int(use_graph), int(chunk)))

    def set_launch(self, lanes: int = 0, max_blocks: int = 0):
        self._rc(self.L.dem_set_launch(self.ctx, int(lanes), int(max_blocks)))

    def prime(self):
        """Bin, build the list and evaluate the initial forces (history untouched)."""
        self.build_list()
        self.forces(False)

    def set_timing(self, enable: bool):
        self._rc(self.L.dem_set_timing(self.ctx, int(enable)))

    def kernel_times(self):
        """{class: (total ms, launches)}: first kick-drift (pack), fused step, last step, rebuild."""
        ms = (ctypes.c_double * 4)()
        n = (ctypes.c_int64 * 4)()
        self._rc(self.L.dem_kernel_times(self.ctx, ms, n))
        return {k: (ms[q], n[q]) for q, k in enumerate(("pack", "step", "last", "rebuild"))}

    def check(self):
        info = (ctypes.c_int64 * 4)()
        rc = self.L.dem_check(self.ctx, info)
        return rc, list(info)

    def stats(self):
        out = (ctypes.c_int64 * 5)()
        self._rc(self.L.dem_stats(self.ctx, out))
        return dict(steps=out[0], builds=out[1], contacts=out[2], wall_contacts=out[3], slots=out[4])

    # ------------------------------------------------------------ host views (by id)
    def host(self, system: int | None = None):
        """Current state of the live particles (of one system, or all) as
        numpy, rows sorted by (global) id: x, v, w, f, t (n,3), r, type, id (n,)."""
        self.torch.cuda.synchronize(self.device)
        if system is None:
            slots = self.live_index()
        else:
            slots = np.arange(self.offsets[system], self.offsets[system] + self.live_counts[system])
        ids = self.id.cpu().numpy()[slots]
        order = np.argsort(ids, kind="stable")
        sel = slots[order]
        out = {"id": ids[order]}
        for k in ("x", "v", "w", "f", "t"):
            out[k] = getattr(self, k).cpu().numpy().T[sel].copy()
        out["r"] = self.r.cpu().numpy()[sel]
        out["type"] = self.type.cpu().numpy()[sel]
        return out

    def export_neighbors(self):
        cnt = ctypes.c_int64()
        self._rc(self.L.dem_export_neighbors(self.ctx, self._state, None, None, 0, ctypes.byref(cnt)))
        a = np.empty(cnt.value, np.int32); b = np.empty(cnt.value, np.int32)
        self._rc(self.L.dem_export_neighbors(self.ctx, self._state, _i32p(a), _i32p(b), cnt.value, ctypes.byref(cnt)))
        return a, b

    def export_contacts(self):
        cnt = ctypes.c_int64()
        self._rc(self.L.dem_export_contacts(self.ctx, self._state, None, None, None, 0, ctypes.byref(cnt)))
        a = np.empty(cnt.value, np.int32); b = np.empty(cnt.value, np.int32); xi = np.empty((cnt.value, 3))
        self._rc(self.L.dem_export_contacts(self.ctx, self._state, _i32p(a), _i32p(b), _dp(xi), cnt.value,
                                            ctypes.byref(cnt)))
        return a, b, xi

    def export_wall(self):
        cnt = ctypes.c_int64()
        self._rc(self.L.dem_export_wall(self.ctx, self._state, None, None, 0, ctypes.byref(cnt)))
        a = np.empty(cnt.value, np.int32); xi = np.empty((cnt.value, 3))
        self._rc(self.L.dem_export_wall(self.ctx, self._state, _i32p(a), _dp(xi), cnt.value, ctypes.byref(cnt)))
        return a, xi

    # ------------------------------------------------------------ coupling (Sec. 2.3)
    def cell_fields(self, grid: Grid, stress: bool = True, out=None):
        """Fields of the cells of `grid` at the current state: device tensor
        (NFIELDS, ncell) with rows F_COUNT, F_MASS, F_MOM..+2, F_VOLUME, F_VMAX,
        F_STRESS..+8 (sigma_ab of Eq. 7 at row F_STRESS + 3 a + b).  Without
        `stress` (dem_cell_mass_fields) the stress rows are left as they are.
        `out`: a contiguous float64 device tensor of that shape to reuse."""
        ncell = grid.n[0] * grid.n[1] * grid.n[2]
        if out is None:
            out = self.torch.empty((NFIELDS, ncell), dtype=self.torch.float64, device=self.device)
        elif out.shape != (NFIELDS, ncell) or out.dtype != self.torch.float64 or not out.is_contiguous():
            raise ValueError("out must be a contiguous float64 tensor of shape (NFIELDS, ncell)")
        self._enter(out)
        fn = self.L.dem_cell_fields if stress else self.L.dem_cell_mass_fields
        self._rc(fn(self.ctx, self._state, ctypes.byref(grid), _ptr(out)))
        self._leave()
        return out

    # The library works on its own stream; tensors come from and go to the
    # caller's current stream: ordered on the device by stream waits, without
    # blocking the host.
    def _enter(self, *tensors):
        cur = self.torch.cuda.current_stream(self.device)
        if cur == self.stream:
            return
        self.stream.wait_stream(cur)
        for t in tensors:
            if t is not None:
                t.record_stream(self.stream)

    def _leave(self):
        cur = self.torch.cuda.current_stream(self.device)
        if cur != self.stream:
            cur.wait_stream(self.stream)

    def pi_control(self, params: PIParams, fine, coarse, integral, u=None):
        """PI controller of the transition layer (fine system params.grid.sys):
        updates `integral` (device, (ncell,)) in place, returns u (device)."""
        ncell = params.grid.n[0] * params.grid.n[1] * params.grid.n[2]
        if u is None:
            u = self.torch.empty(ncell, dtype=self.torch.float64, device=self.device)
        fine, coarse = fine.contiguous(), coarse.contiguous()
        self._enter(fine, coarse, integral, u)
        self._rc(self.L.dem_pi_control(self.ctx, self._state, ctypes.byref(params), _ptr(fine), _ptr(coarse),
                                       _ptr(integral), _ptr(u)))
        self._leave()
        return u

    def p_control(self, params: PParams, fine, coarse):
        """P controller of the coarse system params.grid.sys inside the fine region."""
        fine, coarse = fine.contiguous(), coarse.contiguous()
        self._enter(fine, coarse)
        self._rc(self.L.dem_p_control(self.ctx, self._state, ctypes.byref(params), _ptr(fine), _ptr(coarse)))
        self._leave()

    def coupling_plan(self, pi: PIParams, pi_setpoint_sys: int, p: PParams, p_target_sys: int, interval_steps: int,
                      group: int = 4, integral=None, sum_grid: Grid | None = None):
        """A dem_coupling_plan with its device buffers (kept on the returned
        object: pi_fine, pi_coarse, p_fine, p_coarse, integral, u, and with
        sum_grid the running sum `sum` and its scratch)."""
        t = self.torch
        f64 = dict(dtype=t.float64, device=self.device)
        cells = lambda g: g.n[0] * g.n[1] * g.n[2]  # noqa: E731
        plan = CouplingPlan()
        plan.pi, plan.pi_setpoint_sys, plan.p, plan.p_target_sys = pi, int(pi_setpoint_sys), p, int(p_target_sys)
        plan.interval_steps, plan.group = int(interval_steps), int(group)
        bufs = {"pi_fine": t.zeros((NFIELDS, cells(pi.grid)), **f64), "pi_coarse": t.zeros((NFIELDS, cells(pi.grid)), **f64),
                "p_fine": t.zeros((NFIELDS, cells(p.grid)), **f64), "p_coarse": t.zeros((NFIELDS, cells(p.grid)), **f64),
                "integral": t.zeros(cells(pi.grid), **f64) if integral is None else integral,
                "u": t.zeros(cells(pi.grid), **f64)}
        if sum_grid is not None:
            plan.sum_grid = sum_grid
            bufs["sum"] = t.zeros((NFIELDS, cells(sum_grid)), **f64)
            bufs["sum_tmp"] = t.zeros((NFIELDS, cells(sum_grid)), **f64)
        for k, v in bufs.items():
            setattr(plan, k, v.data_ptr())
        plan.buffers = bufs
        return plan

    def step_coupled(self, nintervals: int, plan: CouplingPlan):
        """nintervals coupling intervals (dem_step_coupled)."""
        self._enter(*plan.buffers.values())
        self._rc(self.L.dem_step_coupled(self.ctx, self._state, int(nintervals), ctypes.byref(plan)))
        self._leave()

    def set_external_force(self, fext=None):
        """External forces of all spheres, device (3, n) in the current order, or None."""
        if fext is not None:
            fext = fext.to(self.torch.float64).contiguous()
        self._enter(fext)
        self._rc(self.L.dem_set_external_force(self.ctx, self._state, _ptr(fext)))
        self._leave()

    def exchange(self, sys: int, params: ExchangeParams, fields, budget, cand_x=None, cand_r=None, cand_type=None,
                 cand_cell=None):
        """One insertion and deletion event on system `sys` (dem_exchange):
        fields device (NFIELDS, ncell) of the coarse level on the boundary
        cells, budget device (ncell,) updated in place, candidates as device or
        host arrays (positions (k, 3)).  The system's list and forces are
        rebuilt by the call.  Returns (accepted device int32 (k,), inserted,
        removed)."""
        torch = self.torch
        k = 0 if cand_r is None else int(len(cand_r))
        dev = dict(device=self.device)
        if k:
            cx = torch.as_tensor(np.asarray(cand_x, np.float64).T if isinstance(cand_x, np.ndarray) else cand_x.T,
                                 dtype=torch.float64, **dev).contiguous()
            cr = torch.as_tensor(cand_r, dtype=torch.float64, **dev).contiguous()
            ct = torch.as_tensor(cand_type, dtype=torch.int32, **dev).contiguous()
            cc = torch.as_tensor(cand_cell, dtype=torch.int32, **dev).contiguous()
        else:
            cx = cr = ct = cc = None
        acc = torch.zeros(max(k, 1), dtype=torch.int32, **dev)
        fields = fields.to(torch.float64).contiguous()
        counts = (ctypes.c_int64 * 3)()
        self._enter(fields, budget, cx, cr, ct, cc, acc)
        self._rc(self.L.dem_exchange(self.ctx, self._state, int(sys), ctypes.byref(params), _ptr(fields),
                                     _ptr(budget), k, _ptr(cx), _ptr(cr), _ptr(ct), _ptr(cc), _ptr(acc), counts))
        self.live_counts[sys] = int(counts[2])
        self._leave()
        return acc[:k], int(counts[0]), int(counts[1])

    def live(self, sys: int) -> int:
        n = ctypes.c_int64()
        self._rc(self.L.dem_live_count(self.ctx, int(sys), ctypes.byref(n)))
        return int(n.value)

    def set_materials(self, materials, sys: int = 0):
        """New per-type materials of system `sys` (objects with E, nu, rho, e, mu)."""
        arr = (Material * len(materials))()
        for t, m in enumerate(materials):
            arr[t].E, arr[t].nu, arr[t].rho, arr[t].e, arr[t].mu = m.E, m.nu, m.rho, m.e, m.mu
        self._rc(self.L.dem_set_materials(self.ctx, int(sys), arr, len(materials)))

    def adjoint(self, nsteps: int, window: int = 20, max_windows: int = 0, keep: bool = False,
                kslots: int = 0) -> "Adjoint":
        return Adjoint(self, nsteps, window, max_windows, keep, kslots)

    def checkpoint(self) -> dict:
        """Host snapshot from which from_checkpoint resumes bit for bit: per
        system its live particles (positions, velocities, spins, radii, types,
        ids relative to the system's slot offset), forces and torques, plus the
        tangential history of every pair in contact, of every wall contact
        and of every surface contact (by id), and the current surfaces.  The list itself is not saved: the step's results do not
        depend on when it was built."""
        from .inputs.workloads import System

        h = [self.host(k) for k in range(self.nsys)]
        systems = []
        for k, s in enumerate(self.systems):
            hk = h[k]
            c = System(hk["x"], hk["v"], hk["w"], hk["r"], hk["type"].astype(np.int32),
                       (hk["id"] - self.offsets[k]).astype(np.int32), list(s.materials), tuple(s.lo), tuple(s.hi),
                       tuple(s.periodic), s.wall_z0, tuple(s.g), s.dt, s.skin, s.steps, s.name, s.alpha, dict(s.meta))
            systems.append(c)
        a, b, xi = self.export_contacts()
        wid, wxi = self.export_wall()
        return {"systems": systems, "f": np.concatenate([q["f"] for q in h]), "t": np.concatenate([q["t"] for q in h]),
                "pairs": (a, b, xi), "wall": (wid, wxi), "capacity": list(self.counts),
                "surfaces": [list(sf) for sf in self.surfaces], "surface_history": self.export_surface_history(),
                "steps": self.stats()["steps"]}

    @classmethod
    def from_checkpoint(cls, ckpt: dict, **kwargs) -> "DemSystem":
        """A new context resumed from checkpoint(): same slot capacities, the
        state and history loaded, the saved forces declared current."""
        surfs = ckpt.get("surfaces")
        if surfs and any(surfs) and "surfaces" not in kwargs:
            kwargs["surfaces"] = surfs
        g = cls(ckpt["systems"], capacity=ckpt["capacity"], **kwargs)
        g.load_state(f=ckpt["f"], t=ckpt["t"])
        g.reset()
        g.build_list()
        g.import_history(*ckpt["pairs"], *ckpt["wall"])
        sh = ckpt.get("surface_history")
        if sh is not None and len(sh[0]):
            g.import_surface_history(*sh)
        g.declare_forces()
        return g

    def import_history(self, id_i, id_j, xi, wall_id=None, wall_xi=None):
        id_i = np.ascontiguousarray(id_i, np.int32); id_j = np.ascontiguousarray(id_j, np.int32)
        xi = np.ascontiguousarray(xi, np.float64).reshape(-1, 3)
        wall_id = np.zeros(0, np.int32) if wall_id is None else np.ascontiguousarray(wall_id, np.int32)
        wall_xi = np.zeros((0, 3)) if wall_xi is None else np.ascontiguousarray(wall_xi, np.float64).reshape(-1, 3)
        self._rc(self.L.dem_import_history(self.ctx, self._state, len(id_i), _i32p(id_i), _i32p(id_j), _dp(xi),
                                           len(wall_id), _i32p(wall_id), _dp(wall_xi)))


class Adjoint:
    """Reverse mode of a rollout on a DemSystem of one system (dem_rollout_*).

    ``forward()`` runs ``nsteps`` steps from the system's current state with
    checkpoints every ``window`` steps (with ``keep``, the inputs of every
    step are stored and the backward recomputes nothing); ``backward(gx, gv, gw)`` takes the
    adjoints of the final x, v, w ((3, n) device tensors in the system's
    current order) and returns the gradients with respect to the per-type
    E, e and mu (host) and to the initial x, v, w (device, in the order of
    ``ids0``; ``initial_by_id`` gives host rows in id order).  ``kslots``
    bounds the neighbour rows the checkpoints hold (0: the context's k_max)."""

    def __init__(self, dsys: DemSystem, nsteps: int, window: int = 20, max_windows: int = 0, keep: bool = False,
                 kslots: int = 0):
        torch = dsys.torch
        self.dsys = dsys
        self.L = dsys.L
        self.nsteps = int(nsteps)
        self.window = int(window)
        self.ntypes = len(dsys.systems[0].materials)
        nb = ctypes.c_size_t()
        self.keep = bool(keep)
        self.kslots = int(kslots)
        dsys._rc(self.L.dem_adjoint_workspace_size(dsys.ctx, self.nsteps, self.window, int(max_windows),
                                                   int(self.keep), self.kslots, ctypes.byref(nb)))
        self.bytes = nb.value
        self.workspace = torch.empty(self.bytes + 256, dtype=torch.uint8, device=dsys.device)
        ptr = (self.workspace.data_ptr() + 255) // 256 * 256
        self.h = ctypes.c_void_p()
        dsys._rc(self.L.dem_adjoint_init(dsys.ctx, self.nsteps, self.window, int(max_windows), int(self.keep),
                                         self.kslots, ctypes.c_void_p(ptr), ctypes.c_size_t(self.bytes),
                                         ctypes.byref(self.h)))

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value:
            self.L.dem_adjoint_destroy(h)
            self.h = None

    def forward(self):
        self.dsys._rc(self.L.dem_rollout_forward(self.h, self.dsys.state))

    @staticmethod
    def initial_by_id(r: dict) -> dict:
        """Host copies of the initial-state adjoints of backward(), rows in id order."""
        ids = r["ids0"].cpu().numpy()
        order = np.argsort(ids, kind="stable")
        return {k: r[k].cpu().numpy().T[order].copy() for k in ("x0", "v0", "w0")}

    def backward(self, gx=None, gv=None, gw=None) -> dict:
        torch = self.dsys.torch
        d = self.dsys
        z = lambda g: torch.zeros((3, d.n), dtype=torch.float64, device=d.device) if g is None else \
            g.to(torch.float64).contiguous()  # noqa: E731
        gx, gv, gw = z(gx), z(gv), z(gw)
        ax, av, aw = (torch.empty((3, d.n), dtype=torch.float64, device=d.device) for _ in range(3))
        ids0 = torch.empty(d.n, dtype=torch.int32, device=d.device)
        grad = (ctypes.c_double * (3 * self.ntypes))()
        torch.cuda.current_stream(d.device).synchronize()
        d._rc(self.L.dem_rollout_backward(self.h, d.state, _ptr(gx), _ptr(gv), _ptr(gw), _ptr(ax), _ptr(av),
                                          _ptr(aw), _ptr(ids0), grad))
        g = np.array(grad[:]).reshape(3, self.ntypes)
        # initial-state adjoints stay on the device, (3, n) in the order of ids0;
        # the last result is also kept on the object (for callers of DemRollout)
        self.last = dict(E=g[0], e=g[1], mu=g[2], x0=ax, v0=av, w0=aw, ids0=ids0)
        return self.last

    def forces_vjp(self, fb, tb) -> dict:
        """Reverse mode of one force evaluation (no history update) at the current
        state: dL/df, dL/dt ((3, n) device, current order) -> dL/dx, dL/dv, dL/dw
        (current order) and the material gradients."""
        torch = self.dsys.torch
        d = self.dsys
        fb = fb.to(torch.float64).contiguous(); tb = tb.to(torch.float64).contiguous()
        xb, vb, wb = (torch.empty((3, d.n), dtype=torch.float64, device=d.device) for _ in range(3))
        grad = (ctypes.c_double * (3 * self.ntypes))()
        torch.cuda.current_stream(d.device).synchronize()
        d._rc(self.L.dem_forces_vjp(self.h, d.state, _ptr(fb), _ptr(tb), _ptr(xb), _ptr(vb), _ptr(wb), grad))
        g = np.array(grad[:]).reshape(3, self.ntypes)
        return dict(E=g[0], e=g[1], mu=g[2], x=xb, v=vb, w=wb)

    def set_lanes(self, lanes: int):
        self.dsys._rc(self.L.dem_adjoint_set_lanes(self.h, int(lanes)))

    def info(self) -> dict:
        out = (ctypes.c_int64 * 4)()
        self.dsys._rc(self.L.dem_adjoint_info(self.h, out))
        return dict(windows=out[0], rebuilds=out[1], bytes=out[2], max_windows=out[3])
