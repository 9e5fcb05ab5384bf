"""GPU (HIP, gfx950) against the FP64 CPU oracle on the same seeded inputs.

Bars (from the method's arithmetic, see the design notes):
  * neighbour list and contact set: identical (bit-exact) sets of directed pairs;
  * history-slot mapping: identical pair sets, xi_ji == -xi_ij bit for bit;
  * forces after one evaluation: |dF_i| <= 1e-12 sum_j |F_ij| per particle;
  * positions after 100 steps: max |dx| <= 1e-9 max(L).
"""
import numpy as np
import pytest

import oracle as O
from paper_1705_03850_amd.inputs import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def gpu(system, **kw):
    from paper_1705_03850_amd import dem
    return dem.DemSystem(system, **kw)


def directed(lo, hi, xi=None):
    a = np.concatenate([lo, hi]); b = np.concatenate([hi, lo])
    order = np.lexsort((b, a))
    if xi is None:
        return a[order], b[order]
    x = np.concatenate([xi, -xi])
    return a[order], b[order], x[order]


def force_scale(o, n, ids, mass):
    """Per particle: m|g| + sum over its contacts of |F_ij| (oracle records)."""
    rec = o.records()
    pos = {int(v): k for k, v in enumerate(ids)}
    s = mass * 9.81
    for lo, hi, fm in zip(rec["lo"], rec["hi"], rec["fmag"]):
        s[pos[int(lo)]] += fm
        if hi >= 0:
            s[pos[int(hi)]] += fm
    return s


def by_id(system, arr):
    order = np.argsort(system.id, kind="stable")
    return arr[order]


def load_oracle_state(g, system, o):
    """Put the oracle's state and history into the GPU context."""
    st = o.state()
    g.load_state(x=st["x"], v=st["v"], w=st["w"], f=st["f"], t=st["t"])
    g.reset()
    g.build_list()
    lo, hi, xi = o.history()
    a, b, x = directed(lo, hi, xi)
    wid, wxi = o.wall_history()
    g.import_history(a, b, x, wid, wxi)
    g.declare_forces()          # f, t are the oracle's forces of this state


def compare_forces(g, system, o, tol=1e-12):
    h = g.host()
    st = o.state()
    m, _ = o.mass()
    scale = by_id(system, force_scale(o, system.n, system.id, m.copy()))
    F = by_id(system, st["f"]); T = by_id(system, st["t"])
    dF = np.linalg.norm(h["f"] - F, axis=1)
    dT = np.linalg.norm(h["t"] - T, axis=1)
    r = by_id(system, system.r)
    assert np.all(dF <= tol * scale), (dF / scale).max()
    assert np.all(dT <= tol * scale * r), (dT / (scale * r)).max()
    return float(np.mean(dF == 0.0))


# --------------------------------------------------------------------------

@pytest.mark.parametrize("k_max", [16, 32, 63])
def test_neighbor_list_bitexact_plain(k_max):
    """Row capacities from just above the FCC rows (12) to the largest
    allowed (63, the most LDS per group)."""
    s = W.plain_fcc()
    g = gpu(s, k_max=k_max)
    g.build_list()
    a, b = g.export_neighbors()
    o = O.Oracle(s)
    lo, hi = o.pairs(s.skin, brute=True)
    ea, eb = directed(lo, hi)
    assert len(a) > 20000
    assert np.array_equal(a, ea) and np.array_equal(b, eb)


def test_neighbor_list_bitexact_bed():
    s = W.settled_bed(seed=7, n=20000, footprint=80e-3 * np.sqrt(0.02))
    g = gpu(s)
    g.build_list()
    a, b = g.export_neighbors()
    o = O.Oracle(s)
    lo, hi = o.pairs(s.skin, brute=False)
    ea, eb = directed(lo, hi)
    assert np.array_equal(a, ea) and np.array_equal(b, eb)


@pytest.mark.parametrize("ncx,ncy,pz", [(2, 3, 0), (3, 3, 0), (4, 2, 0), (5, 3, 1), (7, 4, 1)])
def test_neighbor_list_bitexact_small_periodic_boxes(ncx, ncy, pz):
    """Boxes of two to seven cells per periodic axis: the x-runs of three cells
    (one piece, or two across the seam), the minimum image on short axes and
    the duplicate-free runs of two-cell axes, against brute force."""
    from paper_1705_03850_amd.inputs.workloads import MAT_A, System
    rng = np.random.default_rng(100 + 10 * ncx + ncy)
    edge = 2.6e-3                         # just above the cut-off 2 r_max + skin = 2.52 mm
    L = (ncx * edge, ncy * edge, (3 if pz else 4) * edge)
    n = int(0.2e9 * L[0] * L[1] * L[2])   # about ten neighbours per particle
    x = rng.uniform(0.0, 1.0, size=(n, 3)) * np.array(L)
    s = System(x=x, v=np.zeros((n, 3)), w=np.zeros((n, 3)), r=rng.uniform(0.8e-3, 1.2e-3, n),
               type=np.zeros(n, np.int32), id=rng.permutation(n).astype(np.int32), materials=[MAT_A],
               lo=(0.0, 0.0, 0.0), hi=L, periodic=(1, 1, pz), wall_z0=0, g=(0.0, 0.0, 0.0), dt=1e-6,
               skin=0.12e-3, steps=0, name=f"gas_{ncx}x{ncy}")
    g = gpu(s)
    g.build_list()
    a, b = g.export_neighbors()
    o = O.Oracle(s)
    lo, hi = o.pairs(s.skin, brute=True)
    ea, eb = directed(lo, hi)
    assert len(a) > 4 * n
    assert np.array_equal(a, ea) and np.array_equal(b, eb)


def test_forces_first_evaluation_bed():
    """Settled bed: contacts from the start, zero history; one force evaluation."""
    s = W.settled_bed(seed=8, n=20000, footprint=80e-3 * np.sqrt(0.02))
    g = gpu(s)
    g.prime()
    o = O.Oracle(s)
    o.forces(False)
    exact = compare_forces(g, s, o)
    print("bitwise-equal force fraction", exact)


@pytest.mark.parametrize("k", [50, 100, 300])
def test_resumed_step_parity(k):
    """From oracle-dumped states (positions, velocities, forces, history) one more
    step on both sides: forces, contact set and history mapping."""
    s = W.plain_fcc()
    o = O.Oracle(s)
    o.forces(False)
    o.step(k)
    g = gpu(s)
    load_oracle_state(g, s, o)
    # the imported history is the oracle's, slot for slot
    ca, cb, cx = g.export_contacts()
    lo, hi, xi = o.history()
    ea, eb, ex = directed(lo, hi, xi)
    assert np.array_equal(ca, ea) and np.array_equal(cb, eb)
    assert np.array_equal(cx, ex)
    g.step(1)
    o.step(1)
    compare_forces(g, s, o)
    ca, cb, cx = g.export_contacts()
    lo, hi, xi = o.history()
    ea, eb, ex = directed(lo, hi, xi)
    assert len(ca) > 100                      # the state has contacts (the lattice starts gapped)
    assert np.array_equal(ca, ea) and np.array_equal(cb, eb)
    scale = np.maximum(np.abs(ex).max(), 1e-300)
    assert np.max(np.abs(cx - ex)) <= 1e-12 * scale
    wa, wx = g.export_wall()
    wo, wox = o.wall_history()
    assert np.array_equal(wa, wo)
    if len(wo):
        assert np.max(np.abs(wx - wox)) <= 1e-12 * max(np.abs(wox).max(), 1e-300)


@pytest.mark.parametrize("skin", [0.1e-3, 2e-6])
def test_hundred_steps_positions(skin):
    """100 independent steps from the same start.  The small skin forces list
    rebuilds (history carried by id) every few steps; the result may not depend
    on when the list is rebuilt."""
    s = W.plain_fcc()
    s.skin = skin
    g = gpu(s)
    g.prime()
    g.step(100)
    o = O.Oracle(s)
    o.forces(False)
    o.step(100)
    h = g.host()
    st = o.state()
    X = by_id(s, st["x"])
    d = h["x"] - X
    d[:, :2] -= 20e-3 * np.round(d[:, :2] / 20e-3)
    assert np.max(np.abs(d)) <= 1e-9 * 60e-3
    stats = g.stats()
    if skin < 1e-5:
        assert stats["builds"] > 5
    ca, cb, cx = g.export_contacts()
    lo, hi, xi = o.history()
    ea, eb, ex = directed(lo, hi, xi)
    assert np.array_equal(ca, ea) and np.array_equal(cb, eb)
    assert np.max(np.abs(cx - ex)) <= 1e-9 * max(np.abs(ex).max(), 1e-300)


def test_empty_system_is_a_no_op():
    """No particles: every call succeeds and changes nothing."""
    from paper_1705_03850_amd.inputs.workloads import MAT_A, System
    z = np.zeros((0, 3))
    s = System(x=z, v=z, w=z, r=np.zeros(0), type=np.zeros(0, np.int32), id=np.zeros(0, np.int32), materials=[MAT_A],
               lo=(0.0, 0.0, 0.0), hi=(10e-3, 10e-3, 10e-3), periodic=(1, 1, 0), wall_z0=1, g=(0.0, 0.0, -9.81),
               dt=1e-6, skin=0.1e-3, steps=0, name="empty")
    g = gpu(s)
    g.prime()
    g.step(10)
    h = g.host()
    assert h["x"].shape == (0, 3)
    st = g.stats()
    assert st["contacts"] == 0 and st["slots"] == 0


@pytest.mark.parametrize("case", ["one_on_wall", "two_head_on"])
def test_one_and_two_particles_against_oracle(case):
    """Degenerate sizes: a single sphere dropped onto the wall (no pairs, the
    wall only) and two spheres meeting head-on (one pair, no wall), 600 steps
    through the contact, against the oracle."""
    from systems import sphere_on_wall, two_spheres
    s = sphere_on_wall(1.0e-3 + 2e-6, v=(0.05, 0.0, -0.3)) if case == "one_on_wall" else two_spheres(1.0)
    g = gpu(s)
    g.prime()
    g.step(600)
    o = O.Oracle(s)
    o.forces(False)
    o.step(600)
    h = g.host()
    st = o.state()
    X, V = by_id(s, st["x"]), by_id(s, st["v"])
    assert np.max(np.abs(h["x"] - X)) <= 1e-9 * 40e-3
    assert np.max(np.abs(h["v"] - V)) <= 1e-9 * np.abs(V).max()
    # the contact happened and is over: the spheres move apart, the single
    # sphere has bounced off the wall
    if case == "two_head_on":
        assert V[0, 0] < 0.0 < V[1, 0]
    else:
        assert V[0, 2] > 0.0


def test_history_antisymmetric_bitwise():
    s = W.plain_fcc()
    g = gpu(s)
    g.prime()
    g.step(300)
    a, b, x = g.export_contacts()
    assert len(a) > 100
    key = {(int(p), int(q)): k for k, (p, q) in enumerate(zip(a, b))}
    for k, (p, q) in enumerate(zip(a, b)):
        j = key[(int(q), int(p))]
        assert np.array_equal(x[j], -x[k])


def test_momentum_conserved_gpu():
    s = W.plain_fcc()
    s.periodic = (1, 1, 1); s.hi = (20e-3, 20e-3, 40e-3); s.wall_z0 = 0; s.g = (0.0, 0.0, 0.0)
    g = gpu(s)
    g.prime()
    h0 = g.host()
    m = 4.0 / 3.0 * np.pi * 2500.0 * 1e-9
    p0 = (m * h0["v"]).sum(axis=0)
    g.step(1000)
    h1 = g.host()
    p1 = (m * h1["v"]).sum(axis=0)
    scale = np.sum(m * np.linalg.norm(h1["v"], axis=1))
    assert np.max(np.abs(p1 - p0)) < 1e-14 * scale


def test_deterministic_and_order_independent():
    """Same input twice, and the same particles in another storage order: the
    physics (by id) is identical bit for bit."""
    s = W.plain_fcc()
    outs = []
    for perm_seed in (None, None, 5):
        t = s.copy()
        if perm_seed is not None:
            p = np.random.default_rng(perm_seed).permutation(s.n)
            t.x, t.v, t.w, t.r, t.type, t.id = t.x[p], t.v[p], t.w[p], t.r[p], t.type[p], t.id[p]
        g = gpu(t)
        g.prime()
        g.step(200)
        outs.append(g.host())
    for o in outs[1:]:
        for k in ("x", "v", "w", "f", "t"):
            assert np.array_equal(o[k], outs[0][k]), k


def test_launch_options_do_not_change_results():
    """Block size, cell size, skin and graph replay change the schedule, not the
    results (rows are summed in id order, history follows ids)."""
    s = W.plain_fcc()
    ref = None
    for kw in (dict(), dict(block=64), dict(block=256, cell=5e-3), dict(skin=30e-6),
               dict(use_graph=True, chunk=16), dict(max_blocks=64), dict(block=64, max_blocks=8),
               dict(block=128, max_blocks=100000)):
        g = gpu(s, **kw)
        g.prime()
        g.step(150)
        h = g.host()
        if ref is None:
            ref = h
        for k in ("x", "v", "w", "f", "t"):
            assert np.array_equal(h[k], ref[k]), (kw, k)


@pytest.mark.parametrize("lanes", [8, 16])
def test_lanes_do_not_change_results(lanes):
    """Another split of a row over lanes changes only who computes which pair
    term; the terms are added in the same (id) order, so results are equal.
    The default for these 2,000 spheres (16 lanes) is one of the compared."""
    s = W.plain_fcc()
    out = []
    for kw in (dict(lanes=4), dict(), dict(lanes=lanes), dict(lanes=lanes, block=64, skin=20e-6)):
        g = gpu(s, **kw)
        g.prime()
        g.step(100)
        out.append(g.host())
    for o in out[1:]:
        for k in ("x", "v", "w", "f", "t"):
            assert np.array_equal(o[k], out[0][k]), k


def test_batch_equals_separate_systems():
    """Two systems of different coarse-grain factor in one context evolve exactly
    as each alone (Sec. 2.3 levels as a batch).  The first system's small skin
    makes it ask for a new list every few steps; only that system is rebuilt."""
    a = W.plain_fcc()
    a.skin = 3e-6
    b = W.plain_fcc(seed=9)
    b.x = b.x * 2.0; b.r = b.r * 2.0; b.hi = tuple(2 * q for q in b.hi); b.skin *= 2; b.dt *= 2
    bg = gpu([a, b])
    bg.prime()
    bg.step(120)
    hb = bg.host()
    assert bg.stats()["builds"] > 5
    for k, s in enumerate((a, b)):
        g = gpu(s)
        g.prime()
        g.step(120)
        h = g.host()
        sl = slice(int(bg.offsets[k]), int(bg.offsets[k + 1]))
        for key in ("x", "v", "w", "f", "t"):
            assert np.array_equal(hb[key][sl], h[key]), (k, key)


def test_batch_of_64_systems():
    """The 64-system workload at 5 % size (polydisperse, alpha in {1, 2, 4, 8},
    dt = alpha 1e-6 s): batched with graph replay equals systems run alone, and a
    system of the batch matches the oracle after 40 steps."""
    systems = W.batch_systems(scale=0.05)
    bg = gpu(systems, use_graph=True, chunk=16)
    bg.prime()
    bg.step(40)
    hb = bg.host()
    for k in (0, 7, 33, 63):
        s = systems[k]
        g = gpu(s)
        g.prime()
        g.step(40)
        h = g.host()
        sl = slice(int(bg.offsets[k]), int(bg.offsets[k + 1]))
        for key in ("x", "v", "w", "f", "t"):
            assert np.array_equal(hb[key][sl], h[key]), (k, key)
    k = 7
    s = systems[k]
    o = O.Oracle(s)
    o.forces(False)
    o.step(40)
    X = by_id(s, o.state()["x"])
    sl = slice(int(bg.offsets[k]), int(bg.offsets[k + 1]))
    d = hb["x"][sl] - X
    d[:, 0] -= s.hi[0] * np.round(d[:, 0] / s.hi[0])
    d[:, 1] -= s.hi[1] * np.round(d[:, 1] / s.hi[1])
    assert np.max(np.abs(d)) <= 1e-9 * max(s.hi)


@pytest.mark.parametrize("lanes,block", [(4, 256), (8, 256), (16, 256), (4, 128)])
def test_batch_tiles_within_systems(lanes, block):
    """The batch step walks tiles of block/lanes particles that never span two
    systems (a system's last tile is partly empty; systems of 20 and 70
    spheres are smaller than one or two tiles): every launch shape gives the
    systems' own results bit for bit, with and without graph replay."""
    from paper_1705_03850_amd.inputs import workloads as Wk
    systems = [Wk.chute_adjoint(seed=3, n=20, Lx=14e-3, Ly=10e-3), W.plain_fcc(),
               Wk.chute_adjoint(seed=4, n=70, Lx=14e-3, Ly=10e-3), Wk.chute_adjoint(seed=5, n=600, Lx=14e-3, Ly=10e-3)]
    for graph in (False, True):
        bg = gpu(systems, block=block, lanes=lanes, use_graph=graph, chunk=16)
        bg.prime()
        bg.step(60)
        hb = bg.host()
        for k, s in enumerate(systems):
            g = gpu(s)
            g.prime()
            g.step(60)
            h = g.host()
            sl = slice(int(bg.offsets[k]), int(bg.offsets[k + 1]))
            for key in ("x", "v", "w", "f", "t"):
                assert np.array_equal(hb[key][sl], h[key]), (graph, k, key)


def test_autotuned_batch_equals_default():
    """The autotuner returns a choice from its candidate sets, and a batch run
    with that choice (launch shape, skin, cell) equals the default run bit for
    bit: tuning trades speed only."""
    from paper_1705_03850_amd import autotune
    systems = W.batch_systems(scale=0.05)[:8]
    choice = autotune.autotune(systems, steps=8, long_steps=24, log=None)
    assert choice["lanes"] in (4, 8) and choice["block"] in (128, 256)
    assert choice["skin_factor"] in (0.1, 0.05, 0.2, 0.3) and choice["cell_factor"] in (1.0, 1.25)
    assert len(choice["tried"]) >= 2 * (2 + 2)      # every launch shape timed twice
    outs = []
    for kw in (dict(), autotune.apply(systems, choice)):
        g = gpu(systems, use_graph=True, chunk=16, **kw)
        g.prime()
        g.step(60)
        outs.append(g.host())
    for key in ("x", "v", "w", "f", "t"):
        assert np.array_equal(outs[0][key], outs[1][key]), key


def test_capacity_error_reported():
    from paper_1705_03850_amd import dem
    s = W.plain_fcc()
    g = gpu(s, k_max=4)
    with pytest.raises(dem.DemError) as e:
        g.build_list()
        g.forces(False)
        rc, info = g.check()
        g._rc(rc)
    assert e.value.code == dem.DEM_ERR_CAPACITY
    rc, info = g.check()
    assert info[1] >= 12                      # the k_max a retry needs


def test_nonfinite_reported():
    from paper_1705_03850_amd import dem
    s = W.plain_fcc()
    s.v = s.v.copy(); s.v[17, 1] = np.nan
    g = gpu(s)
    g.prime()
    with pytest.raises(dem.DemError) as e:
        g.step(3)
    assert e.value.code == dem.DEM_ERR_NONFINITE


def test_bad_type_rejected():
    from paper_1705_03850_amd import dem
    s = W.plain_fcc()
    s.type = s.type.copy(); s.type[3] = 2
    with pytest.raises(dem.DemError) as e:
        gpu(s)
    assert e.value.code == dem.DEM_ERR_ARG


def test_step_refuses_stale_forces():
    """dem_step takes its first half kick from f and t: after dem_reset (or a
    drift, or new materials) it returns DEM_ERR_STATE and steps nothing until
    the forces are evaluated or declared; then it runs as usual."""
    from paper_1705_03850_amd import dem
    s = W.plain_fcc()
    g = gpu(s)
    g.build_list()
    x0 = g.x.clone()
    with pytest.raises(dem.DemError) as e:
        g.step(5)
    assert e.value.code == dem.DEM_ERR_STATE
    assert torch.equal(g.x, x0)                          # nothing stepped
    g.forces(False)
    g.step(5)
    g.integrate(0)                                       # a drift: the forces are stale again
    with pytest.raises(dem.DemError) as e:
        g.step(1)
    assert e.value.code == dem.DEM_ERR_STATE
    g.build_list()
    g.forces(True)
    g.integrate(1)
    g.step(1)                                            # forces of the last evaluation, kept by the kick
    g.set_materials(s.materials)
    with pytest.raises(dem.DemError) as e:
        g.step(1)
    assert e.value.code == dem.DEM_ERR_STATE
    g.declare_forces()
    g.step(1)
