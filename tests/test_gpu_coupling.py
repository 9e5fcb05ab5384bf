"""Coupling of coarse-grain levels (Sec. 2.3, Eq. 7) on the GPU against the
FP64 CPU oracle (oracle/coupling.py and the oracle's external force).

Bars:
  * external force in the force pass: |dF_i| <= 1e-12 (sum_j |F_ij| + |F_ext|);
    100 steps: positions within 1e-9 of the box;
  * cell fields on identical states: counts and maximum speeds bit for bit,
    mass, momentum and solids volume to 1e-13 of the cell's mass (volume),
    stress to 1e-12 of the cell's sum of |terms| / V;
  * controller forces on identical fields: 1e-12 of the largest force;
  * a coupled two-level run (PI on the fine transition layer, P on the coarse
    spheres inside the fine region, every 15 steps): positions of both
    systems within 1e-9 of the largest box edge after four intervals.
"""
import math

import numpy as np
import pytest

import coupling as C
import oracle as O
from paper_1705_03850_amd.inputs import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def dem():
    from paper_1705_03850_amd import dem as d
    return d


def by_id(s, arr):
    return arr[np.argsort(s.id, kind="stable")]


def device_rows(g, a_by_id, offset=0):
    """(n,3) rows by (system-local) id -> device (3, n) in the context's order."""
    ids = g.id.long().cpu().numpy() - offset
    return torch.from_numpy(np.ascontiguousarray(a_by_id[ids].T)).to(g.device)


def test_external_force_in_force_pass_and_steps():
    s = W.chute_adjoint(seed=21, n=3000, Lx=30e-3, Ly=20e-3)
    rng = np.random.default_rng(5)
    fext = rng.normal(0.0, 1e-4, (s.n, 3))                 # by input row
    o = O.Oracle(s)
    o.set_external(fext)
    o.forces(False)
    g = dem().DemSystem(s)
    g.build_list()
    fext_by_id = np.empty_like(fext)
    fext_by_id[s.id] = fext
    g.set_external_force(device_rows(g, fext_by_id))
    g.forces(False)
    h = g.host()
    st = o.state()
    rec = o.records()
    m, _ = o.mass()
    pos = {int(v): k for k, v in enumerate(s.id)}
    scale = m * 9.81 + np.linalg.norm(fext, axis=1)
    for lo, hi, fm in zip(rec["lo"], rec["hi"], rec["fmag"]):
        scale[pos[int(lo)]] += fm
        if hi >= 0:
            scale[pos[int(hi)]] += fm
    dF = np.linalg.norm(h["f"] - by_id(s, st["f"]), axis=1)
    assert np.all(dF <= 1e-12 * by_id(s, scale)), (dF / by_id(s, scale)).max()
    # stepping: the force moves with its sphere through the list rebuilds
    g2 = dem().DemSystem(s, skin=0.02e-3)
    g2.build_list()
    g2.set_external_force(device_rows(g2, fext_by_id))
    g2.forces(False)
    g2.step(100)
    assert g2.stats()["builds"] >= 2
    o2 = O.Oracle(s)
    o2.set_external(fext)
    o2.forces(False)
    o2.step(100)
    d = g2.host()["x"] - by_id(s, o2.state()["x"])
    for ax in (0, 1):
        L = s.hi[ax] - s.lo[ax]
        d[:, ax] -= L * np.round(d[:, ax] / L)
    assert np.max(np.abs(d)) <= 1e-9 * max(s.hi), np.max(np.abs(d))
    # cleared: the plain forces again
    g.set_external_force(None)
    g.forces(False)
    o.set_external(None)
    o.forces(False)
    dF = np.linalg.norm(g.host()["f"] - by_id(s, o.state()["f"]), axis=1)
    assert np.all(dF <= 1e-12 * by_id(s, scale))


# ------------------------------------------------------------- two-level setup

N_FINE, N_COARSE = 20000, 4000
ZB = 0.14                      # top of the fine region (m): the boundary face
PI_GRID = ((0.0, 0.0, 0.13), (0.02, 0.02, 0.01), (2, 1, 1))     # transition layer below the face
P_GRID = ((0.0, 0.0, 0.0), (0.02, 0.02, 0.035), (2, 1, 4))      # cells inside the fine region
NRM, FACE, FADE = (0.0, 0.0, -1.0), -ZB, 1.5                    # inward normal -z: depth = ZB - z
KP, KI, KP_COARSE = 1.0, 200.0, 2000.0


def two_level():
    coarse, fine = W.chute_two_level(n_fine=N_FINE, n_coarse=N_COARSE)
    assert fine.hi[0] >= 0.04 and fine.hi[1] >= 0.02 and coarse.hi[0] >= 0.04
    return coarse, fine


def grid(spec, sys):
    return dem().make_grid(*spec, sys=sys)


def pi_params(sys, interval):
    p = dem().PIParams()
    p.grid = grid(PI_GRID, sys)
    for a in range(3):
        p.nrm[a] = NRM[a]
    p.face, p.kp, p.ki, p.interval, p.fade = FACE, KP, KI, interval, FADE
    return p


def p_params(sys, mass_flow):
    p = dem().PParams()
    p.grid = grid(P_GRID, sys)
    p.kp, p.mass_flow = KP_COARSE, int(mass_flow)
    return p


def load_batch_from_oracles(g, systems, oracles):
    """The oracles' states and histories into a batch context (ids shifted by
    each system's offset)."""
    sts = [o.state() for o in oracles]
    g.load_state(*(np.concatenate([st[k] for st in sts]) for k in ("x", "v", "w", "f", "t")))
    g.reset()
    g.build_list()
    a, b, x, wid, wxi = [], [], [], [], []
    for k, o in enumerate(oracles):
        off = int(g.offsets[k])
        lo, hi, xi = o.history()
        a += [lo + off, hi + off]; b += [hi + off, lo + off]; x += [xi, -xi]
        i, w = o.wall_history()
        wid.append(i + off); wxi.append(w)
    g.import_history(np.concatenate(a), np.concatenate(b), np.concatenate(x), np.concatenate(wid),
                     np.concatenate(wxi))
    g.declare_forces()


def fields_scale(system, orc, spec):
    """Per cell: sum over its spheres and contacts of |1/2 d (x) f| and of m |v'|^2, / V."""
    lo, h, n = spec
    st = orc.state()
    c = C.cell_index(st["x"], lo, h, n)
    ncell = int(np.prod(n))
    sc = np.zeros(ncell)
    f = C.cell_fields(system, orc, lo, h, n)
    m, _ = orc.mass()
    inn = c >= 0
    vp = st["v"][inn] - f["favre"][c[inn]]
    np.add.at(sc, c[inn], m[inn] * np.sum(vp ** 2, axis=1))
    lo_id, hi_id, d, fo = orc.pair_forces()
    pos = {int(q): k for k, q in enumerate(system.id)}
    t = 0.5 * np.linalg.norm(d, axis=1) * np.linalg.norm(fo, axis=1)
    for ids in (lo_id, hi_id):
        cs = c[[pos[int(q)] for q in ids]]
        ok = cs >= 0
        np.add.at(sc, cs[ok], t[ok])
    return f, sc / float(np.prod(h))


def compare_fields(gf, f, scale, what):
    gf = gf.cpu().numpy()
    d = dem()
    assert np.array_equal(gf[d.F_COUNT], f["count"]), what
    assert np.array_equal(gf[d.F_VMAX], f["vmax"]), what
    assert f["count"].sum() > 0
    np.testing.assert_allclose(gf[d.F_MASS], f["mass"], rtol=1e-13, atol=0, err_msg=what)
    np.testing.assert_allclose(gf[d.F_VOLUME], f["volume"], rtol=1e-13, atol=0, err_msg=what)
    for k in range(3):
        atol = 1e-13 * f["mass"] * (np.abs(f["favre"]).max() + 1e-300)
        assert np.all(np.abs(gf[d.F_MOM + k] - f["momentum"][:, k]) <= atol + 1e-300), what
    for a in range(3):
        for b in range(3):
            got = gf[d.F_STRESS + 3 * a + b]
            assert np.all(np.abs(got - f["stress"][:, a, b]) <= 1e-12 * scale + 1e-300), (what, a, b)


@pytest.fixture(scope="module")
def stepped():
    """Both levels after 30 oracle steps (flowing down the 30-degree chute)."""
    systems = two_level()
    oracles = []
    for s in systems:
        o = O.Oracle(s)
        o.forces(False)
        o.step(30)
        oracles.append(o)
    return systems, oracles


def test_cell_fields_against_oracle(stepped):
    systems, oracles = stepped
    g = dem().DemSystem(list(systems))
    load_batch_from_oracles(g, systems, oracles)
    for k, s in enumerate(systems):
        for spec in (PI_GRID, P_GRID, ((0.0, 0.0, 0.0), (s.hi[0] / 3, s.hi[1] / 2, 0.05), (3, 2, 5))):
            f, scale = fields_scale(s, oracles[k], spec)
            gf = g.cell_fields(grid(spec, k))
            compare_fields(gf, f, scale, (s.name, spec))
            # without the stress: the other rows bit for bit, the stress rows untouched
            mf = torch.full_like(gf, float("nan"))
            g.cell_fields(grid(spec, k), stress=False, out=mf)
            d = dem()
            assert torch.equal(mf[:d.F_STRESS], gf[:d.F_STRESS]), (s.name, spec)
            assert torch.isnan(mf[d.F_STRESS:]).all(), (s.name, spec)


def test_controllers_against_oracle(stepped):
    systems, oracles = stepped
    coarse, fine = systems
    g = dem().DemSystem(list(systems))
    load_batch_from_oracles(g, systems, oracles)
    dt = fine.dt
    # PI on the fine system (1) with the coarse system's (0) fields as setpoint
    ff = g.cell_fields(grid(PI_GRID, 1))
    fc = g.cell_fields(grid(PI_GRID, 0))
    integral = torch.full((2,), 0.01, dtype=torch.float64, device=g.device)
    u = g.pi_control(pi_params(1, 15 * dt), ff, fc, integral)
    of = C.cell_fields(fine, oracles[1], *PI_GRID)
    oc = C.cell_fields(coarse, oracles[0], *PI_GRID)
    u_ref, i_ref = C.pi_update(C.normal_stress(oc["stress"], NRM), C.normal_stress(of["stress"], NRM),
                               np.full(2, 0.01), KP, KI, 15 * dt)
    np.testing.assert_allclose(u.cpu().numpy(), u_ref, rtol=1e-11)
    np.testing.assert_allclose(integral.cpu().numpy(), i_ref, rtol=1e-11)
    st = oracles[1].state()
    m, _ = oracles[1].mass()
    F_pi = C.pi_forces(st["x"], st["v"], fine.r, m, dt, *PI_GRID, NRM, FACE, FADE, u_ref, oc["vmax"])
    assert np.count_nonzero(F_pi[:, 2]) > 20
    # P on the coarse system (0) with the fine fields as target, both modes
    pf = g.cell_fields(grid(P_GRID, 1))
    pc = g.cell_fields(grid(P_GRID, 0))
    opf = C.cell_fields(fine, oracles[1], *P_GRID)
    opc = C.cell_fields(coarse, oracles[0], *P_GRID)
    stc = oracles[0].state()
    mc, _ = oracles[0].mass()
    for mass_flow in (False, True):
        g.p_control(p_params(0, mass_flow), pf, pc)
        F_p = C.p_forces(stc["x"], mc, *P_GRID, opf, opc, KP_COARSE, mass_flow)
        # the external forces enter the next force evaluation: compare forces with and without
        g.forces(False)
        h = g.host()
        for o, F in zip(oracles, (F_p, F_pi)):
            o.set_external(F)
            o.forces(False)
        for k, s in enumerate(systems):
            sl = slice(int(g.offsets[k]), int(g.offsets[k + 1]))
            ref = by_id(s, oracles[k].state()["f"])
            rec = oracles[k].records()
            mk, _ = oracles[k].mass()
            Fk = (F_p, F_pi)[k]
            sc = mk * 9.81 + np.linalg.norm(Fk, axis=1)
            pos = {int(v): q for q, v in enumerate(s.id)}
            for lo, hi, fm in zip(rec["lo"], rec["hi"], rec["fmag"]):
                sc[pos[int(lo)]] += fm
                if hi >= 0:
                    sc[pos[int(hi)]] += fm
            dF = np.linalg.norm(h["f"][sl] - ref, axis=1)
            assert np.all(dF <= 1e-12 * by_id(s, sc)), (k, mass_flow, (dF / by_id(s, sc)).max())
        assert np.count_nonzero(F_p) > 20
        for o in oracles:
            o.set_external(None)


def test_coupled_two_level_run_against_oracle():
    """Four coupling intervals of 15 steps: fields of both levels, the PI
    controller on the fine transition layer, the P controller (velocity mode)
    on the coarse spheres inside the fine region, then 15 steps of both levels
    as one batch; the oracle runs the same loop with its own fields."""
    coarse, fine = two_level()
    systems = [coarse, fine]
    dt = fine.dt
    g = dem().DemSystem(systems, use_graph=True, chunk=16)
    g.prime()
    oracles = [O.Oracle(s) for s in systems]
    for o in oracles:
        o.forces(False)
    integral = torch.zeros(2, dtype=torch.float64, device=g.device)
    i_ref = np.zeros(2)
    for it in range(4):
        ff = g.cell_fields(grid(PI_GRID, 1))
        fc = g.cell_fields(grid(PI_GRID, 0))
        g.pi_control(pi_params(1, 15 * dt), ff, fc, integral)
        pf = g.cell_fields(grid(P_GRID, 1))
        pc = g.cell_fields(grid(P_GRID, 0))
        g.p_control(p_params(0, False), pf, pc)
        g.step(15)
        # oracle side
        of = C.cell_fields(fine, oracles[1], *PI_GRID)
        oc = C.cell_fields(coarse, oracles[0], *PI_GRID)
        u_ref, i_ref = C.pi_update(C.normal_stress(oc["stress"], NRM), C.normal_stress(of["stress"], NRM), i_ref,
                                   KP, KI, 15 * dt)
        st = oracles[1].state()
        m, _ = oracles[1].mass()
        oracles[1].set_external(C.pi_forces(st["x"], st["v"], fine.r, m, dt, *PI_GRID, NRM, FACE, FADE, u_ref,
                                            oc["vmax"]))
        opf = C.cell_fields(fine, oracles[1], *P_GRID)
        opc = C.cell_fields(coarse, oracles[0], *P_GRID)
        stc = oracles[0].state()
        mc, _ = oracles[0].mass()
        oracles[0].set_external(C.p_forces(stc["x"], mc, *P_GRID, opf, opc, KP_COARSE, False))
        for o in oracles:
            o.step(15)
    np.testing.assert_allclose(integral.cpu().numpy(), i_ref, rtol=1e-9)
    h = g.host()
    for k, s in enumerate(systems):
        sl = slice(int(g.offsets[k]), int(g.offsets[k + 1]))
        d = h["x"][sl] - by_id(s, oracles[k].state()["x"])
        for ax in (0, 1):
            L = s.hi[ax] - s.lo[ax]
            d[:, ax] -= L * np.round(d[:, ax] / L)
        assert np.max(np.abs(d)) <= 1e-9 * max(s.hi), (k, np.max(np.abs(d)))


def test_coupling_interval_replayed_as_a_graph():
    """The calls of a coupling interval (four field reductions, PI and P)
    captured once in a HIP graph and replayed every interval, with steps,
    host reads and insertion-free eager work in between, give bit for bit
    what the same calls made one by one give on a twin context."""
    coarse, fine = two_level()
    dt = fine.dt
    twins = [dem().DemSystem([coarse, fine], use_graph=True, chunk=16) for _ in range(2)]
    bufs = []
    for g in twins:
        g.prime()
        bufs.append({"pf": torch.empty((16, 2), dtype=torch.float64, device=g.device),
                     "pc": torch.empty((16, 2), dtype=torch.float64, device=g.device),
                     "qf": torch.empty((16, 8), dtype=torch.float64, device=g.device),
                     "qc": torch.empty((16, 8), dtype=torch.float64, device=g.device),
                     "I": torch.full((2,), 0.01, dtype=torch.float64, device=g.device),
                     "u": torch.empty(2, dtype=torch.float64, device=g.device)})
    pi, pp = pi_params(1, 15 * dt), p_params(0, True)

    def couple(g, b):
        g.pi_control(pi, g.cell_fields(grid(PI_GRID, 1), out=b["pf"]), g.cell_fields(grid(PI_GRID, 0), out=b["pc"]),
                     b["I"], b["u"])
        g.p_control(pp, g.cell_fields(grid(P_GRID, 1), stress=False, out=b["qf"]),
                    g.cell_fields(grid(P_GRID, 0), stress=False, out=b["qc"]))

    eager, replayed = twins
    for g, b in zip(twins, bufs):
        with torch.cuda.stream(g.stream):
            couple(g, b)                         # first use: the external forces start at zero
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=replayed.stream):
        couple(replayed, bufs[1])
    for it in range(5):
        for g in twins:
            g.step(15)
        with torch.cuda.stream(eager.stream):
            couple(eager, bufs[0])
        with torch.cuda.stream(replayed.stream):
            graph.replay()
        torch.cuda.synchronize()
        for key in ("pf", "pc", "I", "u"):
            assert torch.equal(bufs[0][key], bufs[1][key]), (it, key)
        for key in ("qf", "qc"):
            assert torch.equal(bufs[0][key][:dem().F_STRESS], bufs[1][key][:dem().F_STRESS]), (it, key)
        h0, h1 = eager.host(), replayed.host()
        for key in ("x", "v", "w", "f", "t"):
            assert np.array_equal(h0[key], h1[key]), (it, key)
    assert eager.stats()["builds"] == replayed.stats()["builds"]


@pytest.mark.parametrize("multirate,graph", [(False, True), (True, True), (False, False)])
def test_step_coupled_equals_the_calls(multirate, graph):
    """dem_step_coupled (three intervals per synchronisation) against the
    same calls made one by one, on twin contexts: with a small skin the list
    is rebuilt inside intervals and groups, so intervals are interrupted and
    issued again; states, PI state, fields and the running sum bit for bit.
    Multi-rate: the coarse level at 2 dt, 16 substeps per interval.  Without
    graphs the coupled context enqueues each interval kernel by kernel."""
    d = dem()
    coarse, fine = (s.copy() for s in two_level())
    rng = np.random.default_rng(17)
    for s in (coarse, fine):                       # moving spheres: rebuilds every 20 steps or so
        s.v = rng.normal(0.0, 0.05, (s.n, 3))
    if multirate:
        coarse.dt = 2 * fine.dt
    interval = 16 if multirate else 15
    skin = [2e-6, 2e-6]
    twins = [d.DemSystem([coarse, fine], skin=skin, use_graph=use, chunk=16) for use in (True, graph)]
    for g in twins:
        if multirate:
            g.set_multirate(True)
        g.prime()
    pi, pp = pi_params(1, interval * fine.dt), p_params(0, True)
    sum_spec = ((0.0, 0.0, 0.10), (0.02, 0.02, 0.01), (2, 1, 1))
    plans = [g.coupling_plan(pi, 0, pp, 1, interval, group=3, sum_grid=grid(sum_spec, 0)) for g in twins]
    eager, coupled = twins
    b = plans[0].buffers
    pf, pc = grid(P_GRID, 1), grid(P_GRID, 0)
    nint = 7
    for _ in range(nint):
        eager.pi_control(pi, eager.cell_fields(grid(PI_GRID, 1), out=b["pi_fine"]),
                         eager.cell_fields(grid(PI_GRID, 0), out=b["pi_coarse"]), b["integral"], b["u"])
        eager.p_control(pp, eager.cell_fields(pf, stress=False, out=b["p_fine"]),
                        eager.cell_fields(pc, stress=False, out=b["p_coarse"]))
        b["sum"][:d.F_STRESS] += eager.cell_fields(grid(sum_spec, 0), stress=False, out=b["sum_tmp"])[:d.F_STRESS]
        eager.step(interval)
    coupled.step_coupled(nint, plans[1])
    torch.cuda.synchronize()
    builds = [g.stats()["builds"] for g in twins]
    assert builds[0] == builds[1] and builds[0] >= 3, builds
    for key in ("integral", "u", "pi_fine", "pi_coarse", "sum"):
        assert torch.equal(plans[0].buffers[key], plans[1].buffers[key]), key
    for key in ("p_fine", "p_coarse"):
        assert torch.equal(plans[0].buffers[key][:d.F_STRESS], plans[1].buffers[key][:d.F_STRESS]), key
    for k in range(2):
        h0, h1 = eager.host(k), coupled.host(k)
        for key in ("x", "v", "w", "f", "t", "id"):
            assert np.array_equal(h0[key], h1[key]), (k, key)
    # and both continue alike
    eager.step(interval)
    coupled.step(interval)
    assert np.array_equal(eager.host()["x"], coupled.host()["x"])


def test_coupling_errors():
    d = dem()
    s = W.plain_fcc()
    g = d.DemSystem(s)
    gr = grid(((0.0, 0.0, 0.0), (0.01, 0.01, 0.01), (2, 2, 2)), 0)
    with pytest.raises(d.DemError) as e:
        g.cell_fields(gr)                        # no neighbour list yet
    assert e.value.code == d.DEM_ERR_STATE
    g.prime()
    bad = grid(((0.0, 0.0, 0.0), (0.0, 0.01, 0.01), (2, 2, 2)), 0)
    with pytest.raises(d.DemError) as e:
        g.cell_fields(bad)
    assert e.value.code == d.DEM_ERR_ARG
    g.cell_fields(gr)
    # drifts without a rebuild until spheres have left their list cells: refused
    s2 = W.plain_fcc()
    s2.v = s2.v * 100.0
    g2 = d.DemSystem(s2)
    g2.prime()
    for _ in range(400):
        g2.integrate(0)
    g2.cell_fields(gr)                           # enqueued; the next synchronising call reports it
    rc, _ = g2.check()
    assert rc == d.DEM_ERR_STATE
    g.set_external_force(torch.zeros((3, s.n), dtype=torch.float64, device=g.device))
    adj = g.adjoint(5, window=5)
    with pytest.raises(d.DemError) as e:
        adj.forward()
    assert e.value.code == d.DEM_ERR_STATE


def test_step_coupled_errors():
    """dem_step_coupled refuses a plan it cannot run, before enqueuing any
    work: the state is left as it was; zero intervals do nothing; a valid
    plan then runs on the same context."""
    d = dem()
    coarse, fine = two_level()
    interval = 15
    pi, pp = pi_params(1, interval * fine.dt), p_params(0, True)
    g = d.DemSystem([coarse, fine], use_graph=True, chunk=16)
    g.build_list()
    plan = g.coupling_plan(pi, 0, pp, 1, interval, group=2)
    with pytest.raises(d.DemError) as e:
        g.step_coupled(1, plan)                  # no forces of the current state yet
    assert e.value.code == d.DEM_ERR_STATE
    g.forces(False)
    before = g.host()

    def refused(plan, nint=1):
        with pytest.raises(d.DemError) as e:
            g.step_coupled(nint, plan)
        return e.value.code

    assert refused(plan, -1) == d.DEM_ERR_ARG
    for field in ("interval_steps", "group", "u", "pi_fine"):
        bad = g.coupling_plan(pi, 0, pp, 1, interval)
        setattr(bad, field, 0 if field in ("interval_steps", "group") else None)
        assert refused(bad) == d.DEM_ERR_ARG, field
    bad = g.coupling_plan(pi, 0, pp, 1, interval, sum_grid=grid(PI_GRID, 0))
    bad.sum_tmp = None
    assert refused(bad) == d.DEM_ERR_ARG
    bad = g.coupling_plan(pi, 0, pp, 1, interval)
    bad.pi.nrm[2] = -0.5                         # not a unit vector
    assert refused(bad) == d.DEM_ERR_ARG
    bad = g.coupling_plan(pi, 0, pp, 1, interval)
    bad.pi_setpoint_sys = 2                      # no such system
    assert refused(bad) == d.DEM_ERR_ARG
    g.step_coupled(0, plan)
    after = g.host()
    for key in ("x", "v", "w", "f", "t"):
        assert np.array_equal(before[key], after[key]), key
    assert g.stats()["steps"] == 0
    g.step_coupled(3, plan)
    assert g.stats()["steps"] == 3 * interval
    # multi-rate: the interval must be a whole number of the coarse level's steps
    c2 = coarse.copy()
    c2.dt = 2 * fine.dt
    m = d.DemSystem([c2, fine], use_graph=True, chunk=16)
    m.set_multirate(True)
    m.prime()
    with pytest.raises(d.DemError) as e:
        m.step_coupled(1, m.coupling_plan(pi, 0, pp, 1, interval))
    assert e.value.code == d.DEM_ERR_ARG
    m.step_coupled(1, m.coupling_plan(pi, 0, pp, 1, 2 * 8))
    assert m.stats()["steps"] == 16


def test_step_coupled_after_launch_changes():
    """The captured interval follows the launch shape: with dem_set_launch
    (4, 8, 16 lanes) between dem_step_coupled calls, the coupled context stays
    bit for bit equal to the same calls made one by one on a twin."""
    d = dem()
    coarse, fine = two_level()
    interval = 15
    twins = [d.DemSystem([coarse, fine], use_graph=True, chunk=16) for _ in range(2)]
    for g in twins:
        g.prime()
    pi, pp = pi_params(1, interval * fine.dt), p_params(0, True)
    plans = [g.coupling_plan(pi, 0, pp, 1, interval, group=2) for g in twins]
    eager, coupled = twins
    b = plans[0].buffers
    for lanes in (4, 8, 16, 0):
        coupled.set_launch(lanes)
        coupled.step_coupled(3, plans[1])
        for _ in range(3):
            eager.pi_control(pi, eager.cell_fields(grid(PI_GRID, 1), out=b["pi_fine"]),
                             eager.cell_fields(grid(PI_GRID, 0), out=b["pi_coarse"]), b["integral"], b["u"])
            eager.p_control(pp, eager.cell_fields(grid(P_GRID, 1), stress=False, out=b["p_fine"]),
                            eager.cell_fields(grid(P_GRID, 0), stress=False, out=b["p_coarse"]))
            eager.step(interval)
        torch.cuda.synchronize()
        for k in range(2):
            h0, h1 = eager.host(k), coupled.host(k)
            for key in ("x", "v", "w", "f", "t"):
                assert np.array_equal(h0[key], h1[key]), (lanes, k, key)
        for key in ("integral", "u"):
            assert torch.equal(plans[0].buffers[key], plans[1].buffers[key]), (lanes, key)
