"""Insertion and deletion at the boundary of the fine region (Sec. 2.3) on
the GPU against the oracle (oracle/insertion.py).

  * one event from the same state on both sides: the accepted flags and the
    remaining budget bit for bit, the removed and inserted spheres, the new
    spheres' positions, velocities and ids bit for bit; then forces and 100
    steps (positions within 1e-9 of the box), the kept pairs' history carried;
  * several events between stretches of steps, each side on its own;
  * in a two-system batch the other system is untouched (bit for bit against
    the same batch without the event);
  * edge cases: no candidates, every candidate blocked, every sphere removed
    and spheres inserted into the empty system, a full system
    (DEM_ERR_CAPACITY, nothing changed), a bad candidate (DEM_ERR_ARG,
    nothing changed), stale forces (DEM_ERR_STATE), and stepping refused until
    the forces of the new state are evaluated.
"""
import numpy as np
import pytest

import insertion as S
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


def bed(n=3000, fp=20e-3, seed=21):
    return W.settled_bed(seed=seed, n=n, footprint=fp, cache=False)


def params(ev):
    p = dem().ExchangeParams()
    for a in range(3):
        p.nrm[a] = ev["nrm"][a]
    p.face, p.slab, p.interval, p.ncell = ev["face"], ev["slab"], ev["interval"], ev["ncell"]
    return p


def gpu_event(g, sys, ev, budget=None):
    fields = torch.from_numpy(ev["fields"]).to(g.device)
    if budget is None:
        budget = torch.from_numpy(ev["budget"].copy()).to(g.device)
    acc, ins, rem = g.exchange(sys, params(ev), fields, budget, ev["cand_x"], ev["cand_r"], ev["cand_type"],
                               ev["cand_cell"])
    return acc.cpu().numpy(), budget, ins, rem


def oracle_event(s, o, ev, id_base, budget=None, fext=None):
    b = ev["budget"] if budget is None else budget
    b = S.inflow_budget(b, ev["fields"][W.ROW_MOM:W.ROW_MOM + 3].T, ev["nrm"], ev["slab"], ev["interval"])
    return S.exchange(s, o, ev["nrm"], ev["face"], ev["cand_x"], ev["cand_r"], ev["cand_type"], ev["cand_cell"], b,
                      ev["fields"][W.ROW_MASS], ev["fields"][W.ROW_MOM:W.ROW_MOM + 3].T, id_base, fext)


def settle(s, steps=60):
    o = O.Oracle(s)
    o.forces(False)
    o.step(steps)
    return o


def load(g, o):
    import test_gpu_parity as T
    T.load_oracle_state(g, None, o)


def top_of(o, q=0.8):
    return float(np.quantile(o.state()["x"][:, 2], q))


def assert_positions(h, s2, o2, tol=1e-9):
    d = h["x"] - by_id(s2, o2.state()["x"])
    for ax in (0, 1):
        L = s2.hi[ax] - s2.lo[ax]
        d[:, ax] -= L * np.round(d[:, ax] / L)
    assert np.max(np.abs(d)) <= tol * max(s2.hi), np.max(np.abs(d))


def test_event_matches_oracle_bit_for_bit():
    s = bed()
    o = settle(s)
    zf = top_of(o)
    # candidates in a slab across the face: above it, where the removal empties the bed
    ev = W.exchange_inputs(s, zf + 4e-3, 400, seed=7, budget_spheres=20.0, depth=5e-3)
    ev["face"] = -zf
    g = dem().DemSystem(s, capacity=s.n + 600)
    load(g, o)
    acc, budget, ins, rem = gpu_event(g, 0, ev)
    s2, o2, acc_ref, left_ref, keep, _ = oracle_event(s, o, ev, int(s.id.max()) + 1)
    assert acc.tolist() == acc_ref.tolist()
    assert ins == int(acc_ref.sum()) > 10 and rem == int((~keep).sum()) > 10
    assert np.array_equal(budget.cpu().numpy(), left_ref)
    assert g.live(0) == s2.n == g.live_counts[0]
    h = g.host(0)
    assert np.array_equal(h["id"], np.sort(s2.id))
    new = h["id"] > s.id.max()
    ref_x, ref_v = by_id(s2, s2.x), by_id(s2, s2.v)
    assert np.array_equal(h["x"][new], ref_x[new]) and np.array_equal(h["v"][new], ref_v[new])
    assert np.array_equal(h["x"][~new], ref_x[~new])
    assert np.all(h["w"][new] == 0.0)
    # the kept pairs' history: the GPU's contacts against the oracle's carried history
    a, b, xi = g.export_contacts()
    lo, hi, xo = o2.history()
    ref = {(int(p), int(q)): x for p, q, x in zip(lo, hi, xo)}
    for p, q, x in zip(a, b, xi):
        if p < q and (int(p), int(q)) in ref:
            np.testing.assert_allclose(x, ref[(int(p), int(q))], rtol=0, atol=1e-15)
    # then the same forces and steps
    o2.forces(False)
    g.step(100)
    o2.step(100)
    assert_positions(g.host(0), s2, o2)


def test_repeated_events_against_oracle():
    s = bed(seed=22)
    o = settle(s)
    zf = top_of(o, 0.85)
    g = dem().DemSystem(s, capacity=s.n + 1500, use_graph=True, chunk=16)
    load(g, o)
    bud_g = torch.from_numpy(np.zeros(4)).to(g.device)
    bud_o = np.zeros(4)
    s_cur, o_cur = s, o
    for k in range(4):
        ev = W.exchange_inputs(s, zf + 4e-3, 300, seed=30 + k, budget_spheres=4.0, inflow_mass=5e-2, depth=5e-3)
        ev["face"] = -zf
        acc, bud_g, ins, rem = gpu_event(g, 0, ev, budget=bud_g)
        # new ids follow the largest live id before the event
        s_cur, o_cur, acc_ref, bud_o, keep, _ = oracle_event(s_cur, o_cur, ev, int(s_cur.id.max()) + 1, budget=bud_o)
        assert acc.tolist() == acc_ref.tolist(), k
        assert np.array_equal(bud_g.cpu().numpy(), bud_o), k
        assert ins == int(acc_ref.sum()) and rem == int((~keep).sum()), k
        o_cur.forces(False)
        g.step(48)
        o_cur.step(48)
        assert_positions(g.host(0), s_cur, o_cur)
    assert g.live(0) == s_cur.n


def test_other_system_of_batch_untouched():
    s = bed(n=2000, seed=23)
    other = bed(n=1500, seed=24)
    o = settle(s)
    zf = top_of(o)
    ev = W.exchange_inputs(s, zf + 4e-3, 200, seed=9, budget_spheres=4.0, depth=5e-3)
    ev["face"] = -zf
    runs = []
    for event in (False, True):
        g = dem().DemSystem([other, s], capacity=[None, s.n + 300])
        g.prime()
        g.step(20)
        if event:
            acc, _, ins, rem = gpu_event(g, 1, ev)
            assert ins > 0 and rem > 0
        g.step(40)
        runs.append(g.host(0))
    for key in ("x", "v", "w", "f", "t", "id"):
        assert np.array_equal(runs[0][key], runs[1][key]), key


def test_events_in_a_multirate_batch():
    """Insertion events on the fine system of a multi-rate batch (the coarse
    system at 2 dt, 16 substeps per interval): the fine system evolves bit
    for bit as it does alone with the same events, the coarse one as it does
    alone with 8 steps per interval."""
    fine = bed(n=2000, seed=26)
    coarse = bed(n=1500, seed=27).copy()
    coarse.dt = 2 * fine.dt
    zf = float(np.quantile(fine.x[:, 2], 0.8))
    g = dem().DemSystem([coarse, fine], capacity=[None, fine.n + 400], use_graph=True, chunk=16)
    g.set_multirate(True)
    g.prime()
    gf = dem().DemSystem(fine, capacity=fine.n + 400, use_graph=True, chunk=16)
    gf.prime()
    gc = dem().DemSystem(coarse, use_graph=True, chunk=16)
    gc.prime()
    total = 0
    for k in range(3):
        g.step(16)
        gf.step(16)
        gc.step(8)
        ev = W.exchange_inputs(fine, zf + 4e-3, 200, seed=40 + k, budget_spheres=4.0, depth=5e-3)
        ev["face"] = -zf
        acc_b, bud_b, ins_b, rem_b = gpu_event(g, 1, ev)
        acc_a, bud_a, ins_a, rem_a = gpu_event(gf, 0, ev)
        assert acc_b.tolist() == acc_a.tolist() and (ins_b, rem_b) == (ins_a, rem_a), k
        assert torch.equal(bud_a, bud_b), k
        total += ins_a + rem_a
    assert total > 0
    g.step(32)
    gf.step(32)
    gc.step(16)
    hb, ha = g.host(1), gf.host(0)
    for key in ("x", "v", "w", "f", "t"):
        assert np.array_equal(hb[key], ha[key]), key
    hb, ha = g.host(0), gc.host(0)
    for key in ("x", "v", "w", "f", "t", "id"):
        assert np.array_equal(hb[key], ha[key]), ("coarse", key)


def test_edge_cases():
    d = dem()
    s = bed(n=1500, seed=25)
    o = settle(s, 30)
    zf = top_of(o)
    ztop = float(o.state()["x"][:, 2].max()) + float(s.r.max())
    g = d.DemSystem(s, capacity=s.n + 50)
    load(g, o)
    live0 = g.live(0)
    # more accepted than free slots (50): DEM_ERR_CAPACITY, nothing changed
    before = g.host(0)
    ev = W.exchange_inputs(s, ztop + 6e-3, 600, seed=4, budget_spheres=500.0, depth=5e-3)
    ev["face"] = -(ztop + 20e-3)                     # no removal
    b0 = torch.from_numpy(ev["budget"].copy()).to(g.device)
    with pytest.raises(d.DemError) as e:
        gpu_event(g, 0, ev, budget=b0)
    assert e.value.code == d.DEM_ERR_CAPACITY and "free slots" in str(e.value)
    assert np.array_equal(b0.cpu().numpy(), ev["budget"])
    after = g.host(0)
    assert all(np.array_equal(before[k], after[k]) for k in before)
    assert g.live(0) == live0
    g.step(10)                                       # still usable
    # no candidates: removal only
    ev = W.exchange_inputs(s, zf, 0, seed=1)
    acc, budget, ins, rem = gpu_event(g, 0, ev)
    assert ins == 0 and rem > 0 and g.live(0) == live0 - rem == g.host(0)["id"].size
    assert np.array_equal(budget.cpu().numpy(),
                          S.inflow_budget(ev["budget"], ev["fields"][2:5].T, ev["nrm"], ev["slab"], ev["interval"]))
    # every candidate on top of a kept sphere: none accepted, budget only topped up
    h = g.host(0)
    ev = W.exchange_inputs(s, zf, 40, seed=2, budget_spheres=50.0)
    pick = np.argsort(h["x"][:, 2])[-40:]
    ev["cand_x"] = h["x"][pick].copy()
    acc, budget, ins, rem = gpu_event(g, 0, ev)
    assert ins == 0 and not acc.any()
    # a bad candidate (radius above r_max): DEM_ERR_ARG, nothing changed
    before = g.host(0)
    ev = W.exchange_inputs(s, zf, 20, seed=3, budget_spheres=50.0)
    ev["cand_r"][5] = 2.0 * float(s.r.max())
    b0 = torch.from_numpy(ev["budget"].copy()).to(g.device)
    with pytest.raises(d.DemError) as e:
        gpu_event(g, 0, ev, budget=b0)
    assert e.value.code == d.DEM_ERR_ARG
    assert np.array_equal(b0.cpu().numpy(), ev["budget"])
    after = g.host(0)
    assert all(np.array_equal(before[k], after[k]) for k in before)
    # the call leaves the forces of the new state: dem_forces gives the same bits
    ev = W.exchange_inputs(s, zf + 4e-3, 100, seed=5, budget_spheres=20.0, depth=5e-3)
    ev["face"] = -zf
    acc, budget, ins, rem = gpu_event(g, 0, ev)
    assert ins > 0
    h1 = g.host(0)
    g.forces(False)
    h2 = g.host(0)
    assert np.array_equal(h1["f"], h2["f"]) and np.array_equal(h1["t"], h2["t"])
    # the exchange needs the forces of the current state
    g.integrate(0)
    fields = torch.from_numpy(ev["fields"]).to(g.device)
    with pytest.raises(d.DemError) as e:
        g.exchange(0, params(ev), fields, budget)
    assert e.value.code == d.DEM_ERR_STATE
    g.bin()
    g.neighbors()
    g.forces(False)
    g.exchange(0, params(ev), fields, budget)
    g.step(5)


def test_empty_system_and_refill():
    d = dem()
    s = bed(n=1200, seed=26)
    o = settle(s, 20)
    g = d.DemSystem(s, capacity=s.n + 200)
    load(g, o)
    ev = W.exchange_inputs(s, 0.0, 0, seed=1)
    ev["face"] = 1.0                                  # x . (0, 0, -1) < 1 everywhere: remove all
    acc, budget, ins, rem = gpu_event(g, 0, ev)
    assert rem == s.n and g.live(0) == 0
    g.step(5)
    assert g.stats()["slots"] == 0
    # refill from the bottom: candidates near the wall, against the oracle's SSI on an empty system
    ev = W.exchange_inputs(s, 6e-3, 300, seed=8, budget_spheres=30.0, depth=5e-3)
    acc, budget, ins, rem = gpu_event(g, 0, ev)
    b = S.inflow_budget(ev["budget"], ev["fields"][2:5].T, ev["nrm"], ev["slab"], ev["interval"])
    rho = np.full(300, s.materials[0].rho)
    ref, left = S.ssi_accept(np.zeros((0, 3)), np.zeros(0), ev["cand_x"], ev["cand_r"], rho, ev["cand_cell"], b,
                             [s.hi[a] - s.lo[a] for a in range(3)], s.periodic)
    assert acc.tolist() == ref.tolist() and ins == int(ref.sum()) > 0 and rem == 0
    assert np.array_equal(budget.cpu().numpy(), left)
    assert g.live(0) == ins
    g.step(20)
    rc, info = g.check()
    assert rc == d.DEM_OK


def test_event_that_changes_nothing_keeps_the_run_bitwise():
    s = bed(n=1500, seed=29)
    runs = []
    for event in (False, True):
        g = dem().DemSystem(s, capacity=s.n + 10, use_graph=True, chunk=16)
        g.prime()
        g.step(40)
        if event:
            ev = W.exchange_inputs(s, 1.0, 0, seed=1)
            ev["face"] = -1.0                       # region z <= 1 m: nothing removed
            ev["fields"][:] = 0.0                   # no inflow
            acc, budget, ins, rem = gpu_event(g, 0, ev)
            assert ins == 0 and rem == 0 and g.live(0) == s.n
        g.step(60)
        runs.append(g.host(0))
    for key in ("x", "v", "w", "f", "t", "id"):
        assert np.array_equal(runs[0][key], runs[1][key]), key
