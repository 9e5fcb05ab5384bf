"""The silo's static wall surfaces (Sec. 3: a cylinder on a cone, the plug
over the orifice, the orifice's rim) on the GPU against the oracle.

  * a small silo (the paper's shape at a tenth of its size, 4,635 spheres of
    r = 0.4 mm +- 10 % thrown at 0.2 m/s): 300 steps with the orifice closed,
    then the plug removed and the rim enabled on both sides, 300 more steps;
    positions within 1e-9 of the box, and the surface contact histories (the
    same (id, surface) pairs, values within 1e-9 of the box); the first
    forces within 1e-12 of the largest;
  * a silo and its coarse-grain twin (alpha = 2, dt = 2e-6 s) as one batch,
    single-rate and multi-rate, bit for bit equal to each system alone;
  * 4, 8 and 16 lanes per sphere bit for bit alike;
  * the outlet of an insertion event removes what has left through the
    orifice.
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


def dem():
    from paper_1705_03850_amd import dem as d
    return d


def by_id(s, arr):
    return arr[np.argsort(s.id, kind="stable")]


def small_silo(seed=9):
    return W.silo_system(scale=0.1, r=0.4e-3, spread=0.1, speed=0.2, fill=0.5, seed=seed)


def compare(g, s, o, tol=1e-9):
    h = g.host()
    d = h["x"] - by_id(s, o.state()["x"])
    assert np.max(np.abs(d)) <= tol * max(s.hi[a] - s.lo[a] for a in range(3)), np.max(np.abs(d))


def compare_forces(g, s, o):
    h = g.host()
    F = by_id(s, o.state()["f"])
    assert np.max(np.abs(h["f"] - F)) <= 1e-12 * np.max(np.abs(F)), np.max(np.abs(h["f"] - F))


def test_silo_against_oracle_closed_then_open():
    s = small_silo()
    surf = s.meta["surfaces"]
    g = dem().DemSystem(s, surfaces=surf, use_graph=True, chunk=16)
    g.prime()
    o = O.Oracle(s)
    o.set_surfaces(surf)
    o.forces(False)
    compare_forces(g, s, o)
    g.step(300)
    o.step(300)
    compare(g, s, o)
    opened = W.silo_surfaces(scale=0.1, open_orifice=True)
    g.set_surfaces(0, opened)
    o.set_surfaces(opened)
    g.step(300)
    o.step(300)
    compare(g, s, o)
    # the surface contact histories, by (id, surface)
    ids, ks, xi = g.export_surface_history()
    oid, ok_, oxi = o.surface_history()
    order = np.lexsort((ok_, oid))
    assert np.array_equal(ids, oid[order]) and np.array_equal(ks, ok_[order]) and len(ids) >= 10
    edge = max(s.hi[a] - s.lo[a] for a in range(3))
    assert np.max(np.abs(xi - oxi[order])) <= 1e-9 * edge, np.max(np.abs(xi - oxi[order]))
    st = g.stats()
    assert st["wall_contacts"] > 0


@pytest.mark.parametrize("lanes", [8, 16])
def test_silo_lanes_do_not_change_results(lanes):
    """A sphere's surface terms are dealt to its lanes (lane g takes surface
    g) and added in table order, so 4, 8 or 16 lanes give the same silo bit
    for bit, orifice closed and then open: states, surface histories and the
    count of surface contacts."""
    s = small_silo()
    surf = s.meta["surfaces"]
    opened = W.silo_surfaces(scale=0.1, open_orifice=True)
    out = []
    for ln in (4, lanes):
        g = dem().DemSystem(s, surfaces=surf, lanes=ln, use_graph=True, chunk=16)
        g.prime()
        g.step(300)
        g.set_surfaces(0, opened)
        g.step(300)
        out.append((g.host(), g.export_surface_history(), g.stats()["wall_contacts"]))
    (h0, e0, c0), (h1, e1, c1) = out
    for key in ("x", "v", "w", "f", "t"):
        assert np.array_equal(h0[key], h1[key]), key
    for a, b in zip(e0, e1):
        assert np.array_equal(a, b)
    assert len(e0[0]) >= 10 and c0 == c1 > 0


def test_silo_batch_bitwise_and_multirate():
    fine = small_silo(seed=10)
    coarse = W.silo_system(scale=0.1, r=0.8e-3, spread=0.1, speed=0.2, fill=0.5, seed=11, dt=2e-6)
    surf = fine.meta["surfaces"]
    for mr in (False, True):
        g = dem().DemSystem([coarse, fine], surfaces=[surf, surf], use_graph=True, chunk=16)
        if mr:
            g.set_multirate(True)
        g.prime()
        g.step(160)
        hb = [g.host(0), g.host(1)]
        for k, s in enumerate((coarse, fine)):
            gs = dem().DemSystem(s, surfaces=surf, use_graph=True, chunk=16)
            gs.prime()
            gs.step(160 // 2 if (mr and k == 0) else 160)
            h = gs.host(0)
            for key in ("x", "v", "w", "f", "t"):
                assert np.array_equal(hb[k][key], h[key]), (mr, k, key)


def test_outlet_removes_discharged_spheres():
    s = small_silo(seed=12)
    opened = W.silo_surfaces(scale=0.1, open_orifice=True)
    # spheres placed below the orifice as if discharged
    s.x[:40, 0] = np.linspace(-1e-3, 1e-3, 40)
    s.x[:40, 1] = 0.0
    s.x[:40, 2] = -2e-3 - np.arange(40) * 0.9e-3
    g = dem().DemSystem(s, surfaces=opened, capacity=s.n)
    g.prime()
    p = dem().ExchangeParams()
    p.nrm[2] = -1.0
    p.face = -1.0                                   # the top: nothing removed there
    p.slab, p.interval, p.ncell = 1e-3, 0.0, 1
    p.out_nrm[2] = 1.0
    p.out_face = -0.001                             # 1 mm (scaled 1 cm) below the orifice
    fields = torch.zeros((16, 1), dtype=torch.float64, device=g.device)
    budget = torch.zeros(1, dtype=torch.float64, device=g.device)
    _, ins, rem = g.exchange(0, p, fields, budget)
    assert ins == 0 and rem == int(np.sum(s.x[:, 2] < -0.001)) > 0
    assert g.live(0) == s.n - rem
    g.step(10)
