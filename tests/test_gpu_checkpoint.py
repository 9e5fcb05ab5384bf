"""Checkpoint and resume of the plain state (x, v, w, f, t, history keyed by
ids): a context resumed from a checkpoint continues bit for bit like the one
that was never interrupted -- one system with graph replay and rebuilds, a
two-system batch after an insertion event (free slots, new ids), and a silo
with its orifice opened (the current surfaces and their contact history)."""
import numpy as np
import pytest

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


def same(a, b):
    for k in range(len(a)):
        for key in ("x", "v", "w", "f", "t", "id", "r"):
            assert np.array_equal(a[k][key], b[k][key]), (k, key)


def test_resume_one_system_bitwise():
    s = W.plain_fcc()
    skin = 0.002 * float(s.r.max())              # rebuilds every few steps
    g = dem().DemSystem(s, skin=skin, use_graph=True, chunk=16)
    g.prime()
    g.step(120)
    ck = g.checkpoint()
    g.step(200)
    ref = [g.host(0)]
    g2 = dem().DemSystem.from_checkpoint(ck, skin=skin, use_graph=True, chunk=16)
    g2.step(200)
    same(ref, [g2.host(0)])
    assert g.stats()["builds"] > 10


def test_resume_batch_after_exchange_bitwise():
    import test_gpu_exchange as X
    fine = X.bed(n=2000, seed=27)
    other = X.bed(n=1500, seed=28)
    g = dem().DemSystem([other, fine], capacity=[None, fine.n + 400])
    g.prime()
    g.step(30)
    zf = float(np.quantile(g.host(1)["x"][:, 2], 0.8))
    ev = W.exchange_inputs(fine, zf + 4e-3, 300, seed=11, budget_spheres=10.0, depth=5e-3)
    ev["face"] = -zf
    _, _, ins, rem = X.gpu_event(g, 1, ev)
    assert ins > 0 and rem > 0
    g.step(25)
    ck = g.checkpoint()
    g.step(150)
    ref = [g.host(0), g.host(1)]
    g2 = dem().DemSystem.from_checkpoint(ck)
    assert g2.live(1) == g.live(1)
    g2.step(150)
    same(ref, [g2.host(0), g2.host(1)])


def test_resume_silo_with_surfaces_bitwise():
    s = W.silo_system(scale=0.1, r=0.4e-3, spread=0.1, speed=0.2, fill=0.5, seed=13)
    g = dem().DemSystem(s, surfaces=s.meta["surfaces"], capacity=s.n, use_graph=True, chunk=16)
    g.prime()
    g.step(800)
    g.set_surfaces(0, W.silo_surfaces(scale=0.1, open_orifice=True))
    g.step(60)
    ids, ks, xi = g.export_surface_history()
    assert len(ids) >= 10, len(ids)                          # spheres sliding on the walls
    ck = g.checkpoint()
    g.step(200)
    ref = [g.host(0)]
    g2 = dem().DemSystem.from_checkpoint(ck, use_graph=True, chunk=16)
    a2, k2, x2 = g2.export_surface_history()
    assert np.array_equal(ids, a2) and np.array_equal(ks, k2) and np.array_equal(xi, x2)
    g2.step(200)
    same(ref, [g2.host(0)])
    # without the surface history the run departs from the reference
    g3 = dem().DemSystem.from_checkpoint(dict(ck, surface_history=None), use_graph=True, chunk=16)
    g3.step(200)
    assert not np.array_equal(ref[0]["x"], g3.host(0)["x"])
