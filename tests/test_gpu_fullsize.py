"""Parity at the workloads' full sizes, in the launch configuration bench.py
times (4 lanes per particle, 256-thread blocks, resident grid, graph replay).

  * 1e6-sphere settled bed: forces of the first evaluation against the oracle,
    every particle (1e-12 of the sum of its contact-force magnitudes); 10
    steps against the oracle's 10 steps (positions within 1e-9 of the box);
    graph replay of 64-step groups bit for bit equal to launch-by-launch
    stepping over 130 steps.
  * two-level chute (2e5 + 5e5 spheres): the 2-system batch bit for bit
    equal to each system stepped alone.
  * 5e4-sphere adjoint chute: 40 steps against the oracle's dual-number
    tangent (1e-9), with and without list rebuilds between windows, and in
    kept mode; the 200-step flux-loss gradient independent of the window
    length, and kept mode bit for bit equal to recomputation.
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


@pytest.fixture(scope="module")
def bed():
    return W.settled_bed()


def bench_system(s, **kw):
    """DemSystem as bench.py builds it."""
    return dem().DemSystem(s, k_max=32, use_graph=True, chunk=64, **kw)


def by_id(s, arr):
    return arr[np.argsort(s.id, kind="stable")]


def test_full_bed_first_forces_against_oracle(bed):
    s = bed
    assert s.n == 1_000_000
    g = bench_system(s)
    g.prime()
    h = g.host()
    o = O.Oracle(s)
    o.forces(False)
    st = o.state()
    rec = o.records()
    m, _ = o.mass()
    pos = np.empty(s.id.max() + 1, np.int64)
    pos[s.id] = np.arange(s.n)
    scale = m * 9.81
    np.add.at(scale, pos[rec["lo"]], rec["fmag"])
    wall = rec["hi"] < 0
    np.add.at(scale, pos[rec["hi"][~wall]], rec["fmag"][~wall])
    scale = by_id(s, scale)
    F = by_id(s, st["f"])
    T = by_id(s, st["t"])
    r = by_id(s, s.r)
    dF = np.linalg.norm(h["f"] - F, axis=1)
    dT = np.linalg.norm(h["t"] - T, axis=1)
    assert len(rec["lo"]) > 2_000_000          # contacts from the start
    assert np.all(dF <= 1e-12 * scale), (dF / scale).max()
    assert np.all(dT <= 1e-12 * scale * r), (dT / (scale * r)).max()


def test_full_bed_ten_steps_against_oracle(bed):
    s = bed
    g = bench_system(s)
    g.prime()
    g.step(10)
    h = g.host()
    o = O.Oracle(s)
    o.forces(False)
    o.step(10)
    X = by_id(s, o.state()["x"])
    L = s.hi[0] - s.lo[0]
    d = h["x"] - X
    d[:, :2] -= L * np.round(d[:, :2] / L)
    assert np.max(np.abs(d)) <= 1e-9 * L


def test_full_bed_graph_replay_bitwise(bed):
    s = bed
    g1 = bench_system(s)
    g1.prime()
    g1.step(130)                              # two 64-step graphs and two launches
    g2 = dem().DemSystem(s, k_max=32, use_graph=False)
    g2.prime()
    g2.step(130)
    h1, h2 = g1.host(), g2.host()
    for k in ("x", "v", "w", "f", "t"):
        assert np.array_equal(h1[k], h2[k]), k
    assert g1.stats()["builds"] == g2.stats()["builds"]


def test_two_level_chute_batch_equals_separate():
    coarse, fine = W.chute_two_level()
    g = dem().DemSystem([coarse, fine], use_graph=True, chunk=64)
    g.prime()
    g.step(200)
    hb = g.host()
    off = coarse.n
    for k, s in enumerate((coarse, fine)):
        gs = dem().DemSystem(s, use_graph=True, chunk=64)
        gs.prime()
        gs.step(200)
        h = gs.host()
        sel = (hb["id"] >= off) if k else (hb["id"] < off)
        for key in ("x", "v", "w", "f", "t"):
            assert np.array_equal(hb[key][sel], h[key]), (k, key)


def device_by_id(g, a_by_id):
    ids = g.id.long().cpu().numpy()
    return torch.from_numpy(np.ascontiguousarray(a_by_id[ids].T)).to(g.device)


@pytest.mark.parametrize("skin,keep", [(None, False), (0.01e-3, False), (0.01e-3, True)])
def test_full_adjoint_chute_against_oracle_tangent(skin, keep):
    """All 5e4 spheres of the adjoint chute, 40 steps in windows of 8 (the small
    skin forces list rebuilds between windows): the gradient of a linear loss
    in the final x, v, w against the oracle's dual-number tangent, 1e-9."""
    s = W.chute_adjoint()
    nsteps = 40
    rng = np.random.default_rng(31)
    a = rng.normal(size=(s.n, 3)) * 1e3
    b = rng.normal(size=(s.n, 3))
    c = rng.normal(size=(s.n, 3)) * 1e-3
    g = dem().DemSystem(s, skin=skin)
    adj = g.adjoint(nsteps, window=8, keep=keep)
    adj.forward()
    r = adj.backward(device_by_id(g, a), device_by_id(g, b), device_by_id(g, c))
    info = adj.info()
    if skin is not None:
        assert info["rebuilds"] >= 1, info
    got = np.array([r[p][t] for p in ("E", "e", "mu") for t in (0, 1)])
    o = O.Oracle(s, tangent=True)
    o.tan_forces(False)
    o.tan_step(nsteps)
    _, xt = o.tan_vector("x")
    _, vt = o.tan_vector("v")
    _, wt = o.tan_vector("w")
    ref = (np.einsum("ic,ick->k", a[s.id], xt) + np.einsum("ic,ick->k", b[s.id], vt)
           + np.einsum("ic,ick->k", c[s.id], wt))
    for k in range(6):
        assert abs(got[k] - ref[k]) <= 1e-9 * max(abs(ref[k]), 1e-3 * np.abs(ref).max()), (k, got[k], ref[k])


def test_full_adjoint_chute_200_steps():
    """The calibration objective at full size: 200 steps, flux loss.  Windows
    of 20 and of 50 give the same gradient (1e-12) and bit-identical
    initial-state adjoints, kept mode at window 50 the same gradient bit for
    bit; central differences of the rollout (h = 1e-7
    relative) agree within 5e-2 -- at this size the loss has many kinks
    (contact onsets, Coulomb switches), and differences scatter by 1e-4 to
    1e-2 whatever the step, which is why the exact check is the one above."""
    from paper_1705_03850_amd import rollout as R
    s = W.chute_adjoint()
    nsteps = 200
    H0, Lx, Ly = s.meta["H0"], s.hi[0] - s.lo[0], s.hi[1] - s.lo[1]
    target = torch.zeros(20, dtype=torch.float64, device="cuda")
    g = dem().DemSystem(s)
    res = []
    for window, keep in ((20, False), (50, False), (50, True)):
        adj = g.adjoint(nsteps, window=window, keep=keep)
        theta = R.theta_of(s.materials).requires_grad_(True)
        x, v, w = R.rollout(theta, adj, (s.x, s.v, s.w))
        loss = ((R.mass_flux_profile(x, v, R.masses(g), H0, Lx, Ly) - target) ** 2).mean()
        loss.backward()
        res.append((theta.grad.numpy().copy(), adj, adj.initial_by_id(adj.last)))
    g20, g50 = res[0][0], res[1][0]
    assert np.all(np.abs(g20 - g50) <= 1e-12 * np.abs(g20).max())
    for k in ("x0", "v0", "w0"):
        assert np.array_equal(res[0][2][k], res[1][2][k]), k
        assert np.array_equal(res[1][2][k], res[2][2][k]), ("keep", k)
    assert np.array_equal(res[1][0], res[2][0])
    res[2] = None
    th = R.theta_of(s.materials).numpy()
    adj = res[1][1]

    def L(q):
        with torch.no_grad():
            xx, vv, ww = R.rollout(torch.from_numpy(q), adj, (s.x, s.v, s.w))
            return float(((R.mass_flux_profile(xx, vv, R.masses(g), H0, Lx, Ly) - target) ** 2).mean())

    for row in range(3):
        for t in range(2):
            h = 1e-7 * th[row, t]
            qp, qm = th.copy(), th.copy()
            qp[row, t] += h
            qm[row, t] -= h
            fd = (L(qp) - L(qm)) / (2 * h)
            assert abs(fd - g20[row, t]) <= 5e-2 * abs(g20[row, t]), (row, t, fd, g20[row, t])
