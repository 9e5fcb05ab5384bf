"""Pins of the oracle's insertion and deletion (Sec. 2.3: boundary-surface
cells, Favre averaging, SSI insertion; particles leaving the fine region
removed).

  * S-1 inflow: a slab of height h filled evenly with spheres moving across
    the face at speed u: the mass that crosses in time T, counted sphere by
    sphere after moving them, is the budget's increment; outflow adds nothing
    and the budget carries over.
  * S-3 SSI: hand-made cases with a unique answer (spheres on a line, touching
    spheres, a periodic seam, a budget worth exactly one sphere, separation
    along z only); on random candidates, against scipy's pairwise distances:
    no accepted sphere overlaps another or an existing one, and every rejected
    candidate was either over its cell's remaining budget or overlapped an
    existing sphere or one accepted before it; the budget drops by exactly the
    accepted masses.
  * S-4 Favre velocity: momentum over mass, zero in an empty cell.
  * S-5 deletion: the half-space test against hand-placed centres.
  * the whole event on a small bed: kept spheres keep their state and history,
    inserted ones get fresh ids and their cell's velocity, and no accepted
    sphere overlaps any sphere of the new system.
"""
import math

import numpy as np
import pytest
from scipy.spatial.distance import cdist

import insertion as S
import oracle as O
from paper_1705_03850_amd.inputs import workloads as W

BOX = [1.0, 1.0, 1.0]
OPEN = (0, 0, 0)


def test_inflow_budget_counts_crossing_spheres():
    """Spheres of mass m spaced evenly in a slab of height h above the face
    (normal n pointing down into the fine region) all move down at u; after T
    the ones below the face are those that crossed: their mass must equal
    max(0, n . P) / h * T with P the slab's momentum."""
    h, u, T, m = 0.02, 0.5, 0.008, 0.003
    nsph = 400
    z = (np.arange(nsph) + 0.5) * h / nsph          # heights above the face z = 0
    P = np.array([0.0, 0.0, -u * m * nsph])
    crossed = np.count_nonzero(z - u * T < 0.0) * m
    got = S.inflow_budget(np.zeros(1), P[None, :], (0.0, 0.0, -1.0), h, T)
    assert got[0] == pytest.approx(crossed, rel=1e-12)
    # moving up (out of the fine region): nothing; the budget carries over
    got = S.inflow_budget(np.array([0.25]), -P[None, :], (0.0, 0.0, -1.0), h, T)
    assert got[0] == 0.25
    # an oblique normal takes the component along it
    n = np.array([0.6, 0.0, -0.8])
    got = S.inflow_budget(np.zeros(1), np.array([[1.0, 5.0, -2.0]]), n, 0.5, 2.0)
    assert got[0] == pytest.approx((0.6 * 1.0 + 0.8 * 2.0) / 0.5 * 2.0, rel=1e-14)


def test_sphere_mass():
    assert S.sphere_mass(1.0, 3.0 / (4.0 * math.pi)) == pytest.approx(1.0, rel=1e-15)
    assert S.sphere_mass(2e-3, 2500.0) == pytest.approx(2500.0 * 4.0 / 3.0 * math.pi * 8e-9, rel=1e-15)


def line(xs, r=0.1, z=0.5):
    return np.array([[0.25 + x, 0.5, z] for x in xs]), np.full(len(xs), r)


def accept(cx, cr, ex=None, er=None, budget=(1e9,), cell=None, rho=1.0, box=BOX, per=OPEN):
    ex = np.zeros((0, 3)) if ex is None else ex
    er = np.zeros(0) if er is None else er
    cell = np.zeros(len(cx), np.int32) if cell is None else np.asarray(cell)
    return S.ssi_accept(ex, er, cx, cr, np.full(len(cx), rho), cell, np.array(budget, float), box, per)


def test_ssi_line_in_order():
    # r = 0.1: centres 0, 0.15, 0.25, 0.4 -> the second overlaps the first, the
    # third clears the first, the fourth overlaps the third
    cx, cr = line([0.0, 0.15, 0.25, 0.4])
    acc, _ = accept(cx, cr)
    assert acc.tolist() == [1, 0, 1, 0]
    # the order decides: reversed, the last (0.0) clears the accepted 0.25
    acc, _ = accept(cx[::-1].copy(), cr)
    assert acc.tolist() == [1, 0, 1, 0]
    # a rejected candidate blocks nothing: 0.15 rejected, 0.3 clears 0.0 and is
    # 0.15 from 0.15 (which would overlap) -> accepted
    cx, cr = line([0.0, 0.15, 0.3])
    acc, _ = accept(cx, cr)
    assert acc.tolist() == [1, 0, 1]


def test_ssi_touching_is_no_overlap():
    cx, cr = line([0.0, 0.25])
    cr = np.array([0.125, 0.125])                      # exactly touching: 0.25 = 0.125 + 0.125
    acc, _ = accept(cx, cr)
    assert acc.tolist() == [1, 1]
    cr = np.array([0.125, 0.125 + 2.0 ** -20])
    acc, _ = accept(cx, cr)
    assert acc.tolist() == [1, 0]


def test_ssi_existing_spheres_block():
    ex = np.array([[0.5, 0.5, 0.5]])
    er = np.array([0.2])
    cx = np.array([[0.5, 0.5, 0.75], [0.5, 0.5, 0.85], [0.5, 0.81, 0.5]])
    acc, _ = accept(cx, np.full(3, 0.1), ex, er)
    assert acc.tolist() == [0, 1, 1]
    # separation along z only: a mistake that drops dz would accept nothing here
    cx = np.array([[0.5, 0.5, 0.2], [0.5, 0.5, 0.8]])
    acc, _ = accept(cx, np.full(2, 0.1))
    assert acc.tolist() == [1, 1]


def test_ssi_periodic_seam():
    cx = np.array([[0.05, 0.5, 0.5], [0.97, 0.5, 0.5]])
    cr = np.full(2, 0.05)
    assert accept(cx, cr)[0].tolist() == [1, 1]                              # open box: 0.92 apart
    assert accept(cx, cr, per=(1, 0, 0))[0].tolist() == [1, 0]               # periodic: 0.08 apart
    cy = cx[:, [1, 0, 2]]
    assert accept(cy, cr, per=(0, 1, 0))[0].tolist() == [1, 0]
    assert accept(cy, cr, per=(1, 0, 0))[0].tolist() == [1, 1]


def test_ssi_budget_per_cell():
    r, rho = 0.05, 1000.0
    m = S.sphere_mass(r, rho)
    cx = np.array([[0.1, 0.1, 0.5], [0.4, 0.1, 0.5], [0.7, 0.1, 0.5], [0.1, 0.7, 0.5], [0.4, 0.7, 0.5]])
    cell = [0, 0, 0, 1, 1]
    acc, left = accept(cx, np.full(5, r), budget=(m, 2.5 * m), cell=cell, rho=rho)
    # cell 0 affords exactly one sphere (m <= m), cell 1 two
    assert acc.tolist() == [1, 0, 0, 1, 1]
    assert left[0] == 0.0
    assert left[1] == pytest.approx(0.5 * m, rel=1e-12)
    # a budget a hair under one sphere affords none
    acc, left = accept(cx[:1], np.full(1, r), budget=(m * (1 - 1e-15),), rho=rho)
    assert acc.tolist() == [0]


def random_case(seed, ncand=600, nex=150, ncell=4):
    rng = np.random.default_rng(seed)
    ex = rng.uniform(0, 1, (nex, 3))
    er = rng.uniform(0.01, 0.03, nex)
    cx = rng.uniform(0, 1, (ncand, 3))
    cr = rng.uniform(0.01, 0.03, ncand)
    rho = rng.uniform(500, 3000, ncand)
    cell = rng.integers(0, ncell, ncand)
    budget = rng.uniform(0.3, 1.0, ncell) * 60 * S.sphere_mass(0.02, 1500.0)
    return ex, er, cx, cr, rho, cell, budget


def pdist_min_image(a, b, per):
    d = a[:, None, :] - b[None, :, :]
    for ax in range(3):
        if per[ax]:
            d[..., ax] -= np.round(d[..., ax])
    return np.sqrt((d * d).sum(-1))


@pytest.mark.parametrize("per", [OPEN, (1, 1, 0)])
@pytest.mark.parametrize("seed", [11, 12])
def test_ssi_random_is_valid_and_maximal(seed, per):
    ex, er, cx, cr, rho, cell, budget = random_case(seed)
    acc, left = S.ssi_accept(ex, er, cx, cr, rho, cell, budget, BOX, per)
    a = acc.astype(bool)
    assert 0 < a.sum() < len(a)
    if per == OPEN:
        dcc = cdist(cx, cx)
        dce = cdist(cx, ex)
    else:
        dcc = pdist_min_image(cx, cx, per)
        dce = pdist_min_image(cx, ex, per)
    scc = cr[:, None] + cr[None, :]
    sce = cr[:, None] + er[None, :]
    eps = 1e-12
    # valid: no overlap among the accepted, nor with an existing sphere
    acc_idx = np.flatnonzero(a)
    sub = dcc[np.ix_(acc_idx, acc_idx)] - scc[np.ix_(acc_idx, acc_idx)]
    np.fill_diagonal(sub, 1.0)
    assert sub.min() > -eps
    assert (dce[a] - sce[a]).min() > -eps
    # the budget dropped by exactly the accepted masses and stayed >= 0
    masses = np.array([S.sphere_mass(cr[k], rho[k]) for k in range(len(cr))])
    for c in range(len(budget)):
        assert left[c] == pytest.approx(budget[c] - masses[a & (cell == c)].sum(), rel=0, abs=1e-12 * budget[c])
        assert left[c] >= 0.0
    # maximal: replay the budget; every rejection has a reason
    rem = budget.copy()
    for k in range(len(cr)):
        if a[k]:
            rem[cell[k]] -= masses[k]
            continue
        over_budget = masses[k] > rem[cell[k]] * (1 + 1e-12)
        blocked_ex = np.any(dce[k] < sce[k] + eps)
        earlier = acc_idx[acc_idx < k]
        blocked_acc = np.any(dcc[k, earlier] < scc[k, earlier] + eps)
        assert over_budget or blocked_ex or blocked_acc, k


def test_favre_velocity():
    m = np.array([2.0, 0.0, 0.5])
    p = np.array([[1.0, -2.0, 4.0], [3.0, 3.0, 3.0], [0.5, 0.0, -0.25]])
    v = S.favre_velocity(m, p)
    assert v.tolist() == [[0.5, -1.0, 2.0], [0.0, 0.0, 0.0], [1.0, 0.0, -0.5]]


def test_outside_half_space():
    x = np.array([[0.0, 0.0, 0.049], [0.0, 0.0, 0.05], [5.0, -3.0, 0.051]])
    assert S.outside(x, (0.0, 0.0, 1.0), 0.05).tolist() == [True, False, False]
    # inward normal pointing down: a top face at z = 0.2 is n . x >= -0.2
    x = np.array([[0.0, 0.0, 0.19], [0.0, 0.0, 0.21]])
    assert S.outside(x, (0.0, 0.0, -1.0), -0.2).tolist() == [False, True]


def small_bed():
    return W.settled_bed(seed=21, n=300, footprint=12e-3, cache=False)


def test_exchange_event_on_small_bed():
    s = small_bed()
    o = O.Oracle(s)
    o.forces(False)
    o.step(30)
    zs = o.state()["x"][:, 2]
    top = float(np.quantile(zs, 0.9))
    rng = np.random.default_rng(5)
    k = 80
    cand_x = np.column_stack([rng.uniform(0, 12e-3, k), rng.uniform(0, 12e-3, k),
                              rng.uniform(top - 2e-3, top + 3e-3, k)])
    cand_r = rng.uniform(0.9e-3, 1.1e-3, k)
    cand_t = np.zeros(k, np.int32)
    cand_c = rng.integers(0, 2, k)
    cm = np.array([1.0, 0.0])
    cp = np.array([[0.01, 0.0, -0.2], [0.0, 0.0, 0.0]])
    budget = np.array([1e-4, 1e-4])
    hist_before = o.history()
    st = o.state()
    new, o2, acc, left, keep, _ = S.exchange(s, o, (0.0, 0.0, -1.0), -top, cand_x, cand_r, cand_t, cand_c, budget,
                                             cm, cp, id_base=int(s.id.max()) + 1)
    na = int(acc.sum())
    assert 0 < na < k and 0 < keep.sum() < s.n
    assert new.n == int(keep.sum()) + na
    assert np.all(st["x"][keep][:, 2] <= top)
    np.testing.assert_array_equal(new.x[: keep.sum()], st["x"][keep])
    np.testing.assert_array_equal(new.id[keep.sum():], np.arange(na) + s.id.max() + 1)
    v_new = new.v[keep.sum():]
    c_new = cand_c[acc.astype(bool)]
    assert np.all(v_new[c_new == 0] == [0.01, 0.0, -0.2]) and np.all(v_new[c_new == 1] == 0.0)
    # history of kept pairs carried, of removed ones dropped
    kept = set(s.id[keep].tolist())
    lo, hi, xi = hist_before
    want = {(int(p), int(q)): x for p, q, x in zip(lo, hi, xi) if p in kept and q in kept}
    lo2, hi2, xi2 = o2.history()
    assert {(int(p), int(q)) for p, q in zip(lo2, hi2)} == set(want)
    for p, q, x in zip(lo2, hi2, xi2):
        assert np.array_equal(x, want[(int(p), int(q))])
    # no accepted sphere overlaps any other sphere of the new system
    d = cdist(new.x, new.x)
    d[:, :] -= new.r[:, None] + new.r[None, :]
    np.fill_diagonal(d, 1.0)
    assert d[keep.sum():].min() > -1e-15
