"""Reverse mode of the rollout (dem_rollout_*, dem_forces_vjp) on the GPU.

References, none of which shares code with the library's adjoint:
  * the oracle's forward-mode (dual-number) tangent in the six directions
    (E_0, E_1, e_0, e_1, mu_0, mu_1), contracted with the same loss weights:
    agreement to 1e-9 relative;
  * central differences (h = 1e-6 relative) of the GPU's own plain rollout
    (dem_step), which never runs the adjoint kernels: 1e-5 relative;
  * the windowed forward against dem_step: bit for bit, also in kept mode
    (every step's inputs stored, the steps run by the adjoint's own
    evaluation kernel), which must give bit-identical gradients.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_1705_03850_amd.inputs import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

DIRS = [("E", 0), ("E", 1), ("e", 0), ("e", 1), ("mu", 0), ("mu", 1)]


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def dem():
    from paper_1705_03850_amd import dem as d
    return d


def chute(n=600, seed=11, Lx=14e-3, Ly=10e-3):
    return W.chute_adjoint(seed=seed, n=n, Lx=Lx, Ly=Ly)


def with_materials(s, E=None, e=None, mu=None):
    s = s.copy()
    s.materials = [W.Material(E=m.E if E is None else E[t], nu=m.nu, rho=m.rho, e=m.e if e is None else e[t],
                              mu=m.mu if mu is None else mu[t]) for t, m in enumerate(s.materials)]
    return s


def weights(s, seed=3):
    rng = np.random.default_rng(seed)
    # (n, 3) by id; scaled so that the three terms are of similar size
    return rng.normal(size=(s.n, 3)) * 1e3, rng.normal(size=(s.n, 3)), rng.normal(size=(s.n, 3)) * 1e-3


def device_by_id(g, a_by_id):
    """(n, 3) host array indexed by id -> (3, n) device tensor in the current order."""
    ids = g.id.long().cpu().numpy()
    return torch.from_numpy(np.ascontiguousarray(a_by_id[ids].T)).to(g.device)


def oracle_gradient(s, nsteps, a, b, c):
    """d/dtheta of sum a.x + b.v + c.w after nsteps, by the oracle's tangent."""
    o = O.Oracle(s, tangent=True)
    o.tan_forces(False)
    o.tan_step(nsteps)
    _, xt = o.tan_vector("x")
    _, vt = o.tan_vector("v")
    _, wt = o.tan_vector("w")
    ids = s.id
    return (np.einsum("ic,ick->k", a[ids], xt) + np.einsum("ic,ick->k", b[ids], vt)
            + np.einsum("ic,ick->k", c[ids], wt))


def gpu_rollout_grad(s, nsteps, a, b, c, window=20, skin=None, max_windows=0, keep=False):
    g = dem().DemSystem(s, skin=skin)
    adj = g.adjoint(nsteps, window=window, max_windows=max_windows, keep=keep)
    adj.forward()
    r = adj.backward(device_by_id(g, a), device_by_id(g, b), device_by_id(g, c))
    r.update(adj.initial_by_id(r))
    vec = np.array([r[p][t] for p, t in DIRS])
    return vec, r, adj.info(), g


def assert_close(got, ref, rtol, what=""):
    scale = np.abs(ref).max()
    for k, (x, y) in enumerate(zip(got, ref)):
        assert abs(x - y) <= rtol * max(abs(y), 1e-3 * scale), (what, k, x, y, abs(x - y) / max(abs(y), 1e-300))


# ------------------------------------------------------------ forward

@pytest.mark.parametrize("keep", [False, True])
def test_windowed_forward_equals_dem_step(keep):
    """Windows, checkpoints and rebuilds only at window ends change nothing:
    the final state equals dem_step's bit for bit (small skin: several
    rebuilds), and so does the state after 25 more plain steps (the list and
    its history are left as dem_step leaves them)."""
    s = chute(n=800)
    skin = 0.006e-3
    g1 = dem().DemSystem(s, skin=skin)
    g1.prime()
    g1.step(90)
    h1 = g1.host()
    g2 = dem().DemSystem(s, skin=skin)
    adj = g2.adjoint(90, window=7, keep=keep)
    adj.forward()
    h2 = g2.host()
    info = adj.info()
    assert info["rebuilds"] >= 2, info
    assert info["windows"] >= math.ceil(90 / 7)
    for k in ("x", "v", "w", "f", "t"):
        assert np.array_equal(h1[k], h2[k]), k
    g1.step(25)
    g2.step(25)
    h1, h2 = g1.host(), g2.host()
    for k in ("x", "v", "w", "f", "t"):
        assert np.array_equal(h1[k], h2[k]), ("after", k)


@pytest.mark.parametrize("keep", [False, True])
def test_kslots_shrinks_the_workspace_and_changes_nothing(keep):
    """Checkpoints and stored inputs sized for the longest neighbour row
    instead of k_max: the gradients and the final state are bit for bit those
    of the full-size workspace; a bound below the current list's longest row
    is a capacity error before anything runs."""
    d = dem()
    s = chute(n=800)
    skin = 0.006e-3
    rng = np.random.default_rng(3)
    a, b, c = (rng.normal(size=(s.n, 3)) for _ in range(3))
    ref, rr, info, g0 = gpu_rollout_grad(s, 60, a, b, c, window=7, skin=skin, keep=keep)
    assert info["rebuilds"] >= 1, info
    g = d.DemSystem(s, skin=skin)
    g.build_list()
    lo, _ = g.export_neighbors()
    row0 = int(np.bincount(lo).max())
    with pytest.raises(d.DemError) as e:
        g.adjoint(60, window=7, keep=keep, kslots=row0 - 1).forward()
    assert e.value.code == d.DEM_ERR_CAPACITY
    full = g0.adjoint(60, window=7, keep=keep).bytes
    for k in range(row0, 64):
        g = d.DemSystem(s, skin=skin)
        adj = g.adjoint(60, window=7, keep=keep, kslots=k)
        try:
            adj.forward()
            break
        except d.DemError as err:                # a row built during the rollout is longer
            assert err.code == d.DEM_ERR_CAPACITY
    assert adj.bytes < full * (k + 8) / 32.0, (adj.bytes, full, k)
    r = adj.backward(device_by_id(g, a), device_by_id(g, b), device_by_id(g, c))
    r.update(adj.initial_by_id(r))
    got = np.array([r[p][t] for p, t in DIRS])
    assert np.array_equal(got, ref), (got, ref)
    for key in ("x0", "v0", "w0"):
        assert np.array_equal(r[key], rr[key]), key
    h0, h = g0.host(), g.host()
    for key in ("x", "v", "w", "f", "t"):
        assert np.array_equal(h0[key], h[key]), key


# ------------------------------------------------------------ one force evaluation

def test_integrate_vjp_matches_oracle():
    """dem_integrate_vjp for both halves of the step against the oracle's
    reverse mode of kick and drift (pinned on the CPU by the adjoint
    identity): x and w adjoints bit for bit, the others to rounding."""
    d = dem()
    s = chute(n=600)
    g = d.DemSystem(s)
    g.prime()
    o = O.Oracle(s)
    rng = np.random.default_rng(11)
    ys = {k: rng.normal(size=(s.n, 3)) for k in ("x", "v", "w")}       # rows by id
    per = np.argsort(g.id.long().cpu().numpy(), kind="stable")
    for phase in (0, 1):
        back = g.integrate_vjp(phase, *(device_by_id(g, ys[k]) for k in ("x", "v", "w")))
        ref = o.integrate_vjp(phase, *(ys[k][s.id] for k in ("x", "v", "w")))   # input rows
        for k in ("x", "v", "w", "f", "t"):
            got = back[k].cpu().numpy().T[per]
            want = ref[k][np.argsort(s.id, kind="stable")]
            if k in ("x", "w"):
                assert np.array_equal(got, want), (phase, k)
            else:
                np.testing.assert_allclose(got, want, rtol=4e-16 * 8, atol=0, err_msg=f"{phase} {k}")
    with pytest.raises(d.DemError) as e:
        g.integrate_vjp(2, *(device_by_id(g, ys[k]) for k in ("x", "v", "w")))
    assert e.value.code == d.DEM_ERR_ARG


def test_forces_vjp_matches_oracle_tangent():
    s = chute(n=600)
    rng = np.random.default_rng(5)
    fb = rng.normal(size=(s.n, 3))
    tb = rng.normal(size=(s.n, 3)) * 1e3
    o = O.Oracle(s, tangent=True)
    o.tan_forces(False)
    _, ft = o.tan_vector("f")
    _, tt = o.tan_vector("t")
    ref = np.einsum("ic,ick->k", fb[s.id], ft) + np.einsum("ic,ick->k", tb[s.id], tt)
    g = dem().DemSystem(s)
    g.build_list()
    adj = g.adjoint(1, window=1)
    r = adj.forces_vjp(device_by_id(g, fb), device_by_id(g, tb))
    got = np.array([r[p][t] for p, t in DIRS])
    assert np.abs(ref).max() > 0
    assert_close(got, ref, 1e-9, "forces_vjp")


def test_forces_vjp_positions_match_central_differences():
    """dL/dx of L = sum fb.f + tb.t along random directions, against central
    differences of the oracle's forces (double precision, h = 1e-10 m)."""
    s = chute(n=600)
    rng = np.random.default_rng(6)
    fb = rng.normal(size=(s.n, 3))
    tb = rng.normal(size=(s.n, 3)) * 1e3
    g = dem().DemSystem(s)
    g.build_list()
    adj = g.adjoint(1, window=1)
    r = adj.forces_vjp(device_by_id(g, fb), device_by_id(g, tb))
    ids = g.id.long().cpu().numpy()
    xb = np.empty((s.n, 3)); vb = np.empty((s.n, 3)); wb = np.empty((s.n, 3))
    xb[ids] = r["x"].cpu().numpy().T
    vb[ids] = r["v"].cpu().numpy().T
    wb[ids] = r["w"].cpu().numpy().T

    def L(x=None, v=None, w=None):
        q = s.copy()
        if x is not None: q.x = x
        if v is not None: q.v = v
        if w is not None: q.w = w
        o = O.Oracle(q)
        o.forces(False)
        st = o.state()
        return np.sum(fb[q.id] * st["f"]) + np.sum(tb[q.id] * st["t"])

    for name, base, adjv, h in (("x", s.x, xb, 1e-10), ("v", s.v, vb, 1e-7), ("w", s.w, wb, 1e-4)):
        for trial in range(3):
            d = rng.normal(size=base.shape)
            fd = (L(**{name: base + h * d}) - L(**{name: base - h * d})) / (2 * h)
            an = np.sum(adjv[s.id] * d)
            assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-30), (name, fd, an)


# ------------------------------------------------------------ rollouts

@pytest.mark.parametrize("skin,window,keep", [(None, 20, False), (0.006e-3, 7, False), (0.006e-3, 7, True)])
def test_rollout_gradient_matches_oracle_tangent(skin, window, keep):
    s = chute(n=600)
    nsteps = 60
    a, b, c = weights(s)
    ref = oracle_gradient(s, nsteps, a, b, c)
    got, r, info, _ = gpu_rollout_grad(s, nsteps, a, b, c, window=window, skin=skin, keep=keep)
    if skin is not None:
        assert info["rebuilds"] >= 1, info
    assert_close(got, ref, 1e-9, f"rollout skin={skin} window={window} keep={keep}")


def test_window_length_changes_nothing():
    """Window lengths 1, 6 and 40 agree (1e-13; sums split differently), and
    kept mode equals the recomputing mode at the same window bit for bit."""
    s = chute(n=600)
    a, b, c = weights(s, seed=8)
    res = [gpu_rollout_grad(s, 40, a, b, c, window=w, skin=0.006e-3) for w in (1, 6, 40)]
    for got, r, info, _ in res[1:]:
        assert_close(got, res[0][0], 1e-13, "window")
        for k in ("x0", "v0", "w0"):
            assert np.array_equal(r[k], res[0][1][k]), k
    got, r, info, _ = gpu_rollout_grad(s, 40, a, b, c, window=6, skin=0.006e-3, keep=True)
    assert np.array_equal(got, res[1][0])
    for k in ("x0", "v0", "w0"):
        assert np.array_equal(r[k], res[1][1][k]), ("keep", k)


def test_initial_state_adjoint_matches_oracle_tangent():
    """dL/d(x0, v0, w0) along random directions against the oracle's tangent
    seeded along the same initial-state directions, and against central
    differences of the plain GPU rollout (dem_step, none of the adjoint
    kernels) with steps that move positions by ~4e-12 m (larger ones straddle
    contact onsets)."""
    s = chute(n=600)
    nsteps = 30
    a, b, c = weights(s, seed=9)
    _, r, _, _ = gpu_rollout_grad(s, nsteps, a, b, c, window=10, skin=0.006e-3)
    rng = np.random.default_rng(10)
    dirs = {k: rng.normal(size=(s.n, 3)) for k in ("x", "v", "w")}      # by id
    o = O.Oracle(s, tangent=True)
    o.tan_seed_state(0, dx=dirs["x"][s.id])
    o.tan_seed_state(1, dv=dirs["v"][s.id])
    o.tan_seed_state(2, dw=dirs["w"][s.id])
    o.tan_forces(False)
    o.tan_step(nsteps)
    _, xt = o.tan_vector("x")
    _, vt = o.tan_vector("v")
    _, wt = o.tan_vector("w")
    ref = (np.einsum("ic,ick->k", a[s.id], xt) + np.einsum("ic,ick->k", b[s.id], vt)
           + np.einsum("ic,ick->k", c[s.id], wt))
    got = np.array([np.sum(r[k + "0"] * dirs[k]) for k in ("x", "v", "w")])
    assert_close(got, ref[:3], 1e-9, "initial state")

    def L(q):
        g = dem().DemSystem(q)
        g.prime()
        g.step(nsteps)
        h = g.host()
        return np.sum(a * h["x"]) + np.sum(b * h["v"]) + np.sum(c * h["w"])

    for k, (name, h) in enumerate((("x", 5e-12), ("v", 1e-7), ("w", 1e-4))):
        qp, qm = s.copy(), s.copy()
        setattr(qp, name, getattr(s, name) + h * dirs[name][s.id])
        setattr(qm, name, getattr(s, name) - h * dirs[name][s.id])
        fd = (L(qp) - L(qm)) / (2 * h)
        assert abs(fd - got[k]) <= 1e-5 * abs(got[k]), (name, fd, got[k])


def flux_loss_np(x, v, m, H0, Lx, Ly, target, bins=20):
    hgt = H0 / bins
    k = np.floor(x[:, 2] / hgt)
    ok = (k >= 0) & (k < bins)
    flux = np.zeros(bins)
    np.add.at(flux, k[ok].astype(int), m[ok] * v[ok, 0])
    flux /= Lx * Ly * hgt
    return np.mean((flux - target) ** 2)


def test_flux_loss_gradient_matches_central_differences():
    """The chute calibration objective (mass-flux profile in 20 bins) through
    DemRollout and loss.backward(), against central differences of the plain
    GPU rollout at h = 1e-6 relative."""
    from paper_1705_03850_amd import rollout as R
    s = chute(n=800)
    nsteps = 40
    H0, Lx, Ly = s.meta["H0"], s.hi[0] - s.lo[0], s.hi[1] - s.lo[1]
    rng = np.random.default_rng(12)
    target = rng.normal(size=20) * 5.0
    g = dem().DemSystem(s)
    adj = g.adjoint(nsteps, window=10)
    theta = R.theta_of(s.materials).requires_grad_(True)
    init = (s.x, s.v, s.w)
    x, v, w = R.rollout(theta, adj, init)
    m = R.masses(g)
    flux = R.mass_flux_profile(x, v, m, H0, Lx, Ly)
    loss = ((flux - torch.from_numpy(target).to(flux.device)) ** 2).mean()
    loss.backward()
    grad = theta.grad.numpy()
    rho = np.array([mm.rho for mm in s.materials])

    def L(q):
        gg = dem().DemSystem(q)
        gg.prime()
        gg.step(nsteps)
        h = gg.host()
        mass = 4.0 / 3.0 * math.pi * rho[q.type[np.argsort(q.id)]] * h["r"] ** 3
        return flux_loss_np(h["x"], h["v"], mass, H0, Lx, Ly, target)

    th = theta.detach().numpy()
    for row, p in enumerate(("E", "e", "mu")):
        for t in range(2):
            hh = 1e-6 * th[row, t]
            vals = []
            for sgn in (1, -1):
                q = th.copy()
                q[row, t] += sgn * hh
                vals.append(L(with_materials(s, E=q[0], e=q[1], mu=q[2])))
            fd = (vals[0] - vals[1]) / (2 * hh)
            assert abs(fd - grad[row, t]) <= 1e-5 * max(abs(grad[row, t]), 1e-6 * np.abs(grad * th).max() / th[row, t]), \
                (p, t, fd, grad[row, t])


# ------------------------------------------------------------ errors

def test_adjoint_errors():
    d = dem()
    s = chute(n=300)
    g = d.DemSystem(s, skin=0.003e-3)
    adj = g.adjoint(40, window=20, max_windows=2)
    with pytest.raises(d.DemError) as e:
        adj.backward()
    assert e.value.code == d.DEM_ERR_STATE
    with pytest.raises(d.DemError) as e:
        adj.forward()                        # the small skin needs rebuilds: more windows than 2
    assert e.value.code == d.DEM_ERR_CAPACITY
    with pytest.raises(d.DemError) as e:
        g.adjoint(10, window=0)
    assert e.value.code == d.DEM_ERR_ARG
    with pytest.raises(d.DemError) as e:
        g.set_materials([W.Material(E=m.E, nu=m.nu, rho=2 * m.rho, e=m.e, mu=m.mu) for m in s.materials])
    assert e.value.code == d.DEM_ERR_ARG
    batch = d.DemSystem([chute(n=200, seed=1), chute(n=200, seed=2)])
    with pytest.raises(d.DemError) as e:
        batch.adjoint(10)
    assert e.value.code == d.DEM_ERR_ARG


def test_set_materials_changes_the_dynamics_like_a_new_context():
    s = chute(n=400)
    q = with_materials(s, E=[6e6, 9e6], e=[0.8, 0.75], mu=[0.4, 0.35])
    g1 = dem().DemSystem(q)
    g1.prime()
    g1.step(25)
    g2 = dem().DemSystem(s)
    g2.set_materials(q.materials)
    g2.prime()
    g2.step(25)
    h1, h2 = g1.host(), g2.host()
    for k in ("x", "v", "w"):
        assert np.array_equal(h1[k], h2[k])
