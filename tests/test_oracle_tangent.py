"""Pins of the oracle's forward-mode (dual-number) derivatives with respect to
the per-type material parameters E, e and mu.

The tangent directions are (E_0, E_1, e_0, e_1, mu_0, mu_1).  Every pin is a
derivative that follows from the contact law of Sec. 2.1 (Eq. 3-6) by hand or
from a closed form of the dynamics, or a central difference of the oracle's
own double-precision run; none re-uses the dual-number code.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_1705_03850_amd.inputs import workloads as W
from systems import e_star, mat, sphere_mass, sphere_on_wall, two_spheres

G0 = W.G0
DIR = {"E0": 0, "E1": 1, "e0": 2, "e1": 3, "mu0": 4, "mu1": 5}


def beta_of(e):
    return math.log(e) / math.sqrt(math.log(e) ** 2 + math.pi ** 2)


def dbeta_de(e):
    """d beta / d e for beta = ln e / sqrt(ln^2 e + pi^2)."""
    L = math.log(e)
    return math.pi ** 2 / (e * (L * L + math.pi ** 2) ** 1.5)


def test_dbeta_de_closed_form():
    """The derivative of the damping factor of Eq. 6 at e = 0.9 (0.353081791)."""
    assert abs(dbeta_de(0.9) - 0.353081791) < 1e-9
    h = 1e-5
    fd = (beta_of(0.9 + h) - beta_of(0.9 - h)) / (2 * h)
    assert abs(fd - dbeta_de(0.9)) < 1e-9


def overlapping_pair(m1, m2, delta=2e-6, v_rel=0.3, vt=0.0):
    s = two_spheres(v_rel, m1=m1, m2=m2, gap=-delta)
    s.v[0, 1] = vt
    return s


@pytest.mark.parametrize("mixed", [False, True])
def test_normal_force_tangent_matches_hand_derivative(mixed):
    """dF_n/dE and dF_n/de from Eq. 3 and 6 differentiated by hand:
    F_n = k_n delta - g_n v_n with k_n = 4/3 E* sqrt(R delta),
    g_n = -beta(e) sqrt(5 m* k_n); for a pair of two types e = (e_0 + e_1)/2 and
    dE*/dE_0 = E*^2 (1 - nu_0^2) / E_0^2."""
    ma = mat(E=5e6, nu=0.25, e=0.9)
    mb = mat(E=1e7, nu=0.3, e=0.7) if mixed else ma
    s = overlapping_pair(ma, mb)
    o = O.Oracle(s, tangent=True)
    o.tan_forces(False)
    f, ft = o.tan_vector("f")
    # particle 0 sits at -x: n = (-1, 0, 0), F_x(0) = -f_n
    r = 1e-3
    delta = 2e-6
    m = sphere_mass(r, 2500.0)
    R, mstar = r / 2, m / 2
    Es = e_star(ma, mb)
    e = (ma.e + mb.e) / 2
    kn = 4.0 / 3.0 * Es * math.sqrt(R * delta)
    b = beta_of(e)
    gn = -b * math.sqrt(5.0 * mstar * kn)
    vn = -0.3                                   # approaching
    fn = kn * delta - gn * vn
    assert abs(-f[0, 0] / fn - 1.0) < 1e-12
    # E_0 enters both terms of the harmonic sum when the two sides share a type
    dEs_dE0 = Es ** 2 * (1 - ma.nu ** 2) / ma.E ** 2 * (1.0 if mixed else 2.0)
    dfn_dEs = kn * delta / Es - vn * gn / (2 * Es)
    de_de0 = 0.5 if mixed else 1.0              # the same type on both sides: e = e_0
    dfn_de0 = -vn * (-dbeta_de(e) * math.sqrt(5.0 * mstar * kn)) * de_de0
    got_E0 = -ft[0, 0, DIR["E0"]]
    got_e0 = -ft[0, 0, DIR["e0"]]
    assert abs(got_E0 / (dfn_dEs * dEs_dE0) - 1.0) < 1e-10
    assert abs(got_e0 / dfn_de0 - 1.0) < 1e-10
    if mixed:
        dEs_dE1 = Es ** 2 * (1 - mb.nu ** 2) / mb.E ** 2
        assert abs(-ft[0, 0, DIR["E1"]] / (dfn_dEs * dEs_dE1) - 1.0) < 1e-10
        assert abs(-ft[0, 0, DIR["e1"]] / dfn_de0 - 1.0) < 1e-10
    else:
        assert np.all(ft[..., DIR["E1"]] == 0.0) and np.all(ft[..., DIR["e1"]] == 0.0)
    # no tangential motion: nothing depends on mu
    assert np.all(ft[..., DIR["mu0"]] == 0.0) and np.all(ft[..., DIR["mu1"]] == 0.0)
    # equal and opposite tangents on the two particles
    assert np.array_equal(ft[0], -ft[1])


def test_sliding_force_tangent_is_mean_mu():
    """Eq. 5 on a sliding contact: |F_t| = mu |f_n| with mu = (mu_0 + mu_1)/2, so
    d|F_t|/d mu_k = |f_n| / 2 for a pair of two types."""
    ma = mat(mu=0.5)
    mb = mat(E=5e6, mu=0.3)
    s = overlapping_pair(ma, mb, vt=0.5)
    o = O.Oracle(s, tangent=True)
    o.tan_forces(False)
    f, ft = o.tan_vector("f")
    fn = -f[0, 0]
    # the trial force is pure damping along y (no history yet): sliding
    assert abs(abs(f[0, 1]) / (0.4 * abs(fn)) - 1.0) < 1e-12
    sgn = math.copysign(1.0, f[0, 1])
    for k in ("mu0", "mu1"):
        assert abs(sgn * ft[0, 1, DIR[k]] / (0.5 * abs(fn)) - 1.0) < 1e-12


def impact_tangents(e, E=5e6):
    """Head-on impact of two equal spheres at 1 m/s; the tangent state one
    step after separation and the step before it."""
    s = two_spheres(1.0, m1=mat(E=E, e=e))
    o = O.Oracle(s, tangent=True)
    o.tan_forces(False)
    rs = 2e-3
    prev = None
    for n in range(1, 4000):
        o.tan_step(1)
        xv, xt, vv, vt = o.tan_state()
        d = xv[1, 0] - xv[0, 0] - rs
        dd = xt[1, 0] - xt[0, 0]
        if prev is not None and prev[1] < 0.0 <= d and n > 10:
            return dict(t=n * s.dt, d=d, dd=dd, prev=prev, vrel=vv[1, 0] - vv[0, 0], dvrel=vt[1, 0] - vt[0, 0],
                        dt=s.dt)
        prev = (n * s.dt, d, dd)
    raise AssertionError("no separation")


def test_rebound_velocity_derivative_is_minus_v0():
    """P-2 differentiated: the rebound speed is e v0, so d(rebound)/de = v0 (the
    rebound velocity -e v0 changes by -v0)."""
    r = impact_tangents(0.9)
    assert abs(r["vrel"] / 0.9 - 1.0) < 5e-5
    # the discrete restitution differs from e by a step-quantised onset and
    # separation error that varies with e at the 1e-3 level (2.2e-3, 4.7e-3 and
    # 4e-5 at dt = 1, 0.5 and 0.25 us): a wrong damping derivative is off by O(1)
    assert abs(r["dvrel"][DIR["e0"]] / 1.0 - 1.0) < 1e-2


def test_contact_time_derivative_wrt_E():
    """P-1 differentiated: t_c scales as E*^(-2/5) (also with the damping of Eq. 6,
    which keeps the restitution fixed), so dt_c/dE = -(2/5) t_c / E."""
    r = impact_tangents(0.9)
    t0, d0, dd0 = r["prev"]
    t1, d1, dd1 = r["t"], r["d"], r["dd"]
    # separation time by linear interpolation of the gap between the two steps
    ts = t0 + (t1 - t0) * (-d0) / (d1 - d0)
    k = DIR["E0"]
    dts = (t1 - t0) * (-(dd0[k]) * (d1 - d0) + d0 * (dd1[k] - dd0[k])) / (d1 - d0) ** 2
    t_in = 1e-6 / 1.0                       # the gap of 1 um closes at 1 m/s (free flight)
    tc = ts - t_in
    expect = -0.4 * tc / 5e6
    assert abs(dts / expect - 1.0) < 2e-3


def test_sliding_distance_derivative_wrt_mu():
    """P-7 differentiated: a sphere launched at v0 on the wall slides until it
    rolls at t_r = 2 v0 / (7 mu g); afterwards x(T) = 2 v0^2 / (49 mu g) + 5/7 v0 T,
    so dx(T)/dmu = -2 v0^2 / (49 mu^2 g) = -1.664e-4 m at v0 = 0.1 m/s, mu = 0.5."""
    expect = -2 * 0.1 ** 2 / (49 * 0.25 * G0)
    assert abs(expect - -1.664e-4) < 1e-7
    m = mat(E=5e8, e=0.9, mu=0.5)
    K = 4.0 / 3.0 * e_star(m, m) * math.sqrt(1e-3)
    ds = (sphere_mass(1e-3, m.rho) * G0 / K) ** (2.0 / 3.0)
    o = O.Oracle(sphere_on_wall(1e-3 - ds, m=m, v=(0.1, 0.0, 0.0)), tangent=True)
    o.tan_forces(False)
    o.tan_step(8000)                        # t_r = 5.8 ms
    xv, xt, vv, vt = o.tan_state()
    assert abs(vv[0, 0] / (5.0 / 7.0 * 0.1) - 1.0) < 1e-3
    assert abs(xt[0, 0, DIR["mu0"]] / expect - 1.0) < 1e-2


def small_chute(seed=11, n=300):
    return W.chute_adjoint(seed=seed, n=n, Lx=14e-3, Ly=10e-3)


def oracle_final(sysm, nsteps, E=None, e=None, mu=None):
    s = sysm.copy()
    mats = []
    for t, m in enumerate(s.materials):
        mats.append(W.Material(E=m.E if E is None else E[t], nu=m.nu, rho=m.rho, e=m.e if e is None else e[t],
                               mu=m.mu if mu is None else mu[t]))
    s.materials = mats
    o = O.Oracle(s)
    o.forces(False)
    o.step(nsteps)
    st = o.state()
    return st["x"], st["v"]


def test_tangent_matches_central_difference():
    """The tangent of a linear functional of the final state after 40 steps of a
    two-type chute against central differences of the double-precision oracle
    (h = 1e-6 relative)."""
    s = small_chute()
    nsteps = 40
    rng = np.random.default_rng(3)
    a = rng.normal(size=(s.n, 3))
    b = rng.normal(size=(s.n, 3))
    o = O.Oracle(s, tangent=True)
    o.tan_forces(False)
    o.tan_step(nsteps)
    xv, xt, vv, vt = o.tan_state()
    x0, v0 = oracle_final(s, nsteps)
    assert np.array_equal(xv, x0) and np.array_equal(vv, v0)   # the dual run's values are the plain run
    scale_x = 1.0 / np.abs(x0).max()
    scale_v = 1.0 / max(np.abs(v0).max(), 1e-30)
    tan = np.einsum("ic,ick->k", a, xt) * scale_x + np.einsum("ic,ick->k", b, vt) * scale_v
    base = {"E": [m.E for m in s.materials], "e": [m.e for m in s.materials], "mu": [m.mu for m in s.materials]}
    for name, k in DIR.items():
        p, t = name[:-1], int(name[-1])
        h = 1e-6 * base[p][t]
        vals = []
        for sgn in (1, -1):
            q = {kk: list(vv_) for kk, vv_ in base.items()}
            q[p][t] += sgn * h
            xf, vf = oracle_final(s, nsteps, **q)
            vals.append(np.sum(a * xf) * scale_x + np.sum(b * vf) * scale_v)
        fd = (vals[0] - vals[1]) / (2 * h)
        assert abs(fd - tan[k]) <= 1e-5 * max(abs(tan[k]), 1e-3 * np.abs(tan).max()), (name, fd, tan[k])


def test_state_tangent_free_flight():
    """A state-seeded tangent direction in free flight: velocity Verlet under
    constant gravity gives x(T) = x0 + v0 T + g T^2 / 2 exactly, so
    dx(T)/dx0 = 1 and dx(T)/dv0 = T, and dv(T)/dv0 = 1."""
    s = sphere_on_wall(5e-3, v=(0.1, 0.0, 0.0))
    o = O.Oracle(s, tangent=True)
    o.tan_seed_state(0, dx=np.array([[1.0, 0.0, 0.0]]))
    o.tan_seed_state(1, dv=np.array([[0.0, 0.0, 1.0]]))
    o.tan_seed_state(2, dw=np.array([[0.0, 1.0, 0.0]]))
    o.tan_forces(False)
    o.tan_step(100)
    _, xt = o.tan_vector("x")
    _, vt = o.tan_vector("v")
    _, wt = o.tan_vector("w")
    T = 100 * s.dt
    assert xt[0, 0, 0] == 1.0 and xt[0, 1, 0] == 0.0 and xt[0, 2, 0] == 0.0
    assert abs(xt[0, 2, 1] - T) < 1e-15 and vt[0, 2, 1] == 1.0
    assert wt[0, 1, 2] == 1.0 and xt[0, 0, 2] == 0.0
    # the remaining directions are still the parameters (no contact: zero)
    assert np.all(xt[..., 3:] == 0.0)


def test_state_tangent_matches_central_difference():
    """State-seeded tangents of a linear functional after 40 steps of the
    two-type chute against central differences of the plain oracle."""
    s = small_chute()
    nsteps = 40
    rng = np.random.default_rng(21)
    a = rng.normal(size=(s.n, 3))
    b = rng.normal(size=(s.n, 3))
    dirs = {"x": rng.normal(size=(s.n, 3)), "v": rng.normal(size=(s.n, 3)), "w": rng.normal(size=(s.n, 3))}
    o = O.Oracle(s, tangent=True)
    o.tan_seed_state(0, dx=dirs["x"])
    o.tan_seed_state(1, dv=dirs["v"])
    o.tan_seed_state(2, dw=dirs["w"])
    o.tan_forces(False)
    o.tan_step(nsteps)
    _, xt = o.tan_vector("x")
    _, vt = o.tan_vector("v")
    tan = np.einsum("ic,ick->k", a, xt) * 1e3 + np.einsum("ic,ick->k", b, vt)

    def L(**kw):
        q = s.copy()
        for k, val in kw.items():
            setattr(q, k, val)
        oo = O.Oracle(q)
        oo.forces(False)
        oo.step(nsteps)
        st = oo.state()
        return np.sum(a * st["x"]) * 1e3 + np.sum(b * st["v"])

    # differences that move positions by ~4e-12 m: larger steps straddle contact
    # onsets (damping ~ delta^(1/4) has an infinite slope there) and Coulomb
    # switches, and the difference quotient converges to the tangent only below
    # ~1e-11 m (2.4e-2, 3.9e-4, 3.8e-6 at 1e-9, 1e-10, 1e-11 m)
    for k, (name, h) in enumerate((("x", 5e-12), ("v", 1e-7), ("w", 1e-4))):
        base = getattr(s, name)
        fd = (L(**{name: base + h * dirs[name]}) - L(**{name: base - h * dirs[name]})) / (2 * h)
        assert abs(fd - tan[k]) <= 1e-5 * abs(tan[k]), (name, fd, tan[k])
