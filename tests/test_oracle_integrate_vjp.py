"""Pin of the oracle's reverse mode of the integration halves
(Oracle.integrate_vjp) against the oracle's own forward kick and drift: for
random output adjoints y and input directions d, <y, J d> (J d by central
differences of kick/drift, exact up to rounding for this linear map) equals
<J^T y, d>.  A reverse mode that drops the drift's dependence on v', the
half step or the mass fails it (planted below)."""
import numpy as np
import pytest

import oracle as O
from paper_1705_03850_amd.inputs import workloads as W


def system():
    # a small periodic gas: spheres well inside the box, so that no difference
    # step carries one across a seam
    s = W.chute_adjoint(seed=3, n=200)
    return s


def forward(o, z, phase):
    o.set_state(x=z["x"], v=z["v"], w=z["w"], f=z["f"], t=z["t"])
    o.kick()
    if phase == 0:
        o.drift()
    st = o.state()
    return {k: st[k] for k in ("x", "v", "w")}


def check(o, phase, vjp, seed):
    """True when the identity holds for a direction in each input block
    alone (x, v, w, f, t), to 1e-9 of that block's terms."""
    rng = np.random.default_rng(seed)
    st = o.state()
    z = {k: st[k].copy() for k in ("x", "v", "w", "f", "t")}
    m, inertia = o.mass()
    z["f"] = rng.normal(size=(o.n, 3)) * m[:, None] * 9.81
    z["t"] = rng.normal(size=(o.n, 3)) * inertia[:, None] * 100.0
    scale = {"x": 1e-3, "v": 1e-1, "w": 1e2, "f": 1e-2, "t": 1e-6}
    y = {k: rng.normal(size=(o.n, 3)) for k in ("x", "v", "w")}
    back = vjp(o, phase, y["x"], y["v"], y["w"])
    h = 1e-3
    for k in z:
        d = rng.normal(size=(o.n, 3)) * scale[k]
        zp = {q: z[q] + (h * d if q == k else 0.0) for q in z}
        zm = {q: z[q] - (h * d if q == k else 0.0) for q in z}
        fp, fm = forward(o, zp, phase), forward(o, zm, phase)
        lhs = sum(np.sum(y[q] * (fp[q] - fm[q]) / (2 * h)) for q in y)
        rhs = np.sum(back[k] * d)
        if not abs(lhs - rhs) <= 1e-9 * np.sum(np.abs(back[k] * d)):
            return False, k, lhs, rhs
    return True, None, None, None


@pytest.mark.parametrize("phase", [0, 1])
def test_integrate_vjp_is_the_transpose_of_kick_and_drift(phase):
    o = O.Oracle(system())
    for seed in range(3):
        ok, block, lhs, rhs = check(o, phase, O.Oracle.integrate_vjp, seed)
        assert ok, (phase, seed, block, lhs, rhs)


def _no_drift_term(o, phase, xb, vb, wb):
    return O.Oracle.integrate_vjp(o, 1, xb, vb, wb)    # phase 0 taken as a kick alone


def _full_step_kick(o, phase, xb, vb, wb):
    r = O.Oracle.integrate_vjp(o, phase, xb, vb, wb)
    r["f"] = 2.0 * r["f"]
    return r


def _mass_for_inertia(o, phase, xb, vb, wb):
    r = O.Oracle.integrate_vjp(o, phase, xb, vb, wb)
    m, inertia = o.mass()
    r["t"] = r["t"] * inertia[:, None] / m[:, None]
    return r


@pytest.mark.parametrize("mistake", [_no_drift_term, _full_step_kick, _mass_for_inertia])
def test_planted_mistakes_fail_the_pin(mistake):
    o = O.Oracle(system())
    assert not check(o, 0, mistake, 7)[0]
