"""The oracle's pins catch plausible mistakes in the readings they pin.

Each case plants one mistake in a copy of oracle/dem_oracle.cpp (compiled
into a temporary directory, never into the repository) and runs the checks of
test_oracle_history_pins.py against it; the mistake must fail the named
checks.  The unmodified oracle passes them all (the pin tests themselves).

One reordering is not a mistake: projecting the history after adding v_t dt
instead of before changes the result only by (v_t . n) dt n, and v_t is
tangential by construction, so the two orders agree to rounding.  That case
checks the agreement instead.
"""
import functools

import numpy as np
import pytest

import oracle as O
import test_oracle_history_pins as P

CHECKS = {
    "rigid_rotation": P.check_rigid_rotation_history,
    "reset_onset": P.check_history_reset_and_onset,
    "backsolve": P.check_backsolve_reproduces_cap,
    "tangent_plane": P.check_tangential_force_in_tangent_plane,
    "wrap": P.check_periodic_wrap,
}

# name: (edits as (original text, planted text), checks that must fail)
MUTANTS = {
    # C-5: history kept in the lab frame instead of projected onto the tangent plane
    "no_projection": (
        [("V3<S> z = {xi.x - xn * n.x, xi.y - xn * n.y, xi.z - xn * n.z};", "V3<S> z = xi;")],
        ["rigid_rotation", "tangent_plane"]),
    # C-12: no periodic wrap of drifted positions
    "no_wrap": (
        [("    if (!periodic) return x;\n    double L = hi - lo;", "    return x;\n    double L = hi - lo;")],
        ["wrap"]),
    # C-12: a position rounded up to hi is left there instead of put at lo
    "no_seam_clamp": (
        [("    if (val(x) >= hi) x = S(lo);\n", "")],
        ["wrap"]),
    # C-4: back-solve of the capped force without the dashpot term
    "backsolve_without_damping": (
        [("z = {-(ft.x + gt * vt.x) / kt, -(ft.y + gt * vt.y) / kt, -(ft.z + gt * vt.z) / kt};",
          "z = {-ft.x / kt, -ft.y / kt, -ft.z / kt};")],
        ["backsolve"]),
    # C-6: contact-point velocity without the spin term
    "no_spin_in_slip": (
        [("V3<S> vt = {vr.x - vn * n.x - wxn.x, vr.y - vn * n.y - wxn.y, vr.z - vn * n.z - wxn.z};",
          "V3<S> vt = {vr.x - vn * n.x, vr.y - vn * n.y, vr.z - vn * n.z};")],
        ["rigid_rotation", "reset_onset"]),
    # Eq. 4 / C-1: history advanced against the slip
    "increment_sign": (
        [("z.x = z.x + vt.x * c.dt;", "z.x = z.x - vt.x * c.dt;"),
         ("z.y = z.y + vt.y * c.dt;", "z.y = z.y - vt.y * c.dt;"),
         ("z.z = z.z + vt.z * c.dt;", "z.z = z.z - vt.z * c.dt;")],
        ["rigid_rotation", "reset_onset"]),
    # C-5: history of pairs that left contact is kept instead of dropped
    "no_reset": (
        [("    if (update) s.hist.swap(next);",
          "    if (update) for (auto &kv : next) s.hist[kv.first] = kv.second;")],
        ["reset_onset"]),
}


def _build(tmp_path, name, edits):
    src = open(O._SRC).read()
    for old, new in edits:
        assert src.count(old) == 1, (name, old)
        src = src.replace(old, new)
    path = tmp_path / f"{name}.cpp"
    path.write_text(src)
    return O.compile_to(str(path), str(tmp_path / f"lib{name}.so"))


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_fails_its_pins(name, tmp_path):
    edits, expected = MUTANTS[name]
    make = functools.partial(O.Oracle, lib_path=_build(tmp_path, name, edits))
    failed = []
    for key, check in CHECKS.items():
        try:
            check(make)
        except AssertionError:
            failed.append(key)
    assert set(expected) <= set(failed), (name, failed)


def test_projection_after_increment_agrees_to_rounding(tmp_path):
    """Moving the projection after the increment is the same map in exact
    arithmetic; on a spinning packing the histories agree to rounding."""
    edits = [("""    V3<S> z = {xi.x - xn * n.x, xi.y - xn * n.y, xi.z - xn * n.z};
    if (update) {
        z.x = z.x + vt.x * c.dt;
        z.y = z.y + vt.y * c.dt;
        z.z = z.z + vt.z * c.dt;
    }""", """    V3<S> z = xi;
    if (update) {
        z.x = z.x + vt.x * c.dt;
        z.y = z.y + vt.y * c.dt;
        z.z = z.z + vt.z * c.dt;
    }
    S zn = z.x * n.x + z.y * n.y + z.z * n.z;
    z = {z.x - zn * n.x, z.y - zn * n.y, z.z - zn * n.z};""")]
    lib = _build(tmp_path, "project_after", edits)
    s = P.W.plain_fcc()
    s.w = np.random.default_rng(4).normal(0.0, 300.0, s.w.shape)
    out = []
    for path in (None, lib):
        o = O.Oracle(s, lib_path=path)
        o.forces(False)
        o.step(200)
        out.append(o.history())
    (lo0, hi0, xi0), (lo1, hi1, xi1) = out
    assert np.array_equal(lo0, lo1) and np.array_equal(hi0, hi1) and len(lo0) > 100
    scale = np.abs(xi0).max()
    assert np.max(np.abs(xi1 - xi0)) < 1e-9 * scale
