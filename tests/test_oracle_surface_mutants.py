"""The surface pins catch plausible mistakes in the oracle's wall surfaces.

Each case plants one mistake in a copy of oracle/dem_oracle.cpp (compiled into
a temporary directory) and runs the checks of test_oracle_surface_pins.py
against it; the named checks must fail.
"""
import pytest

import oracle as O
import test_oracle_surface_pins as P

CHECKS = {
    "geometry": lambda lib: [P.check_geometry(rec, lib) for rec in (P.CYL, P.CONE, P.DISK, P.RING)],
    "static": lambda lib: [P.check_static_force(rec, lib) for rec in (P.CYL, P.CONE, P.DISK, P.RING)],
    "bounce": P.check_bounce,
    "sliding": P.check_sliding,
    "friction": P.check_surface_friction,
}

MUTANTS = {
    # the cone's inner side taken as the outer one
    "cone_side": ([("if (!(side > 0.0 && d > 0.0 && d < r)) return false;",
                    "if (!(side < 0.0 && d > 0.0 && d < r)) return false;")], ["geometry", "static"]),
    # the cylinder without its height range
    "cylinder_unbounded": ([("        if (z < w.z0 || z > w.z1) return false;\n", "")], ["geometry"]),
    # the plug without its radius
    "disk_unbounded": ([("        if (rho > w.r0) return false;\n", "")], ["geometry"]),
    # the cylinder's normal pointing out of the silo
    "cylinder_normal": ([("        n = {-dx / rho, -dy / rho, 0.0};", "        n = {dx / rho, dy / rho, 0.0};")],
                        ["geometry", "static"]),
    # the ring's distance taken to the axis instead of the circle
    "ring_axis": ([("        const double qr = rho - w.r0, qz = z - w.z0;\n        const double d = std::sqrt(qr * qr + qz * qz);\n        if (!(d > 0.0 && d < r)) return false;",
                    "        const double qr = rho, qz = z - w.z0;\n        const double d = std::sqrt(qr * qr + qz * qz);\n        if (!(d > 0.0 && d < r)) return false;")],
                  ["geometry", "static"]),
    # the surface's own friction ignored
    "wall_mu_ignored": ([("    if (!b && wn && wmu >= 0.0) k.mu = wmu;", "    (void)wmu;")], ["friction"]),
    # surface history not kept between steps
    "no_surface_history": ([("        if (update) s.shist.swap(snext);", "        if (update) s.shist.clear();")],
                           ["sliding"]),
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
    lib = _build(tmp_path, name, edits)
    failed = []
    for key, check in CHECKS.items():
        try:
            check(lib)
        except AssertionError:
            failed.append(key)
    assert set(expected) <= set(failed), (name, failed)
