"""The insertion pins catch plausible mistakes in oracle/insertion.py.

Each case plants one mistake in a copy of the module's source (loaded as a
separate module, the file itself untouched) and runs the named pins of
test_oracle_insertion_pins.py against it; each must fail.
"""
import os
import types

import pytest

import insertion
import test_oracle_insertion_pins as P

SRC = open(os.path.abspath(insertion.__file__)).read()

CHECKS = {
    "inflow": P.test_inflow_budget_counts_crossing_spheres,
    "line": P.test_ssi_line_in_order,
    "touching": P.test_ssi_touching_is_no_overlap,
    "existing": P.test_ssi_existing_spheres_block,
    "seam": P.test_ssi_periodic_seam,
    "budget": P.test_ssi_budget_per_cell,
    "outside": P.test_outside_half_space,
}

# name: (edits as (original text, planted text), pins that must fail)
MUTANTS = {
    # S-3: touching spheres counted as overlapping
    "touching_overlaps": ([("    return d2 < s * s\n", "    return d2 <= s * s\n")], ["touching"]),
    # S-3: distance without its z term
    "no_dz": ([("d2 = dx * dx + dy * dy + dz * dz", "d2 = dx * dx + dy * dy"),
               ("d2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2]", "d2 = d[0] * d[0] + d[1] * d[1]")], ["existing"]),
    # S-3: rejected candidates block later ones too
    "rejected_block": ([("for a in taken)", "for a in range(k))")], ["line"]),
    # S-3: a budget of exactly one sphere's mass affords none
    "budget_strict": ([("if not m <= budget[c]:", "if not m < budget[c]:")], ["budget"]),
    # S-3: accepted spheres not charged to the budget
    "budget_unspent": ([("        budget[c] -= m\n", "")], ["budget"]),
    # S-3: minimum image taken the wrong way
    "seam_sign": ([("    if d > 0.5 * L:\n        return d - L", "    if d > 0.5 * L:\n        return d + L"),
                   ("np.where(v > h, v - box_L[a]", "np.where(v > h, v + box_L[a]")], ["seam"]),
    # S-1: outflow counted instead of inflow
    "inflow_sign": ([("np.maximum(flow, 0.0)", "np.maximum(-flow, 0.0)")], ["inflow"]),
    # S-5: a centre on the plane removed
    "delete_on_plane": ([("n[2]) < d\n", "n[2]) <= d\n")], ["outside"]),
}


def mutant(edits):
    src = SRC
    for old, new in edits:
        assert src.count(old) >= 1, old
        src = src.replace(old, new)
    mod = types.ModuleType("insertion_mutant")
    exec(compile(src, "insertion_mutant.py", "exec"), mod.__dict__)
    return mod


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_fails_its_pins(name, monkeypatch):
    edits, must_fail = MUTANTS[name]
    monkeypatch.setattr(P, "S", mutant(edits))
    for check in must_fail:
        with pytest.raises(AssertionError):
            CHECKS[check]()


def test_unmodified_copy_passes(monkeypatch):
    monkeypatch.setattr(P, "S", mutant([]))
    for check in CHECKS.values():
        check()
