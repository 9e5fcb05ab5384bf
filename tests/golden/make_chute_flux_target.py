"""Writes chute_flux_target.json: the target of the chute calibration loss.

The loss of the 50,000-sphere two-type chute is the mean squared difference of
the mass-flux profile (20 equal height bins over the initial bed height) after
200 steps from a target profile.  The target is the profile that the FP64 CPU
oracle produces for a perturbed parameter set theta* = theta0 (1 +- 0.05),
signs drawn with seed 5 (e stays below 1).  Only the oracle and the seeded
input generator are used.

    python tests/golden/make_chute_flux_target.py      (about a minute)
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.join(ROOT, "oracle"))

import oracle as O  # noqa: E402
from paper_1705_03850_amd.inputs import workloads as W  # noqa: E402

STEPS = 200
BINS = 20


def flux_profile(x, v, m, H0, Lx, Ly, bins=BINS):
    h = H0 / bins
    k = np.floor(x[:, 2] / h)
    ok = (k >= 0) & (k < bins)
    flux = np.zeros(bins)
    np.add.at(flux, k[ok].astype(int), m[ok] * v[ok, 0])
    return flux / (Lx * Ly * h)


def main():
    s = W.chute_adjoint()
    rng = np.random.default_rng(5)
    signs = rng.choice([-1.0, 1.0], size=(3, len(s.materials)))
    theta0 = np.array([[m.E for m in s.materials], [m.e for m in s.materials], [m.mu for m in s.materials]])
    theta = theta0 * (1.0 + 0.05 * signs)
    q = s.copy()
    q.materials = [W.Material(E=theta[0, t], nu=m.nu, rho=m.rho, e=theta[1, t], mu=theta[2, t])
                   for t, m in enumerate(s.materials)]
    t0 = time.time()
    o = O.Oracle(q)
    o.forces(False)
    o.step(STEPS)
    st = o.state()
    m, _ = o.mass()
    H0, Lx, Ly = s.meta["H0"], s.hi[0] - s.lo[0], s.hi[1] - s.lo[1]
    prof = flux_profile(st["x"], st["v"], m, H0, Lx, Ly)
    out = {"workload": "chute_adjoint(seed=5, n=50000)", "steps": STEPS, "bins": BINS, "H0": H0,
           "theta0": theta0.tolist(), "theta_star": theta.tolist(), "target_flux": prof.tolist(),
           "units": "kg m^-2 s^-1", "oracle_seconds": round(time.time() - t0, 1)}
    with open(os.path.join(HERE, "chute_flux_target.json"), "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out)[:400])


if __name__ == "__main__":
    main()
