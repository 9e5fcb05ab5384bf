"""Writes chute_flux_gradient.json: the chute calibration loss and its gradient
with respect to the per-type E, e and mu, from the FP64 CPU oracle.

Workload: the 50,000-sphere two-type chute (seed 5), 200 steps from the
generator's state at the parameters theta0 (the generator's materials).  Loss:
mean over 20 equal height bins of (flux_b - target_b)^2, with flux_b the mass
flux along x in bin b (sum of m v_x over the spheres in the bin, divided by the
bin volume; hard bins over the initial bed height) and the target of
chute_flux_target.json.  The gradient chains the oracle's forward-mode
(dual-number) tangent of the final velocities through the flux: bin membership
is piecewise constant in theta, so d flux_b = sum_{i in b} m_i d v_x,i / V_b.
Only the oracle and the seeded input generator are used.

    python tests/golden/make_chute_flux_gradient.py      (about five minutes)
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
sys.path.insert(0, HERE)

import oracle as O  # noqa: E402
from make_chute_flux_target import BINS, STEPS, flux_profile  # noqa: E402
from paper_1705_03850_amd.inputs import workloads as W  # noqa: E402


def main():
    with open(os.path.join(HERE, "chute_flux_target.json")) as fh:
        tgt = json.load(fh)
    s = W.chute_adjoint()
    H0, Lx, Ly = s.meta["H0"], s.hi[0] - s.lo[0], s.hi[1] - s.lo[1]
    assert abs(H0 - tgt["H0"]) == 0.0, "the generator's bed differs from the one the target was made on"
    t0 = time.time()
    o = O.Oracle(s, tangent=True)
    o.tan_forces(False)
    o.tan_step(STEPS)
    x, _ = o.tan_vector("x")
    v, vt = o.tan_vector("v")
    # masses as the oracle computes them (4/3 pi rho r^3)
    rho = np.array([m.rho for m in s.materials])[s.type]
    m = 4.0 / 3.0 * np.pi * rho * s.r * s.r * s.r
    flux = flux_profile(x, v, m, H0, Lx, Ly)
    target = np.array(tgt["target_flux"])
    loss = float(np.mean((flux - target) ** 2))
    h = H0 / BINS
    k = np.floor(x[:, 2] / h)
    ok = (k >= 0) & (k < BINS)
    dflux = np.zeros((BINS, 6))
    np.add.at(dflux, k[ok].astype(int), m[ok, None] * vt[ok, 0, :])
    dflux /= Lx * Ly * h
    grad = (2.0 / BINS) * (flux - target) @ dflux            # directions E0, E1, e0, e1, mu0, mu1
    out = {"workload": "chute_adjoint(seed=5, n=50000)", "steps": STEPS, "bins": BINS, "H0": H0,
           "theta0": tgt["theta0"], "loss": loss, "flux": flux.tolist(),
           "grad": {"E": grad[0:2].tolist(), "e": grad[2:4].tolist(), "mu": grad[4:6].tolist()},
           "oracle_seconds": round(time.time() - t0, 1)}
    with open(os.path.join(HERE, "chute_flux_gradient.json"), "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out)[:600])


if __name__ == "__main__":
    main()
