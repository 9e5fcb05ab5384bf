"""Differentiable DEM rollout for PyTorch.

``DemRollout`` is a ``torch.autograd.Function`` whose forward runs a rollout
in libdem.so (dem_rollout_forward) and whose backward is the library's
hand-written reverse mode (dem_rollout_backward): the gradient of any scalar
of the final x, v, w with respect to the per-type E, e and mu.  This module
only marshals arguments; every step runs in the library's kernels.

``mass_flux_profile`` is the objective of the chute calibration workload:
the mass flux along x in equal height bins of the initial bed.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import torch

from . import dem


class DemRollout(torch.autograd.Function):
    """theta: (3, ntypes) float64 tensor, rows E, e, mu.  ``initial`` (x, v, w
    as (n, 3) host arrays in system order, or None to start from the current
    state) is loaded before the rollout.  Returns the final x, v, w as (3, n)
    device tensors in the system's current order."""

    @staticmethod
    def forward(ctx, theta, adj, initial=None):
        dsys = adj.dsys
        th = theta.detach().cpu().numpy()
        mats = [dataclasses.replace(m, E=float(th[0, t]), e=float(th[1, t]), mu=float(th[2, t]))
                for t, m in enumerate(dsys.systems[0].materials)]
        dsys.set_materials(mats)
        if initial is not None:
            dsys.load_state(*initial)
            dsys.reset()
        adj.forward()
        ctx.adj = adj
        return dsys.x.clone(), dsys.v.clone(), dsys.w.clone()

    @staticmethod
    def backward(ctx, gx, gv, gw):
        r = ctx.adj.backward(gx, gv, gw)
        g = torch.tensor(np.stack([r["E"], r["e"], r["mu"]]), dtype=torch.float64)
        return g, None, None


def rollout(theta, adj, initial=None):
    return DemRollout.apply(theta, adj, initial)


def theta_of(materials) -> torch.Tensor:
    return torch.tensor([[m.E for m in materials], [m.e for m in materials], [m.mu for m in materials]],
                        dtype=torch.float64)


def masses(dsys) -> torch.Tensor:
    """Sphere masses 4/3 pi rho r^3 in the system's current order."""
    rho = torch.tensor([m.rho for m in dsys.systems[0].materials], dtype=torch.float64, device=dsys.device)
    return 4.0 / 3.0 * math.pi * rho[dsys.type.long()] * dsys.r ** 3


def mass_flux_profile(x, v, mass, H0: float, Lx: float, Ly: float, bins: int = 20) -> torch.Tensor:
    """Mass flux along x in `bins` equal z-bins over [0, H0]: sum of m v_x of the
    particles in a bin over the bin volume (hard bins; particles outside [0, H0)
    are not counted)."""
    h = H0 / bins
    k = torch.floor(x[2] / h)
    inside = (k >= 0) & (k < bins)
    onehot = (k.unsqueeze(0) == torch.arange(bins, device=x.device, dtype=k.dtype).unsqueeze(1)) & inside
    return (onehot.to(torch.float64) * (mass * v[0]).unsqueeze(0)).sum(dim=1) / (Lx * Ly * h)


__all__ = ["DemRollout", "rollout", "theta_of", "masses", "mass_flux_profile", "dem"]
