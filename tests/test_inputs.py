"""Seeded workload generators: reproducibility and the stated packing properties."""
import numpy as np
from scipy.spatial import cKDTree

from paper_1705_03850_amd.inputs import workloads as W


def _pairs(x, r, L, cut_extra=0.0):
    tree = cKDTree(np.c_[np.mod(x[:, 0], L[0]), np.mod(x[:, 1], L[1]), x[:, 2]], boxsize=[L[0], L[1], 1e9])
    p = np.array(sorted(tree.query_pairs(2 * r.max() + cut_extra)), dtype=np.int64).reshape(-1, 2)
    d = x[p[:, 0]] - x[p[:, 1]]
    d[:, 0] -= L[0] * np.round(d[:, 0] / L[0])
    d[:, 1] -= L[1] * np.round(d[:, 1] / L[1])
    dist = np.linalg.norm(d, axis=1)
    return p, dist


def test_plain_fcc_reproducible_and_gapped():
    a, b = W.plain_fcc(), W.plain_fcc()
    assert np.array_equal(a.x, b.x) and np.array_equal(a.v, b.v)
    assert a.n == 2000 and abs(a.v.mean(axis=0)).max() < 1e-15
    p, dist = _pairs(a.x, a.r, (20e-3, 20e-3), cut_extra=0.1e-3)
    assert len(p) > 10000                          # ~12 lattice neighbours within 2.1 mm
    assert dist.min() > 2e-3                       # no overlaps: all gaps positive
    assert np.all(a.x[:, 2] > a.r)                 # clear of the wall
    assert np.all((a.x[:, :2] >= 0) & (a.x[:, :2] < 20e-3))


def test_settled_bed_properties():
    n = 20000
    b1 = W.settled_bed(n=n, footprint=80e-3 * np.sqrt(n / 1e6))
    b2 = W.settled_bed(n=n, footprint=80e-3 * np.sqrt(n / 1e6))
    assert np.array_equal(b1.x, b2.x) and np.array_equal(b1.id, b2.id)
    assert b1.meta["deposit_stuck"] == 0
    assert np.array_equal(np.sort(b1.id), np.arange(n))
    assert b1.r.min() >= 0.8e-3 and b1.r.max() <= 1.2e-3
    L = (b1.hi[0], b1.hi[1])
    p, dist = _pairs(b1.x, b1.r, L)
    rs = b1.r[p[:, 0]] + b1.r[p[:, 1]]
    overlap = (rs - dist) / np.minimum(b1.r[p[:, 0]], b1.r[p[:, 1]])
    coord = 2.0 * np.count_nonzero(overlap > 0) / n
    assert 5.5 < coord < 6.6                       # settled bed, mean coordination ~6
    assert overlap.max() < 0.06                    # overlaps stay a few percent of r
    H = b1.x[:, 2].max()
    phi = np.sum(4 / 3 * np.pi * b1.r ** 3) / (L[0] * L[1] * H)
    assert 0.55 < phi < 0.63
