"""O(N^2) all-pairs density, numpy, fp64, for tiny inputs only.

TEST INFRASTRUCTURE ONLY.  Every receiver tests all N particles (the naive
algorithm the paper's introduction starts from) with the minimum-image
convention.  It exists to pin the cell-list oracle: if the cell list misses or
double-counts a neighbour, the two disagree.  The kernel is written out here
again on purpose; its own correctness is pinned separately (normalisation,
continuity, lattice sums).
"""
from __future__ import annotations

import numpy as np

GAMMA = 1.825742


def _w(u):
    u = np.asarray(u, dtype=np.float64)
    inner = 1.0 - 6.0 * u ** 2 + 6.0 * u ** 3
    outer = 2.0 * (1.0 - u) ** 3
    return np.where(u < 0.5, inner, np.where(u < 1.0, outer, 0.0))


def _dw(u):
    u = np.asarray(u, dtype=np.float64)
    inner = -12.0 * u + 18.0 * u ** 2
    outer = -6.0 * (1.0 - u) ** 2
    return np.where(u < 0.5, inner, np.where(u < 1.0, outer, 0.0))


def density_allpairs(pos, h, m, box=(1.0, 1.0, 1.0)):
    x = np.asarray(pos, dtype=np.float64)
    h = np.asarray(h, dtype=np.float64)
    m = np.asarray(m, dtype=np.float64)
    L = np.asarray(box, dtype=np.float64)
    d = x[None, :, :] - x[:, None, :]               # d[i, j] = x_j - x_i
    d -= L * np.rint(d / L)
    r = np.sqrt(np.sum(d * d, axis=2))
    H = GAMMA * h
    inr = r < H[:, None]
    u = np.where(inr, r / H[:, None], 1.0)
    w = np.where(inr, _w(u), 0.0)
    dw = np.where(inr, _dw(u), 0.0)
    norm = 8.0 / (np.pi * H ** 3)
    rho = norm * (w * m[None, :]).sum(1)
    wcount = norm * w.sum(1)
    drho_dh = -norm / h * (m[None, :] * (3.0 * w + u * dw)).sum(1)
    ncount = inr.sum(1) - 1
    return dict(rho=rho, wcount=wcount, drho_dh=drho_dh, ncount=ncount)
