"""Candidate census of the sorted-projection pruning (paper Section 2).

TEST INFRASTRUCTURE ONLY.  For a receiver cell a and a neighbour cell b whose
centres are joined by the unit axis e, the pseudo-Verlet loop inspects the pair
(i, j) only when the projected separation (x_j - x_i) . e is below the
receiver's cut-off H_i (Listing 2 with the per-particle cut-off of Section 3.1);
a pair is in range when the 3D separation is below H_i.  The plain cell list
(Listing 1) inspects every pair.  These functions count both, by definition,
with no sorting: they exist to pin the fractions the paper quotes (Section 1
and Section 2) and to check a GPU sweep's own candidate counter.
"""
from __future__ import annotations

import numpy as np


def pair_census(xa, Ha, xb, e):
    """(candidates, in_range, all_pairs) for receivers xa (n_a, 3) with cut-offs
    Ha against sources xb (n_b, 3), projected on unit axis e.  Coordinates are
    already unwrapped into one frame."""
    xa = np.asarray(xa, dtype=np.float64)
    xb = np.asarray(xb, dtype=np.float64)
    Ha = np.asarray(Ha, dtype=np.float64).reshape(-1)
    e = np.asarray(e, dtype=np.float64)
    e = e / np.linalg.norm(e)
    d = xb[None, :, :] - xa[:, None, :]
    proj = d @ e
    r = np.sqrt(np.sum(d * d, axis=2))
    cand = proj < Ha[:, None]
    inr = r < Ha[:, None]
    return int(cand.sum()), int(inr.sum()), int(xa.shape[0] * xb.shape[0])


def face_pair_fractions(n_per_cell, H_over_C, trials, seed, offset=(1.0, 0.0, 0.0)):
    """Monte-Carlo over `trials` random cell pairs of edge 1 separated by
    `offset`: returns (in_range / candidates, in_range / all pairs)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    c = i = a = 0
    off = np.asarray(offset, dtype=np.float64)
    for _ in range(trials):
        xa = rng.random((n_per_cell, 3))
        xb = rng.random((n_per_cell, 3)) + off
        cc, ii, aa = pair_census(xa, np.full(n_per_cell, H_over_C), xb, off)
        c += cc
        i += ii
        a += aa
    return i / c, i / a
