"""The seeded input generators: determinism, ranges, guard band, shapes."""
import math

import numpy as np

from synth import (GAMMA, uniform_set, plummer_set, adjoint_set, lattice_set,
                   guard_violations, h_for_neighbours, finest_grid)
from synth.generators import batched_sizes


def test_h48_closed_form():
    # (4 pi / 3) H^3 N = 48 -> eta = h N^{1/3} is the same for every N
    for n in (32768, 1 << 20, 1 << 22):
        h = h_for_neighbours(n)
        assert abs(4 * math.pi / 3 * (GAMMA * h) ** 3 * n - 48.0) < 1e-9
        assert abs(h * n ** (1 / 3) - 1.2348422195) < 1e-9


def test_uniform_deterministic_and_guarded():
    a = uniform_set(20000, 3, hmode="lognormal")
    b = uniform_set(20000, 3, hmode="lognormal")
    assert np.array_equal(a.pos, b.pos) and np.array_equal(a.h, b.h)
    assert a.pos.dtype == np.float32 and a.h.dtype == np.float32
    assert a.pos.min() >= 0 and a.pos.max() < 1
    assert guard_violations(a.pos, a.h).size == 0
    c = uniform_set(20000, 4, hmode="const")
    assert np.all(c.h == c.h[0]) and guard_violations(c.pos, c.h).size == 0
    med = np.median(a.h) / h_for_neighbours(20000)
    assert abs(med - 1.0) < 0.01


def test_plummer_clustered():
    s = plummer_set(60000, 5, n_spheres=8)
    assert s.pos.min() >= 0 and s.pos.max() < 1
    assert guard_violations(s.pos, s.h).size == 0
    assert int(s.extra["counts"].sum()) == 30000
    g = finest_grid(s.h)
    cells = np.floor(s.pos.astype(np.float64) * g).astype(int)
    occ = np.bincount((cells[:, 0] * g + cells[:, 1]) * g + cells[:, 2], minlength=g ** 3)
    assert occ.max() > 8 * occ.mean()            # strongly uneven occupancy


def test_adjoint_set_has_target_positions():
    s = adjoint_set(8000, 6)
    p = s.extra["pos_target"]
    assert p.shape == s.pos.shape and p.dtype == np.float32
    d = p.astype(np.float64) - s.pos
    d -= np.rint(d)
    assert 0 < np.std(d) < 0.2 * 8000 ** (-1 / 3)


def test_batched_sizes_log_uniform():
    n = batched_sizes()
    assert n.size == 256 and n.min() >= 4096 and n.max() <= 262144
    assert 10e6 < n.sum() < 25e6


def test_lattice_exact():
    s = lattice_set(16, math.sqrt(4.5))
    assert np.array_equal(s.pos.astype(np.float64) * 16, np.rint(s.pos.astype(np.float64) * 16))
