"""Pins of the FP64 oracle against facts other than itself.

Kernel: normalisation, smoothness at the knots, derivative consistency.
Neighbour sums: O(N^2) brute force, exact lattice shells, uniform-random
expectations, scale and permutation invariance.
Adjoint: fp64 central finite differences and translation invariance.
Pruning census: the in-range fractions the paper quotes.
"""
import math
import os

import numpy as np
import pytest
from scipy import integrate

from oracle import Oracle, kernel_w, ORACLE_GAMMA
from oracle.allpairs import density_allpairs
from oracle.census import face_pair_fractions, pair_census
from synth import uniform_set, lattice_set, lj_set, GAMMA, h_for_neighbours

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    rows = {}
    with open(os.path.join(GOLD, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            parts = line.split()
            rows[parts[0]] = parts[1:]
    return rows


# ---------------------------------------------------------------- kernel pins
def test_kernel_normalised():
    """The 3D kernel integrates to one: int_0^H 4 pi r^2 W(r, H) dr = 1 with
    W = 8/(pi H^3) w(r/H) (H = 1).  A wrong coefficient in either piece of w or
    a wrong prefactor fails this."""
    f = lambda u: 4.0 * math.pi * u * u * 8.0 / math.pi * kernel_w(u)[0]
    a, _ = integrate.quad(f, 0.0, 0.5, epsabs=1e-14, epsrel=1e-14)
    b, _ = integrate.quad(f, 0.5, 1.0, epsabs=1e-14, epsrel=1e-14)
    assert abs(a + b - 1.0) < 1e-12


def test_kernel_smooth_at_knots():
    """w, w' and w'' are continuous at u = 1/2 and u = 1 and w vanishes at the
    support edge: with w'(0) = 0 these conditions plus normalisation fix the
    piecewise cubic uniquely (the M4 spline)."""
    e = 1e-7
    for u0 in (0.5, 1.0):
        wl, dl = kernel_w(u0 - e)
        wr, dr = kernel_w(u0 + e) if u0 < 1.0 else (0.0, 0.0)
        assert abs(wl - wr) < 1e-6 and abs(dl - dr) < 1e-5
        d2l = (kernel_w(u0 - e)[1] - kernel_w(u0 - 2 * e)[1]) / e
        d2r = (kernel_w(u0 + 2 * e)[1] - kernel_w(u0 + e)[1]) / e if u0 < 1.0 else 0.0
        assert abs(d2l - d2r) < 1e-4
    assert kernel_w(1.0) == (0.0, 0.0)
    assert kernel_w(0.0) == (1.0, 0.0)


def test_kernel_derivative_matches_fd():
    for u in np.linspace(0.01, 0.99, 37):
        if abs(u - 0.5) < 1e-3:
            continue
        e = 1e-6
        fd = (kernel_w(u + e)[0] - kernel_w(u - e)[0]) / (2 * e)
        assert abs(fd - kernel_w(u)[1]) < 1e-8


def test_gamma_constant_agrees_with_inputs():
    assert ORACLE_GAMMA == GAMMA == 1.825742


# ------------------------------------------------------- brute-force agreement
@pytest.mark.parametrize("seed,n,ngb,box", [
    (1, 600, 20, (1.0, 1.0, 1.0)),
    (2, 1500, 12, (1.0, 1.0, 1.0)),
    (3, 1000, 10, (1.0, 1.3, 0.8)),
    (4, 2000, 8, (1.0, 1.0, 1.0)),
])
def test_cell_list_equals_all_pairs(seed, n, ngb, box):
    """Cell list (27-cell stencil, periodic wrap) against every pair.  Varying
    h, 3..5 cells per side, a rectangular box."""
    rng = np.random.Generator(np.random.PCG64(seed))
    L = np.asarray(box)
    pos = (rng.random((n, 3)) * L).astype(np.float32)
    h48 = h_for_neighbours(n, ngb, 1.0)
    h = (h48 * np.exp(0.25 * rng.standard_normal(n))).astype(np.float32)
    Hmax = GAMMA * float(h.max())
    lim = 0.97 * float(L.min()) / 3.0           # keep at least 3 cells per side
    if Hmax > lim:
        h = (h * (lim / Hmax)).astype(np.float32)
        Hmax = GAMMA * float(h.max())
    g = [max(3, int(L[a] / (Hmax * 1.000001))) for a in range(3)]
    m = (rng.random(n) + 0.5).astype(np.float32) / n
    o = Oracle(pos, h, m, box, g).density()
    a = density_allpairs(pos, h, m, box)
    assert np.array_equal(o["ncount"], a["ncount"])
    for k in ("rho", "wcount"):
        assert np.max(np.abs(o[k] - a[k]) / np.abs(a[k])) < 1e-12
    assert np.max(np.abs(o["drho_dh"] - a["drho_dh"]) / o["dh_abs"]) < 1e-12


# --------------------------------------------------------------- lattice pins
@pytest.mark.parametrize("M,R2,expect", [(16, 4.5, 32), (16, 5.5, 56), (32, 5.5, 56)])
def test_lattice_shells(M, R2, expect):
    """Simple cubic lattice, spacing a = 1/M, cut-off H = R a.  Every particle
    sees the lattice shells |k|^2 < R^2 (textbook shell populations), so its
    neighbour count is exact and its density is the shell sum
    rho / rho_bar = 8 / (pi R^3) sum_s count_s w(sqrt(s) / R)."""
    shells = {int(k): int(v[0]) for k, v in _golden("lattice_shells.txt").items()}
    R = math.sqrt(R2)
    s = lattice_set(M, R)
    o = Oracle(s.pos, s.h, s.m).density()
    n_expect = sum(c for q, c in shells.items() if q < R2)
    assert n_expect == expect
    assert np.all(o["ncount"] == expect)
    H = ORACLE_GAMMA * float(s.h[0])        # the exact cut-off used (fp32 h)
    Ra = H * M                              # R as seen by the oracle
    ratio = 8.0 / (math.pi * Ra ** 3) * (1.0 + sum(c * kernel_w(math.sqrt(q) / Ra)[0]
                                                   for q, c in shells.items() if q < R2))
    rho_bar = 1.0                            # m = 1/M^3, a^3 = 1/M^3
    assert np.allclose(o["rho"], ratio * rho_bar, rtol=1e-13, atol=0)
    # a normalised smooth kernel summed on a lattice gives nearly the mean density
    assert abs(ratio - 1.0) < 0.01
    # every particle is equivalent
    assert np.ptp(o["rho"]) < 1e-13 and np.ptp(o["drho_dh"]) < 1e-10


# ------------------------------------------------------------ statistical pins
def test_uniform_expectations():
    """Uniform random points (unit periodic box, H < 1/2), constant h, m = 1/N:
    E[ncount] = (N-1)(4 pi / 3) H^3, E[rho] = (N-1)/N + c, E[drho_dh] = -3c/h with
    c = 8 / (pi N H^3) the self term.  The non-self part of drho_dh has zero mean
    because the h-derivative of a normalised kernel integrates to zero."""
    n = 32768
    s = uniform_set(n, 101, hmode="const")
    o = Oracle(s.pos, s.h, s.m, grid=8).density()
    h = float(s.h[0])
    H = ORACLE_GAMMA * h
    c = 8.0 / (math.pi * n * H ** 3)
    se = lambda x: np.std(x) / math.sqrt(x.size)
    e_n = (n - 1) * 4.0 * math.pi / 3.0 * H ** 3
    assert abs(o["ncount"].mean() - e_n) < 6 * se(o["ncount"]) + 1e-9
    assert abs(o["rho"].mean() - ((n - 1) / n + c)) < 6 * se(o["rho"])
    assert abs(o["drho_dh"].mean() - (-3.0 * c / h)) < 6 * se(o["drho_dh"])
    # and the tests are sharp enough to see a dropped self term
    assert 6 * se(o["rho"]) < 0.5 * c


def test_scale_and_permutation_invariance():
    """Scaling positions, box and h by lam scales rho by lam^-3 and leaves the
    counts unchanged; permuting the input permutes the output."""
    s = uniform_set(4000, 7, hmode="lognormal")
    base = Oracle(s.pos, s.h, s.m).density()
    lam = 2.0                                 # exact in fp32
    sc = Oracle(s.pos * np.float32(lam), s.h * np.float32(lam), s.m, (lam,) * 3).density()
    assert np.array_equal(sc["ncount"], base["ncount"])
    assert np.allclose(sc["rho"], base["rho"] / lam ** 3, rtol=1e-12)
    assert np.allclose(sc["drho_dh"], base["drho_dh"] / lam ** 4, rtol=1e-9, atol=1e-12)
    perm = np.random.Generator(np.random.PCG64(3)).permutation(s.n)
    pr = Oracle(s.pos[perm], s.h[perm], s.m[perm]).density()
    assert np.array_equal(pr["ncount"], base["ncount"][perm])
    assert np.allclose(pr["rho"], base["rho"][perm], rtol=1e-13)


def test_receiver_subset_matches_full():
    s = uniform_set(5000, 8, hmode="jitter")
    o = Oracle(s.pos, s.h, s.m)
    full = o.density()
    idx = np.array([0, 17, 4999, 2500, 17])
    sub = o.density(idx)
    for k in ("rho", "wcount", "drho_dh", "ncount"):
        assert np.array_equal(sub[k], full[k][idx])


# ------------------------------------------------------------------ adjoint pins
def test_drho_dh_matches_fd():
    """drho_dh against an fp64 central difference of rho in h: with target
    t = rho - 1/2, dL/dh_k = 2 (rho_k - t_k) drho_dh_k = drho_dh_k."""
    s = uniform_set(3000, 9, hmode="jitter")
    o = Oracle(s.pos, s.h, s.m)
    d = o.density()
    t = d["rho"] - 0.5
    ks = np.arange(0, 3000, 97)
    eps = 1e-5 * s.h[ks].astype(np.float64)
    fd = o.fd_loss(t, ks, np.full(ks.size, 3), eps)
    assert np.max(np.abs(fd - d["drho_dh"][ks]) / d["dh_abs"][ks]) < 1e-7


def test_gradient_matches_fd_and_is_translation_invariant():
    """Analytic adjoint of L = sum (rho - t)^2 against fp64 central differences
    of L itself (positions and h), Richardson-checked; and sum_k dL/dx_k = 0."""
    s = uniform_set(4000, 10, hmode="jitter")
    o = Oracle(s.pos, s.h, s.m)
    rng = np.random.Generator(np.random.PCG64(12))
    t = o.density()["rho"] * (1.0 + 0.1 * rng.standard_normal(s.n))
    rho = o.density()["rho"]
    G = 2.0 * (rho - t)
    g = o.grad(G)
    ks = np.repeat(np.arange(0, s.n, 211), 4)
    comps = np.tile(np.arange(4), ks.size // 4)
    Hk = ORACLE_GAMMA * s.h[ks].astype(np.float64)
    eps = np.where(comps < 3, 1e-4 * Hk, 1e-4 * s.h[ks])
    fd1 = o.fd_loss(t, ks, comps, eps)
    fd2 = o.fd_loss(t, ks, comps, eps / 2)
    ana = np.where(comps < 3, g["gx"][ks, np.minimum(comps, 2)], g["gh"][ks])
    scale = np.where(comps < 3, g["gx_abs"][ks, np.minimum(comps, 2)], g["gh_abs"][ks])
    rich = (4 * fd2 - fd1) / 3
    assert np.max(np.abs(rich - ana) / scale) < 1e-8
    assert np.max(np.abs(fd2 - ana) / scale) < 1e-5
    tot = g["gx"].sum(0)
    assert np.all(np.abs(tot) < 1e-10 * g["gx_abs"].sum(0))
    # dL/dh_k = G_k drho_dh_k
    d = o.density()
    assert np.allclose(g["gh"], G * d["drho_dh"], rtol=1e-14, atol=0)


def test_gradient_sign_flip_is_caught():
    """A planted sign error in the second adjoint term is visible to the FD
    comparison above (guards the sharpness of that test)."""
    s = uniform_set(2000, 13, hmode="jitter")
    o = Oracle(s.pos, s.h, s.m)
    rng = np.random.Generator(np.random.PCG64(2))
    rho = o.density()["rho"]
    t = rho * (1.0 + 0.1 * rng.standard_normal(s.n))
    G = 2.0 * (rho - t)
    g_good = o.grad(G)
    # only the receiver term: gradient with G_j zeroed for every j != k, evaluated
    # on one particle, differs from the full adjoint by far more than the tolerance
    k = 5
    Gk = np.zeros(s.n)
    Gk[k] = G[k]
    g_recv = o.grad(Gk, [k])
    diff = np.abs(g_recv["gx"][0] - g_good["gx"][k]) / g_good["gx_abs"][k]
    assert np.max(diff) > 1e-3


# ------------------------------------------------------------ paper fractions
def test_sorted_pruning_in_range_fraction():
    """Paper, Section 2: about 68% of pairs inspected under the sorted
    projection test are in range (face pair, cut-off = cell edge)."""
    gold = _golden("paper_fractions.txt")
    val, tol = float(gold["sorted_face_inrange_over_candidates"][0]), \
        float(gold["sorted_face_inrange_over_candidates"][1])
    frac, naive_face = face_pair_fractions(150, 1.0, 40, 5)
    assert abs(frac - val) < tol
    # the naive face pair alone is ~1/3 in range: the paper's <=16% is the
    # 27-cell-stencil figure, (4 pi / 3) / 27
    assert abs(naive_face - 0.335) < 0.01
    stencil = 4.0 * math.pi / 3.0 / 27.0
    assert stencil <= float(gold["naive_stencil_inrange_over_candidates"][0])


def test_census_projection_never_exceeds_distance():
    """The pruning is exact: every in-range pair is a candidate."""
    rng = np.random.Generator(np.random.PCG64(1))
    for off in [(1, 0, 0), (1, 1, 0), (1, 1, 1), (1, -1, 0), (0, 1, -1)]:
        xa = rng.random((100, 3))
        xb = rng.random((100, 3)) + np.asarray(off)
        Ha = rng.uniform(0.3, 1.0, 100)
        e = np.asarray(off, dtype=np.float64)
        d = xb[None] - xa[:, None]
        r = np.linalg.norm(d, axis=2)
        proj = d @ (e / np.linalg.norm(e))
        assert np.all(proj[r < Ha[:, None]] < Ha[np.nonzero(r < Ha[:, None])[0]])
        c, i, a = pair_census(xa, Ha, xb, e)
        assert i <= c <= a


# ------------------------------------------------------- smoothing-length solve
def test_solve_h_lattice_shells():
    """On a simple cubic lattice every particle has the same density, a shell
    sum over the textbook shell populations, so rho h^3 = m eta^3 reduces to one
    equation in R = H / a: (8 / (pi gamma^3)) (R a / H)^3 ... written out below
    and solved by scipy's brentq; the oracle's per-particle bisection must give
    the same h for every particle."""
    from scipy.optimize import brentq
    from oracle import solve_h_fp64, eta_for_neighbours
    shells = {int(k): int(v[0]) for k, v in _golden("lattice_shells.txt").items()}
    M = 16
    a = 1.0 / M
    eta = eta_for_neighbours(48.0)
    s = lattice_set(M, 2.0)

    # rho(h) h^3 / m = (8 / (pi gamma^3)) (1 + sum_s count_s w(sqrt(s) a / (gamma h)))
    def g(h):
        H = ORACLE_GAMMA * h
        tot = 1.0 + sum(c * kernel_w(math.sqrt(q) * a / H)[0] for q, c in shells.items()
                        if math.sqrt(q) * a < H)
        return 8.0 / (math.pi * ORACLE_GAMMA ** 3) * tot - eta ** 3
    h_shell = brentq(g, 0.5 * eta * a, 1.6 * eta * a, xtol=1e-15)
    h = solve_h_fp64(s.pos, s.m, 0.6 * eta * a, 1.5 * eta * a, eta)
    assert np.max(np.abs(h - h_shell)) < 1e-12 * h_shell
    # the shells inside the solved cut-off: 1, 2, 3, 4 and 5 (|k|^2 < R^2)
    assert 5.0 < (ORACLE_GAMMA * h_shell / a) ** 2 < 6.0


def test_solve_h_satisfies_relation_and_neighbour_number():
    """At the solved h the density loop (a different code path from the
    solver's) gives rho h^3 = m eta^3, and with equal masses the weighted
    neighbour number (4 pi / 3) H^3 wcount equals the target."""
    from oracle import solve_h_fp64, eta_for_neighbours
    s = uniform_set(3000, 41, hmode="lognormal")
    eta = eta_for_neighbours(48.0)
    h0 = h_for_neighbours(3000)
    h = solve_h_fp64(s.pos, s.m, 0.4 * h0, 1.9 * h0, eta)
    o = Oracle(s.pos, h, s.m).density()
    m = s.m.astype(np.float64)
    assert np.max(np.abs(o["rho"] * h ** 3 / (m * eta ** 3) - 1.0)) < 1e-11
    H = ORACLE_GAMMA * h
    assert np.max(np.abs(4.0 * math.pi / 3.0 * H ** 3 * o["wcount"] - 48.0)) < 1e-9
    with pytest.raises(ValueError):
        solve_h_fp64(s.pos, s.m, 0.4 * h0, 0.5 * h0, eta)     # no root in the bracket


# -------------------------------------------------------------- Lennard-Jones
def test_lj_pair_minimum():
    """Two particles at the textbook minimum r = 2^(1/6) sigma: zero force and a
    pair energy of -eps (each particle holds half)."""
    sigma, eps = 0.05, 1.7
    r = 2.0 ** (1.0 / 6.0) * sigma
    pos = np.array([[0.4, 0.5, 0.5], [0.4 + r, 0.5, 0.5]])
    h = np.full(2, 0.2 / ORACLE_GAMMA)
    o = Oracle(pos, h, np.ones(2)).lj(eps, sigma)
    assert np.max(np.abs(o["force"])) < 1e-12 * eps / sigma       # the natural force scale
    assert np.allclose(o["energy"], -0.5 * eps, rtol=1e-13)
    # and off the minimum the pair is pushed apart / pulled together
    for dr, sign in ((-0.1 * sigma, -1.0), (0.1 * sigma, 1.0)):
        p2 = pos.copy()
        p2[1, 0] += dr
        f = Oracle(p2, h, np.ones(2)).lj(eps, sigma)["force"]
        assert np.sign(f[0, 0]) == sign and f[1, 0] == -f[0, 0]


def test_lj_lattice_shell_sum():
    """Perfect simple cubic lattice: every force vanishes by symmetry and each
    particle's energy is half the shell sum of U(a sqrt(s)) over the textbook
    shell populations inside the cut-off."""
    shells = {int(k): int(v[0]) for k, v in _golden("lattice_shells.txt").items()}
    M, a = 8, 1.0 / 8
    s = lj_set(M, 1, jitter=0.0, rc_over_a=2.2)
    sigma, eps = a, 1.0
    o = Oracle(s.pos, s.h, s.m).lj(eps, sigma)
    assert np.max(np.abs(o["force"])) < 1e-12 * np.max(o["f_abs"])
    rc = ORACLE_GAMMA * float(s.h[0])
    U = lambda r: 4.0 * eps * ((sigma / r) ** 12 - (sigma / r) ** 6)
    e = 0.5 * sum(c * U(a * math.sqrt(q)) for q, c in shells.items() if a * math.sqrt(q) < rc)
    assert np.allclose(o["energy"], e, rtol=1e-12)


def test_lj_force_is_minus_energy_gradient():
    """Jittered lattice: the force on a particle equals minus the fp64 central
    difference of the total energy, and the forces sum to zero."""
    s = lj_set(8, 2, jitter=0.2, rc_over_a=2.2)
    sigma, eps = 1.0 / 8, 1.0
    o = Oracle(s.pos, s.h, s.m)
    f = o.lj(eps, sigma)
    assert np.all(np.abs(f["force"].sum(0)) < 1e-10 * f["f_abs"].sum(0))
    d = 1e-6
    for k in (0, 17, 300, 511):
        for c in range(3):
            fd = -(o.lj_energy_moved(eps, sigma, k, c, d) - o.lj_energy_moved(eps, sigma, k, c, -d)) / (2 * d)
            assert abs(fd - f["force"][k, c]) < 1e-6 * f["f_abs"][k, c] + 1e-9, (k, c)
