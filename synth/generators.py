"""Seeded particle-set generators.

Every workload is a periodic box (the unit cube unless stated) of fp32 particle
positions, fp32 smoothing lengths h and fp32 masses m = 1/N.  The cut-off radius
of a receiver is H = GAMMA * h (cubic-spline support over smoothing length).

Guard band: an input is accepted only when no particle pair (i, j) has a
separation within a relative 1e-5 of the receiver's cut-off,
|r_ij - H_i| > 1e-5 * H_i, with r_ij and H_i = GAMMA * (double) h_i taken in
fp64.  Within that band the fp32 and fp64 answers to "is j a neighbour of i"
could differ; outside it they cannot, so neighbour counts can be compared
exactly.  Offending inputs are repaired deterministically: a varying h_i is
nudged, a position drawn from a uniform distribution is re-drawn from a
sub-seeded stream.

Random streams are numpy PCG64 with the seed recorded on the returned set.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
from scipy.spatial import cKDTree

__all__ = [
    "GAMMA", "GUARD", "ParticleSet", "h_for_neighbours", "finest_grid",
    "guard_violations", "uniform_set", "lattice_set", "plummer_set",
    "adjoint_set", "drift_set", "lj_set", "batched_sets", "batched_sizes", "BatchedSet", "batched_workload",
    "workload", "WORKLOADS",
]

GAMMA = 1.825742     # cubic-spline support H over smoothing length h (3D)
_WORKERS = -1        # threads of the k-d tree queries (-1: all cores)
GUARD = 1e-5         # relative guard band around every receiver's cut-off
_CHECK = 1.25e-5     # the check is a little wider than the band it enforces


@dataclasses.dataclass
class ParticleSet:
    pos: np.ndarray          # (n, 3) float32, each coordinate in [0, L)
    h: np.ndarray            # (n,) float32 smoothing length
    m: np.ndarray            # (n,) float32 mass
    box: tuple               # (Lx, Ly, Lz) as python floats
    seed: int
    name: str
    grid: int | None = None  # cells per side the workload is quoted on (None = finest legal)
    extra: dict = dataclasses.field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.pos.shape[0])

    def cutoff64(self) -> np.ndarray:
        return GAMMA * self.h.astype(np.float64)


def h_for_neighbours(n: int, ngb: float = 48.0, L: float = 1.0) -> float:
    """Smoothing length giving `ngb` expected neighbours at number density n/L^3:
    (4 pi / 3) H^3 n / L^3 = ngb, h = H / GAMMA."""
    H = L * (3.0 * ngb / (4.0 * math.pi * n)) ** (1.0 / 3.0)
    return H / GAMMA


def finest_grid(h: np.ndarray, L: float = 1.0) -> int:
    """Finest cells-per-side whose edge is not below the largest cut-off."""
    hmax = GAMMA * float(np.max(h.astype(np.float64)))
    return int(math.floor(L / (hmax * (1.0 + 4e-6))))


def _wrap32(x64: np.ndarray, L: float) -> np.ndarray:
    """Wrap fp64 coordinates into [0, L) and round to fp32 without reaching L."""
    x = np.mod(x64, L).astype(np.float32)
    x[x >= np.float32(L)] = 0.0
    return x


def guard_violations(pos: np.ndarray, h: np.ndarray, L: float = 1.0,
                     band: float = _CHECK, workers: int | None = None, subset=None,
                     tree=None) -> np.ndarray:
    """Indices i having some j with |r_ij - H_i| <= band * H_i (periodic, fp64).
    With `subset`, only those receivers are examined."""
    p = pos.astype(np.float64)
    H = GAMMA * h.astype(np.float64)
    workers = _WORKERS if workers is None else workers
    if tree is None:
        tree = cKDTree(p, boxsize=L)
    idx = np.arange(p.shape[0]) if subset is None else np.asarray(subset)
    q = p[idx]
    hi = tree.query_ball_point(q, H[idx] * (1.0 + band), return_length=True, workers=workers)
    lo = tree.query_ball_point(q, H[idx] * (1.0 - band), return_length=True, workers=workers)
    return idx[np.nonzero(hi != lo)[0]]


def _fix_by_nudging_h(pos, h, L, rng_seed):
    """Nudge offending h_i upward in small deterministic steps until clean.
    Changing h_i only changes receiver i's own neighbour test, so after the
    first full check only the nudged receivers are re-examined."""
    h = h.copy()
    tree = cKDTree(pos.astype(np.float64), boxsize=L)
    bad = guard_violations(pos, h, L, tree=tree)
    for step in range(64):
        if bad.size == 0:
            return h
        h[bad] = (h[bad].astype(np.float64) * (1.0 + 5e-5)).astype(np.float32)
        bad = guard_violations(pos, h, L, subset=bad, tree=tree)
    raise RuntimeError("guard band: h nudging did not converge")


def _fix_by_redrawing(pos, h, L, seed):
    """Re-draw offending particle positions from a sub-seeded stream (constant h)."""
    pos = pos.copy()
    for it in range(1, 64):
        bad = guard_violations(pos, h, L)
        if bad.size == 0:
            return pos
        rng = np.random.Generator(np.random.PCG64([seed, 0x6A09E667, it]))
        pos[bad] = rng.random((bad.size, 3), dtype=np.float32) * np.float32(L)
        pos[pos >= np.float32(L)] = 0.0
    raise RuntimeError("guard band: position re-draw did not converge")


def uniform_set(n: int, seed: int, hmode: str = "const", sigma: float = 0.2,
                jitter: float = 0.2, ngb: float = 48.0, L: float = 1.0,
                grid: int | None = None, name: str | None = None,
                guard: bool = True) -> ParticleSet:
    """n uniform-random particles in a periodic cube of side L.

    hmode: "const"     every h = h_for_neighbours(n)
           "lognormal" h_i = h48 * exp(sigma * z_i), z ~ N(0, 1) (median h48)
           "jitter"    h_i = h48 * U(1 - jitter, 1 + jitter)
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    pos = rng.random((n, 3), dtype=np.float32) * np.float32(L)
    pos[pos >= np.float32(L)] = 0.0
    h48 = h_for_neighbours(n, ngb, L)
    if hmode == "const":
        h = np.full(n, h48, dtype=np.float32)
    elif hmode == "lognormal":
        z = rng.standard_normal(n)
        h = (h48 * np.exp(sigma * z)).astype(np.float32)
    elif hmode == "jitter":
        u = rng.random(n)
        h = (h48 * (1.0 - jitter + 2.0 * jitter * u)).astype(np.float32)
    else:
        raise ValueError(hmode)
    if guard:
        if hmode == "const":
            pos = _fix_by_redrawing(pos, h, L, seed)
        else:
            h = _fix_by_nudging_h(pos, h, L, seed)
    m = np.full(n, 1.0 / n, dtype=np.float32)
    return ParticleSet(pos, h, m, (L, L, L), seed, name or f"uniform-{hmode}-{n}", grid)


def lattice_set(M: int, R: float, L: float = 1.0) -> ParticleSet:
    """Simple cubic lattice of M^3 particles at (i, j, k) * L / M with cut-off
    H = R * L / M.  With M a power of two every coordinate is exact in fp32."""
    a = L / M
    g = np.arange(M, dtype=np.float64) * a
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    pos = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1).astype(np.float32)
    n = M ** 3
    h = np.full(n, R * a / GAMMA, dtype=np.float32)
    m = np.full(n, 1.0 / n, dtype=np.float32)
    return ParticleSet(pos, h, m, (L, L, L), 0, f"lattice-{M}-R{R:.4f}", None)


def _plummer_points(rng, n, centre, a, L):
    """n points of a Plummer sphere of scale radius a, truncated at 10 a."""
    out = np.empty((0, 3))
    while out.shape[0] < n:
        k = int((n - out.shape[0]) * 1.05) + 16
        X = rng.random(k)
        X = np.clip(X, 1e-300, None)
        r = a / np.sqrt(X ** (-2.0 / 3.0) - 1.0)
        r = r[r <= 10.0 * a]
        v = rng.standard_normal((r.size, 3))
        v /= np.linalg.norm(v, axis=1, keepdims=True)
        out = np.concatenate([out, centre + v * r[:, None]])
    return out[:n]


def _knn_h(pos, L, ngb=48, workers=None):
    """h_i such that exactly ngb particles lie inside H_i = GAMMA h_i: H_i is the
    midpoint of the ngb-th and (ngb+1)-th neighbour distance.  Where that gap is
    narrower than twice the guard band, the widest gap among neighbours
    ngb-2 .. ngb+2 is used instead."""
    p = pos.astype(np.float64)
    workers = _WORKERS if workers is None else workers
    tree = cKDTree(p, boxsize=L)
    k = ngb + 4                                   # self + neighbours 1 .. ngb+3
    d, _ = tree.query(p, k=k, workers=workers)    # d[:, 0] = 0 (self)
    lo = d[:, ngb]
    hi = d[:, ngb + 1]
    H = 0.5 * (lo + hi)
    narrow = (hi - lo) < 4.0 * GUARD * H
    if np.any(narrow):
        idx = np.nonzero(narrow)[0]
        seg = d[idx][:, ngb - 2: ngb + 3]          # neighbours ngb-2 .. ngb+2
        gaps = np.diff(seg, axis=1)
        best = np.argmax(gaps, axis=1)
        H[idx] = 0.5 * (seg[np.arange(idx.size), best] + seg[np.arange(idx.size), best + 1])
    return (H / GAMMA).astype(np.float32)


def plummer_set(n: int, seed: int, n_spheres: int = 64, frac_uniform: float = 0.5,
                a_range=(0.01, 0.05), ngb: int = 48, L: float = 1.0,
                name: str | None = None) -> ParticleSet:
    """Clustered set: a uniform background plus Plummer spheres.

    Sphere scale radii a_s are log-uniform in a_range; sphere populations are
    proportional to a_s^3 (equal central density); centres are uniform; points
    beyond 10 a_s are rejected; everything wraps periodically.  h_i is solved so
    that every particle has exactly `ngb` neighbours (or ngb +- 2 where the
    neighbour distances crowd the guard band)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n_uni = int(round(n * frac_uniform))
    n_cl = n - n_uni
    bg = rng.random((n_uni, 3))
    a = np.exp(rng.uniform(math.log(a_range[0]), math.log(a_range[1]), n_spheres))
    centres = rng.random((n_spheres, 3))
    w = a ** 3 / np.sum(a ** 3) * n_cl
    cnt = np.floor(w).astype(np.int64)
    rem = n_cl - int(cnt.sum())
    cnt[np.argsort(-(w - cnt), kind="stable")[:rem]] += 1
    parts = [bg * L]
    for s in range(n_spheres):
        if cnt[s]:
            parts.append(_plummer_points(rng, int(cnt[s]), centres[s] * L, a[s] * L, L))
    p64 = np.concatenate(parts)
    perm = rng.permutation(n)
    pos = _wrap32(p64[perm], L)
    h = _knn_h(pos, L, ngb)
    h = _fix_by_nudging_h(pos, h, L, seed)
    m = np.full(n, 1.0 / n, dtype=np.float32)
    return ParticleSet(pos, h, m, (L, L, L), seed, name or f"plummer-{n}", None,
                       {"a_s": a, "centres": centres, "counts": cnt})


def adjoint_set(n: int, seed: int, jitter: float = 0.2, L: float = 1.0) -> ParticleSet:
    """Uniform box with h_i = h48 * U(1 - jitter, 1 + jitter) plus a perturbed copy
    of the positions (per-axis N(0, (0.05 n^{-1/3})^2), periodic) from which a
    density target is made.  The copy only feeds the target values, which are
    never compared between implementations, so it needs no guard band."""
    s = uniform_set(n, seed, hmode="jitter", jitter=jitter, L=L, name=f"adjoint-{n}")
    rng = np.random.Generator(np.random.PCG64([seed, 0xB7E15162]))
    sig = 0.05 * L * n ** (-1.0 / 3.0)
    pert = _wrap32(s.pos.astype(np.float64) + rng.normal(0.0, sig, (n, 3)), L)
    s.extra["pos_target"] = pert
    return s


def lj_set(M: int, seed: int, jitter: float = 0.2, rc_over_a: float = 2.5,
           L: float = 1.0) -> ParticleSet:
    """Molecular-dynamics-like set: a simple cubic lattice of M^3 sites (spacing
    a = L / M) with every particle displaced uniformly in [-jitter a, jitter a]^3,
    so no two particles come closer than (1 - 2 jitter) a; one cut-off
    r_c = rc_over_a * a for all (h = r_c / GAMMA); m = 1/N.  Particles that break
    the guard band get their displacement re-drawn from a sub-seeded stream."""
    a = L / M
    g = np.arange(M, dtype=np.float64) * a
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    sites = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    n = sites.shape[0]
    rng = np.random.Generator(np.random.PCG64(seed))
    pos = _wrap32(sites + rng.uniform(-jitter * a, jitter * a, (n, 3)), L)
    h = np.full(n, rc_over_a * a / GAMMA, dtype=np.float32)
    for it in range(1, 64):
        bad = guard_violations(pos, h, L)
        if bad.size == 0:
            break
        r2 = np.random.Generator(np.random.PCG64([seed, 0xBB67AE85, it]))
        pos[bad] = _wrap32(sites[bad] + r2.uniform(-jitter * a, jitter * a, (bad.size, 3)), L)
    else:
        raise RuntimeError("guard band: lattice jitter re-draw did not converge")
    m = np.full(n, 1.0 / n, dtype=np.float32)
    return ParticleSet(pos, h, m, (L, L, L), seed, f"lj-{M}", None,
                       {"sigma": a, "rc": rc_over_a * a})


def drift_set(n: int, seed: int, steps: int, dmax: float, L: float = 1.0) -> ParticleSet:
    """Uniform particles with lognormal h plus `steps` displacement vectors
    (extra["disp"], each (n, 3) fp32, |d| <= dmax per particle and step, random
    directions).  h is nudged until the guard band holds for the starting
    positions and for every configuration pos + sum of the first k
    displacements (fp64), so neighbour counts can be compared exactly at each
    step."""
    s = uniform_set(n, seed, hmode="lognormal", L=L, guard=False, name=f"drift-{n}")
    rng = np.random.Generator(np.random.PCG64([seed, 0x3C6EF372]))
    disp = []
    for _ in range(steps):
        v = rng.standard_normal((n, 3))
        v /= np.linalg.norm(v, axis=1, keepdims=True)
        r = dmax * rng.random(n) ** (1.0 / 3.0)
        disp.append((v * r[:, None]).astype(np.float32))
    confs = [s.pos.astype(np.float64)]
    for d in disp:
        confs.append(confs[-1] + d.astype(np.float64))
    h = s.h.copy()
    for _ in range(32):
        clean = True
        for x in confs:
            xw = np.mod(x, L)
            bad = guard_violations(xw, h, L)
            if bad.size:
                clean = False
                h[bad] = (h[bad].astype(np.float64) * (1.0 + 5e-5)).astype(np.float32)
        if clean:
            break
    else:
        raise RuntimeError("guard band: drift set did not settle")
    s.h = h
    s.extra["disp"] = disp
    s.extra["positions"] = confs
    return s


def batched_sets(nbox: int = 256, seed: int = 5, nmin: int = 4096, nmax: int = 262144,
                 n_spheres: int = 64, only: list | None = None) -> list:
    """nbox independent unit boxes with log-uniform particle counts in [nmin, nmax];
    even boxes are uniform with lognormal h, odd boxes follow the clustered
    recipe (half uniform, half in `n_spheres` Plummer spheres, kNN h) at their
    own size, so every clustered box has the same density contrast.  `only`
    restricts which boxes are built (the sizes and seeds of the others are
    still drawn)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sizes = np.rint(np.exp(rng.uniform(math.log(nmin), math.log(nmax), nbox))).astype(np.int64)
    seeds = rng.integers(1, 2 ** 31 - 1, nbox)
    out = []
    for b in range(nbox):
        if only is not None and b not in only:
            out.append(None)
            continue
        nb = int(sizes[b])
        if b % 2 == 0:
            out.append(uniform_set(nb, int(seeds[b]), hmode="lognormal", name=f"box{b}-uniform-{nb}"))
        else:
            out.append(plummer_set(nb, int(seeds[b]), n_spheres=n_spheres,
                                   name=f"box{b}-clustered-{nb}"))
    return out


def batched_sizes(nbox: int = 256, seed: int = 5, nmin: int = 4096, nmax: int = 262144):
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.rint(np.exp(rng.uniform(math.log(nmin), math.log(nmax), nbox))).astype(np.int64)


@dataclasses.dataclass
class BatchedSet:
    """Independent periodic boxes laid end to end: box b holds particles
    offsets[b] .. offsets[b+1] of the concatenated arrays."""
    sets: list               # ParticleSet per box
    offsets: np.ndarray      # (nbox + 1,) int64
    pos: np.ndarray          # (N, 3) float32
    h: np.ndarray            # (N,) float32
    m: np.ndarray            # (N,) float32
    boxes: list              # (Lx, Ly, Lz) per box
    grids: list              # cells per side per box (finest legal)
    seed: int
    name: str

    @property
    def n(self) -> int:
        return int(self.offsets[-1])

    @property
    def nbox(self) -> int:
        return len(self.sets)


def _one_box(args):
    nbox, seed, nmin, nmax, b = args
    return batched_sets(nbox, seed, nmin, nmax, only=[b])[b]


def _single_threaded_trees():
    global _WORKERS
    _WORKERS = 1


def batched_workload(nbox: int = 256, seed: int = 5, nmin: int = 4096, nmax: int = 262144,
                     name: str | None = None, progress=None, jobs: int | None = None) -> BatchedSet:
    """The boxes of batched_sets, concatenated, each quoted on its finest legal
    grid (cells per side = floor(L / largest cut-off), at least 3).  Boxes are
    drawn in `jobs` worker processes (fresh interpreters; each box depends only
    on its own seed, so the result does not depend on jobs)."""
    import concurrent.futures as cf
    import multiprocessing as mp
    import os
    if jobs is None:
        jobs = min(16, os.cpu_count() or 1)
    work = [(nbox, seed, nmin, nmax, b) for b in range(nbox)]
    sets = []
    if jobs > 1:
        with cf.ProcessPoolExecutor(jobs, mp_context=mp.get_context("spawn"),
                                    initializer=_single_threaded_trees) as ex:
            for b, s in enumerate(ex.map(_one_box, work, chunksize=1)):
                sets.append(s)
                if progress is not None and (b + 1) % 32 == 0:
                    progress(f"box {b + 1}/{nbox}")
    else:
        for b, w in enumerate(work):
            sets.append(_one_box(w))
            if progress is not None and (b + 1) % 32 == 0:
                progress(f"box {b + 1}/{nbox}")
    offsets = np.zeros(nbox + 1, dtype=np.int64)
    offsets[1:] = np.cumsum([s.n for s in sets])
    grids = [finest_grid(s.h, s.box[0]) for s in sets]
    if min(grids) < 3:
        raise ValueError("a box's largest cut-off leaves fewer than 3 cells per side")
    return BatchedSet(sets, offsets, np.concatenate([s.pos for s in sets]),
                      np.concatenate([s.h for s in sets]), np.concatenate([s.m for s in sets]),
                      [s.box for s in sets], grids, seed, name or f"batched-{nbox}")


# Named workloads (sizes of the paper-shaped benchmark configurations).
WORKLOADS = {
    # 32768 uniform particles, constant h (48 neighbours), quoted on 8^3 cells.
    "uniform-32k": dict(kind="uniform", n=32768, hmode="const", grid=8, seed=1),
    # 2^20 uniform particles, lognormal h (sigma 0.2) around the 48-neighbour value.
    "uniform-1m-lognormal": dict(kind="uniform", n=1 << 20, hmode="lognormal", grid=None, seed=2),
    # 2^22 clustered particles: 50% uniform + 64 Plummer spheres, kNN h (48 neighbours).
    "clustered-4m": dict(kind="plummer", n=1 << 22, seed=3),
    # 2^20 uniform particles, h jittered +-20%, with a perturbed copy for the target.
    "adjoint-1m": dict(kind="adjoint", n=1 << 20, seed=4),
    # 10^6 particles on a jittered 100^3 lattice, one cut-off 2.5 lattice spacings
    # (a molecular-dynamics shape for the Lennard-Jones forces).
    "lj-1m": dict(kind="lj", M=100, seed=77, rc=2.5),
    # 256 unit boxes of 4096 .. 262144 particles (log-uniform), alternately uniform
    # with lognormal h and Plummer-clustered, ~15.4M particles in all.
    "batched-256": dict(kind="batched", nbox=256, seed=5),
}


def workload(name: str, progress=None, **over):
    """The named workload: a ParticleSet, or a BatchedSet for "batched-256"."""
    spec = dict(WORKLOADS[name])
    spec.update(over)
    kind = spec.pop("kind")
    if kind == "batched":
        return batched_workload(spec["nbox"], spec["seed"], name=name, progress=progress)
    if kind == "uniform":
        return uniform_set(spec["n"], spec["seed"], hmode=spec["hmode"], grid=spec.get("grid"),
                           name=name)
    if kind == "plummer":
        return plummer_set(spec["n"], spec["seed"], name=name)
    if kind == "adjoint":
        return adjoint_set(spec["n"], spec["seed"])
    if kind == "lj":
        return lj_set(spec["M"], spec["seed"], rc_over_a=spec["rc"])
    raise ValueError(kind)
