"""GPU parity of the density loop (sorted-pair sweep and plain cell list)
against the fp64 oracle, through the C ABI.  Counts must match exactly; rho and
wcount within 1e-5 relative; drho_dh within 1e-5 of its sum of absolute terms."""
import math

import numpy as np
import pytest
import torch

from gpu_common import compare_density, oracle_for, run_density, upload, dev
from synth import uniform_set, plummer_set, lattice_set, h_for_neighbours, GAMMA, ParticleSet

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_1804_06231_amd as pvl
    c = pvl.Context(0)
    yield c
    c.close()


def _flush(msg):
    print(msg, flush=True)


@pytest.mark.parametrize("algo", ["sorted", "plain"])
def test_uniform_32k_grid8(ctx, algo):
    """32768 uniform particles, constant h (48 neighbours), 8^3 cells."""
    _flush(f"uniform-32k grid 8 {algo}")
    s = uniform_set(32768, 1, hmode="const")
    _, out = run_density(ctx, s, algo, grid=8)
    ref = oracle_for(s).density()
    compare_density(out, ref, label=f"32k-{algo}")


def test_uniform_32k_auto_and_finest_grid(ctx):
    s = uniform_set(32768, 1, hmode="const")
    ref = oracle_for(s).density()
    for algo, grid in [("sorted", None), ("plain", None), ("plain", 14), ("sorted", 10)]:
        _flush(f"uniform-32k {algo} grid {grid}")
        cells, out = run_density(ctx, s, algo, grid=grid)
        compare_density(out, ref, label=f"32k-{algo}-{grid}")
        if grid is None:
            assert cells.info()["grid"] == (14, 14, 14)


@pytest.mark.parametrize("seed,n,g,box", [
    (11, 1000, 3, (1.0, 1.0, 1.0)),
    (12, 777, 4, (1.0, 1.0, 1.0)),
    (13, 3001, 5, (1.0, 1.0, 1.0)),
    (14, 2500, None, (1.0, 1.5, 0.75)),
])
@pytest.mark.parametrize("algo", ["sorted", "plain"])
def test_small_ragged(ctx, seed, n, g, box, algo):
    """Odd particle counts, 3..5 cells per side, lognormal h, rectangular box."""
    _flush(f"ragged seed {seed} n {n} grid {g} {algo}")
    rng = np.random.Generator(np.random.PCG64(seed))
    L = np.asarray(box)
    pos = (rng.random((n, 3)) * L).astype(np.float32)
    gg = g if g is not None else 3
    Hcap = 0.95 * float(L.min()) / gg
    h = (min(h_for_neighbours(n, 30), Hcap / GAMMA / 1.8) *
         np.exp(0.2 * rng.standard_normal(n))).astype(np.float32)
    h = np.minimum(h, np.float32(Hcap / GAMMA))
    from synth.generators import _fix_by_nudging_h
    h = _fix_by_nudging_h(pos, h, np.asarray(box), seed)
    m = ((rng.random(n) + 0.5) / n).astype(np.float32)
    s = ParticleSet(pos, h, m, tuple(box), seed, "ragged")
    _, out = run_density(ctx, s, algo, grid=g)
    ref = oracle_for(s).density()
    compare_density(out, ref, label=f"ragged-{seed}-{algo}")


def test_positions_outside_box_are_wrapped(ctx):
    s = uniform_set(4000, 21, hmode="lognormal")
    shift = np.random.Generator(np.random.PCG64(2)).integers(-2, 3, (s.n, 3)).astype(np.float32)
    s2 = ParticleSet(s.pos + shift, s.h, s.m, s.box, 21, "shifted")
    _, a = run_density(ctx, s, "sorted")
    _, b = run_density(ctx, s2, "sorted")
    ref = oracle_for(s).density()
    compare_density(b, ref, label="shifted")
    assert np.array_equal(a[3], b[3])


def test_lattice_counts(ctx):
    """Simple cubic lattice: every particle has exactly the shell count."""
    for R2, expect in [(4.5, 32), (5.5, 56)]:
        s = lattice_set(32, math.sqrt(R2))
        _, out = run_density(ctx, s, "sorted")
        assert np.all(out[3] == expect)
        ref = oracle_for(s).density()
        compare_density(out, ref, label=f"lattice-{R2}")


def test_empty_and_tiny(ctx):
    import paper_1804_06231_amd as pvl
    d = dev()
    e = torch.empty((0, 3), dtype=torch.float32, device=d)
    z = torch.empty(0, dtype=torch.float32, device=d)
    cells = ctx.build_cells(e, z, z, (1.0, 1.0, 1.0), grid=4)
    ctx.sort_cells(cells)
    out = ctx.density(cells)
    ctx.check()
    assert all(t.numel() == 0 for t in out)
    # one particle: only its self term
    s = ParticleSet(np.array([[0.3, 0.7, 0.1]], np.float32), np.array([0.05], np.float32),
                    np.array([2.0], np.float32), (1.0, 1.0, 1.0), 0, "one")
    _, out = run_density(ctx, s, "sorted")
    H = GAMMA * 0.05
    assert out[3][0] == 0
    assert abs(out[0][0] - 2.0 * 8 / (math.pi * H ** 3)) < 1e-5 * out[0][0]
    # two particles, one pair in range
    s = ParticleSet(np.array([[0.1, 0.1, 0.1], [0.98, 0.1, 0.1]], np.float32),
                    np.array([0.07, 0.07], np.float32), np.array([1.0, 1.0], np.float32),
                    (1.0, 1.0, 1.0), 0, "two")
    _, out = run_density(ctx, s, "sorted", grid=4)
    compare_density(out, oracle_for(s, 4).density(), label="two")
    assert list(out[3]) == [1, 1]


@pytest.mark.parametrize("algo", ["sorted", "plain"])
def test_equal_and_mixed_masses(ctx, algo):
    """Work items whose cell and neighbours share one mass take the unit-mass
    steps; items next to a different mass take the general ones.  Both, and
    the seams between them, give the oracle's results."""
    base = uniform_set(20000, 41, hmode="lognormal")
    x = base.pos[:, 0]
    variants = {
        "equal": np.full(base.n, 1.0 / base.n, np.float32),
        "two-regions": np.where(x < 0.3, 2.0 / base.n, 1.0 / base.n).astype(np.float32),
        "one-odd": np.where(np.arange(base.n) == 777, 3.0 / base.n, 1.0 / base.n).astype(np.float32),
    }
    for name, m in variants.items():
        _flush(f"masses {name} {algo}")
        s = ParticleSet(base.pos, base.h, m, base.box, 41, name)
        _, out = run_density(ctx, s, algo)
        compare_density(out, oracle_for(s).density(), label=f"masses-{name}-{algo}")


def test_heavy_cell_near_max_occupancy(ctx):
    """Most particles packed in one cell (occupancy ~8000, near the largest the
    per-cell sort supports) next to nearly empty cells."""
    import paper_1804_06231_amd as pvl
    rng = np.random.Generator(np.random.PCG64(31))
    n_dense, n_bg = 8000, 600
    dense = (0.34 + 0.3 * rng.random((n_dense, 3))).astype(np.float32)   # inside cell (1,1,1) of 3^3
    bg = rng.random((n_bg, 3)).astype(np.float32)
    pos = np.concatenate([dense, bg])
    n = pos.shape[0]
    h = np.full(n, 0.02, np.float32)
    h[n_dense:] = 0.15
    from synth.generators import _fix_by_nudging_h
    h = _fix_by_nudging_h(pos, h, 1.0, 1)
    m = np.full(n, 1.0 / n, np.float32)
    s = ParticleSet(pos, h, m, (1.0, 1.0, 1.0), 31, "heavy")
    for algo in ("sorted", "plain"):
        cells, out = run_density(ctx, s, algo, grid=3)
        assert 4096 < cells.info()["max_occupancy"] <= pvl.PV_MAX_CELL
        compare_density(out, oracle_for(s, 3).density(), label=f"heavy-{algo}")


def test_overflow_and_grid_errors_are_reported(ctx):
    import paper_1804_06231_amd as pvl
    rng = np.random.Generator(np.random.PCG64(41))
    pos = (0.4 + 0.1 * rng.random((9000, 3))).astype(np.float32)      # 9000 in one cell
    h = np.full(9000, 0.15, np.float32)                               # H = 0.27: grid 3
    m = np.full(9000, 1e-4, np.float32)
    s = ParticleSet(pos, h, m, (1.0, 1.0, 1.0), 0, "over")
    p, hh, mm = upload(s)
    with pytest.raises(pvl.PVError, match="EOVERFLOW"):
        ctx.build_cells(p, hh, mm, (1.0, 1.0, 1.0), grid=None)
    ctx.check()
    cells = ctx.build_cells(p, hh, mm, (1.0, 1.0, 1.0), grid=4)    # explicit: async report
    ctx.sort_cells(cells)
    ctx.density(cells)
    with pytest.raises(pvl.PVError, match="EOVERFLOW"):
        ctx.check()
    # grid finer than the largest cut-off
    s = uniform_set(3000, 42, hmode="const")
    p, hh, mm = upload(s)
    cells = ctx.build_cells(p, hh, mm, (1.0, 1.0, 1.0), grid=12)
    ctx.sort_cells(cells)
    ctx.density(cells)
    with pytest.raises(pvl.PVError, match="EGRID"):
        ctx.check()
    ctx.check()                                                     # cleared
    _, out = run_density(ctx, s, "sorted")                          # and usable again
    compare_density(out, oracle_for(s).density(), label="after-errors")


def test_flagged_error_leaves_no_stale_outputs(ctx):
    """A sweep after a device-detected error writes NaN (counts -1) instead
    of leaving its outputs as they were; the differentiable entry point
    raises at once, and the next call on the same context is correct."""
    import paper_1804_06231_amd as pvl
    s = uniform_set(3000, 43, hmode="const")
    p, hh, mm = upload(s)
    cells = ctx.build_cells(p, hh, mm, (1.0, 1.0, 1.0), grid=12)    # finer than the cut-off
    ctx.sort_cells(cells)
    out = [torch.zeros(s.n, device=dev()) for _ in range(3)] + \
          [torch.zeros(s.n, dtype=torch.int32, device=dev())]
    ctx.density(cells, "sorted", out)
    torch.cuda.synchronize()
    assert all(torch.isnan(t).all().item() for t in out[:3])
    assert (out[3] == -1).all().item()
    with pytest.raises(pvl.PVError, match="EGRID"):
        ctx.check()
    pg = p.clone().requires_grad_(True)
    with pytest.raises(pvl.PVError, match="EGRID"):
        pvl.density(pg, mm, hh, grid=12)
    rho, wc, dh, nc = pvl.density(pg, mm, hh)                       # auto grid, clean again
    (rho * rho).sum().backward()
    ref = oracle_for(s).density()
    compare_density([t.detach().cpu().numpy() for t in (rho, wc, dh, nc)], ref,
                    label="after-flag")
    assert torch.isfinite(pg.grad).all().item()


def test_deterministic_and_permutation_invariant(ctx):
    s = uniform_set(20000, 51, hmode="lognormal")
    _, a = run_density(ctx, s, "sorted")
    _, b = run_density(ctx, s, "sorted")
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    perm = np.random.Generator(np.random.PCG64(5)).permutation(s.n)
    sp = ParticleSet(s.pos[perm], s.h[perm], s.m[perm], s.box, 0, "perm")
    _, c = run_density(ctx, sp, "sorted")
    # the cell-ordered layout is sorted by original index, so a permuted input
    # gives the same counts and values within rounding of a different order
    assert np.array_equal(c[3], a[3][perm])
    assert np.max(np.abs(c[0] - a[0][perm]) / a[0][perm]) < 2e-6


def test_sorted_lists_are_sorted_permutations(ctx):
    s = uniform_set(30000, 61, hmode="lognormal")
    cells, _ = run_density(ctx, s, "sorted")
    cs, order, srt = [t.cpu().numpy() for t in cells.export()]
    srt = srt.view(np.uint16)
    g = cells.info()["grid"][0]
    pos = s.pos.astype(np.float64)[order]
    cell_xyz = np.floor(pos * g)
    rel = pos - cell_xyz / g
    dirs = [(1, y, z) for y in (-1, 0, 1) for z in (-1, 0, 1)] + [(0, 1, z) for z in (-1, 0, 1)] + [(0, 0, 1)]
    for c in np.random.Generator(np.random.PCG64(1)).choice(cs.size - 1, 200, replace=False):
        a, b = cs[c], cs[c + 1]
        cnt = b - a
        for si, d in enumerate(dirs):
            lst = srt[si, a:b].astype(np.int64)
            assert np.array_equal(np.sort(lst), np.arange(cnt))
            e = np.asarray(d, np.float64) / np.linalg.norm(d)
            key = rel[a:b] @ e
            assert np.all(np.diff(key[lst]) >= -1e-6)


def test_census_sorted_vs_plain(ctx):
    """The sorted sweep inspects far fewer pairs than the plain cell list and
    never drops an in-range pair (in-range totals agree)."""
    s = uniform_set(32768, 71, hmode="const")
    ctx.set_census(True)
    try:
        _, a = run_density(ctx, s, "sorted", grid=8)
        cs = ctx.census()
        _, b = run_density(ctx, s, "plain", grid=8)
        cp = ctx.census()
    finally:
        ctx.set_census(False)
    assert cs[1] == cp[1] == int(a[3].sum())
    assert cs[0] >= cs[1]
    n = s.n
    # plain: each receiver tests the 27-cell stencil, itself excluded
    cells_count = np.bincount(
        (np.floor(s.pos.astype(np.float64) * 8).astype(int) @ np.array([64, 8, 1])), minlength=512)
    assert cp[0] == int(sum(cells_count[c] * sum(
        cells_count[((c // 64 + dx) % 8) * 64 + ((c // 8 % 8 + dy) % 8) * 8 + (c % 8 + dz) % 8]
        for dx in (-1, 0, 1) for dy in (-1, 0, 1) for dz in (-1, 0, 1)) for c in range(512)) - n)
    assert cs[0] < 0.2 * cp[0]
    # the tiled sweeps execute at least the candidates of the exact bounds
    assert cs[2] >= cs[0] and cp[2] >= cp[0]
    # the sorted candidates by definition (fp64, no rounding slack): the 26
    # neighbour cells' pairs with (x_j - x_i) . d/|d| < H_i, the own cell's
    # with |x_j - x_i| < H_i; the GPU's slack of 2^-16 of the cell edges can
    # only add the rare pairs within it of a bound
    exact = _census_by_definition(s, 8)
    assert exact <= cs[0] <= exact * 1.002, (exact, cs[0])
    print(f"census per particle: sorted {cs[0] / n:.1f} (exact {exact / n:.1f}, tiled slots "
          f"{cs[2] / n:.1f}), plain {cp[0] / n:.1f} (slots {cp[2] / n:.1f}), in range {cs[1] / n:.1f}")


def _census_by_definition(s, g):
    x = s.pos.astype(np.float64)
    H = 1.825742 * s.h.astype(np.float64)
    cid = np.floor(x * g).astype(np.int64) % g
    flat = (cid[:, 0] * g + cid[:, 1]) * g + cid[:, 2]
    order = np.argsort(flat, kind="stable")
    bounds = np.searchsorted(flat[order], np.arange(g ** 3 + 1))
    total = 0
    for c in range(g ** 3):
        ia = order[bounds[c]:bounds[c + 1]]
        ca = np.array([c // (g * g), c // g % g, c % g])
        for d in np.array(np.meshgrid([-1, 0, 1], [-1, 0, 1], [-1, 0, 1], indexing="ij")).reshape(3, -1).T:
            cb = (ca + d) % g
            b = (cb[0] * g + cb[1]) * g + cb[2]
            ib = order[bounds[b]:bounds[b + 1]]
            rel = x[ib][None, :, :] - x[ia][:, None, :]
            rel -= np.round(rel)                     # minimum image (unit box)
            if not d.any():
                cand = np.abs(rel[:, :, 0]) < H[ia][:, None]
                total += int(cand.sum()) - ia.size    # self excluded
            else:
                e = d / np.linalg.norm(d)
                total += int(((rel @ e) < H[ia][:, None]).sum())
    return total


def test_clustered_small(ctx):
    s = plummer_set(60000, 81, n_spheres=8)
    for algo in ("sorted", "plain"):
        _flush(f"clustered-60k {algo}")
        cells, out = run_density(ctx, s, algo)
        compare_density(out, oracle_for(s).density(), label=f"clustered-{algo}")


@pytest.fixture(scope="module")
def clustered_ref():
    s = plummer_set(40000, 82, n_spheres=16)
    o = oracle_for(s)
    rng = np.random.Generator(np.random.PCG64(83))
    G = rng.standard_normal(s.n).astype(np.float32)
    return s, o.density(), G, o.grad(G.astype(np.float64))


@pytest.mark.parametrize("chunk,wgs,task_sort,reach", [
    (32, 1, 0, 0), (64, 2, 1, 1), (128, 8, 0, 1), (256, 3, 1, 1), (48, 5, 1, 0)])
def test_tuning_parameters_keep_results(ctx, clustered_ref, chunk, wgs, task_sort, reach):
    """Every tuning setting gives the oracle's results: cells larger than the
    chunk are split into several work items, receivers may be reach-ordered."""
    s, ref, G, gref = clustered_ref
    saved = {sw: ctx.get_param("queue_wgs", sw) for sw in ("density", "adjoint")}
    for sw in ("density", "adjoint"):
        ctx.set_param("chunk", chunk, sw)
        ctx.set_param("queue_wgs", wgs, sw)
        ctx.set_param("task_sort", task_sort, sw)
        ctx.set_param("reach_order", reach, sw)
    try:
        _flush(f"tuning chunk={chunk} wgs={wgs} task_sort={task_sort} reach={reach}")
        cells, out = run_density(ctx, s, "sorted")
        assert cells.info()["max_occupancy"] > 2 * chunk
        compare_density(out, ref, label=f"chunk {chunk}")
        gp, gh = ctx.density_backward(cells, torch.from_numpy(G).to(dev()))
        ctx.check()
        gp, gh = gp.cpu().numpy(), gh.cpu().numpy()
        ex = np.max(np.abs(gp - gref["gx"]) / np.maximum(gref["gx_abs"], 1e-300))
        eh = np.max(np.abs(gh - gref["gh"]) / np.maximum(gref["gh_abs"], 1e-300))
        assert ex < 1e-5 and eh < 1e-5, (ex, eh)
    finally:
        for sw in ("density", "adjoint"):
            ctx.set_param("chunk", 256, sw)
            ctx.set_param("queue_wgs", saved[sw], sw)
            ctx.set_param("task_sort", 1, sw)
            ctx.set_param("reach_order", 0, sw)


@pytest.mark.parametrize("split", [0, 1])
@pytest.mark.parametrize("parts,cells", [(1, 0), (2, 0), (4, 37), (2, 2048), (4, 0)])
def test_tail_split_keeps_results(ctx, clustered_ref, parts, cells, split):
    """The queue's last cells split into parts (split 0: each a share of the
    cell's row tasks, added in part order by a second kernel; split 1: each a
    range of the cell's receivers) give the oracle's results in every sweep,
    bit-identically from run to run."""
    s, ref, G, gref = clustered_ref
    sweeps = ("density", "plain", "adjoint")
    for sw in sweeps:
        ctx.set_param("tail_parts", parts, sw)
        ctx.set_param("tail_cells", cells, sw)
        ctx.set_param("tail_split", split, sw)
    try:
        for algo in ("plain", "sorted"):
            _flush(f"tail split parts={parts} cells={cells} split={split} {algo}")
            c1, out = run_density(ctx, s, algo)
            compare_density(out, ref, label=f"tail {parts}x{cells} {algo}")
            _, out2 = run_density(ctx, s, algo, cells=c1)
            for x, y in zip(out, out2):
                assert np.array_equal(x, y)
        g = torch.from_numpy(G).to(dev())     # c1: the sorted cells
        gp, gh = ctx.density_backward(c1, g)
        gp2, gh2 = ctx.density_backward(c1, g)
        ctx.check()
        gp, gh = gp.cpu().numpy(), gh.cpu().numpy()
        assert np.array_equal(gp, gp2.cpu().numpy()) and np.array_equal(gh, gh2.cpu().numpy())
        ex = np.max(np.abs(gp - gref["gx"]) / np.maximum(gref["gx_abs"], 1e-300))
        eh = np.max(np.abs(gh - gref["gh"]) / np.maximum(gref["gh_abs"], 1e-300))
        assert ex < 1e-5 and eh < 1e-5, (ex, eh)
    finally:
        for sw in sweeps:
            ctx.set_param("tail_parts", 2, sw)
            ctx.set_param("tail_cells", 0, sw)
            ctx.set_param("tail_split", 0, sw)


@pytest.mark.parametrize("parts", [1, 4])
def test_xcd_ranges_keep_results(ctx, clustered_ref, parts):
    """Work items taken by die ranges (large-cell chunks first, then each
    die's range of single-chunk items, then the split tail) give results
    bit-identical to the one queue in every sweep, and the oracle's."""
    s, ref, G, gref = clustered_ref
    sweeps = ("density", "plain", "adjoint")
    g = torch.from_numpy(G).to(dev())
    outs = {}
    try:
        for x in (0, 1):
            for sw in sweeps:
                ctx.set_param("xcd_ranges", x, sw)
                ctx.set_param("tail_parts", parts, sw)
            res = []
            for algo in ("plain", "sorted"):
                _flush(f"xcd ranges={x} parts={parts} {algo}")
                c1, out = run_density(ctx, s, algo)
                compare_density(out, ref, label=f"xcd {x} {algo}")
                res.extend(out)
            gp, gh = ctx.density_backward(c1, g)
            ctx.check()
            res.extend([gp.cpu().numpy(), gh.cpu().numpy()])
            outs[x] = res
        for a, b in zip(outs[0], outs[1]):
            assert np.array_equal(a, b)
        gp, gh = outs[1][-2], outs[1][-1]
        ex = np.max(np.abs(gp - gref["gx"]) / np.maximum(gref["gx_abs"], 1e-300))
        eh = np.max(np.abs(gh - gref["gh"]) / np.maximum(gref["gh_abs"], 1e-300))
        assert ex < 1e-5 and eh < 1e-5, (ex, eh)
    finally:
        for sw in sweeps:
            ctx.set_param("xcd_ranges", 0, sw)
            ctx.set_param("tail_parts", 2, sw)


@pytest.mark.parametrize("group", [1, 3, 8, 0])
def test_cell_groups_keep_results(ctx, clustered_ref, group):
    """Runs of small cells swept as one work item (up to `group` cells of a
    z-row whose particles fit one chunk) give the oracle's results in the
    density and adjoint sweeps, bit-identically from run to run, with the
    same exact neighbour counts as one cell per item."""
    s, ref, G, gref = clustered_ref
    for sw in ("density", "adjoint"):
        ctx.set_param("group", group, sw)
    try:
        _flush(f"cell groups {group}")
        c1, out = run_density(ctx, s, "sorted")
        compare_density(out, ref, label=f"group {group}")
        _, out2 = run_density(ctx, s, "sorted", cells=c1)
        for x, y in zip(out, out2):
            assert np.array_equal(x, y)
        g = torch.from_numpy(G).to(dev())
        gp, gh = ctx.density_backward(c1, g)
        gp2, gh2 = ctx.density_backward(c1, g)
        ctx.check()
        gp, gh = gp.cpu().numpy(), gh.cpu().numpy()
        assert np.array_equal(gp, gp2.cpu().numpy()) and np.array_equal(gh, gh2.cpu().numpy())
        ex = np.max(np.abs(gp - gref["gx"]) / np.maximum(gref["gx_abs"], 1e-300))
        eh = np.max(np.abs(gh - gref["gh"]) / np.maximum(gref["gh_abs"], 1e-300))
        assert ex < 1e-5 and eh < 1e-5, (ex, eh)
        # small cells on the finest grid (11^3 cells, about 25 particles per
        # cell): runs of up to eight cells
        u = uniform_set(32768, 5, hmode="jitter")
        _, ou = run_density(ctx, u, "sorted")
        compare_density(ou, oracle_for(u).density(), label=f"group {group} fine grid")
    finally:
        for sw in ("density", "adjoint"):
            ctx.set_param("group", 0, sw)


def test_autotune(ctx, clustered_ref):
    """The autotuner keeps a setting at least as fast as the one in place, and
    the tuned sweeps still give the oracle's results."""
    import paper_1804_06231_amd as pvl
    s, ref, G, gref = clustered_ref
    c2 = pvl.Context(0)
    try:
        pos, h, m = upload(s)
        cells = c2.build_cells(pos, h, m, s.box)
        c2.sort_cells(cells)
        before, after, p = c2.autotune(cells, "density", reps=2)
        _flush(f"autotune density: {before:.3f} -> {after:.3f} ms, {p}")
        assert after <= before and p["chunk"] in (64, 128, 256) and 1 <= p["queue_wgs"] <= 8
        g = torch.from_numpy(G).to(dev())
        before_a, after_a, pa = c2.autotune(cells, "adjoint", g, reps=2)
        _flush(f"autotune adjoint: {before_a:.3f} -> {after_a:.3f} ms, {pa}")
        assert after_a <= before_a and pa["reach_order"] == 0
        before_p, after_p, pp = c2.autotune(cells, "plain", reps=1)
        _flush(f"autotune plain: {before_p:.3f} -> {after_p:.3f} ms, {pp}")
        assert after_p <= before_p
        out = [t.cpu().numpy() for t in c2.density(cells, "sorted")]
        compare_density(out, ref, label="tuned")
        out = [t.cpu().numpy() for t in c2.density(cells, "plain")]
        compare_density(out, ref, label="tuned plain")
        gp, gh = c2.density_backward(cells, g)
        c2.check()
        ex = np.max(np.abs(gp.cpu().numpy() - gref["gx"]) / np.maximum(gref["gx_abs"], 1e-300))
        assert ex < 1e-5
        with pytest.raises(pvl.PVError):
            c2.autotune(c2.build_cells(pos, h, m, s.box), "density")   # not sorted
    finally:
        c2.close()


def test_kernel_timing(ctx, clustered_ref):
    """The context times the persistent sweep kernel of each density call
    with events on its stream (oldest first, at most the ring's size), leaves
    results unchanged, records nothing once disabled, and stays out of a
    captured graph."""
    s, ref, G, gref = clustered_ref
    _flush("kernel timing")
    cells, out0 = run_density(ctx, s, "sorted")
    outs = tuple(torch.from_numpy(x).to(dev()) for x in out0)
    ctx.set_kernel_timing(True)
    try:
        for _ in range(3):
            ctx.density(cells, "sorted", outs)
        ts = ctx.kernel_times(8)
        assert len(ts) == 3 and all(0.0 < t < 1000.0 for t in ts), ts
        for x, y in zip(out0, outs):
            assert np.array_equal(x, y.cpu().numpy())
        assert len(ctx.kernel_times(2)) == 2
        # a captured density call records nothing (the events stay outside)
        torch.cuda.synchronize()
        ctx.set_kernel_timing(True)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            ctx.density(cells, "sorted", outs)
        torch.cuda.synchronize()
        assert ctx.kernel_times(8) == []
        g.replay()
        torch.cuda.synchronize()
        for x, y in zip(out0, outs):
            assert np.array_equal(x, y.cpu().numpy())
    finally:
        ctx.set_kernel_timing(False)
    ctx.density(cells, "sorted", outs)
    assert ctx.kernel_times(8) == []
    cells.free()


def test_autotune_cache(ctx, clustered_ref, tmp_path):
    """A tuned setting stored in the cache is applied by a later context
    without timing, for the same size class."""
    import paper_1804_06231_amd as pvl
    from paper_1804_06231_amd.pvl import TuneCache
    s, ref, G, gref = clustered_ref
    path = str(tmp_path / "tune.json")
    c1, c2 = pvl.Context(0), pvl.Context(0)
    try:
        pos, h, m = upload(s)
        cells = c1.build_cells(pos, h, m, s.box)
        c1.sort_cells(cells)
        before, after, p1 = c1.autotune(cells, "density", reps=1, cache=TuneCache(path))
        assert after <= before
        cells2 = c2.build_cells(pos, h, m, s.box)
        c2.sort_cells(cells2)
        b2, a2, p2 = c2.autotune(cells2, "density", reps=1, cache=TuneCache(path))
        assert np.isnan(b2) and np.isnan(a2) and p2 == p1
        out = [t.cpu().numpy() for t in c2.density(cells2, "sorted")]
        compare_density(out, ref, label="cached setting")
    finally:
        c1.close()
        c2.close()


@pytest.mark.parametrize("group,chunk,parts", [(0, 256, 2), (1, 256, 1), (8, 256, 4), (0, 64, 2)])
def test_symmetric_own_cell_keeps_results(ctx, clustered_ref, group, chunk, parts):
    """The own cell by the symmetric pair update (each unordered pair tested
    once, both particles updated; cells larger than the chunk keep the
    gathered form) gives the oracle's density and adjoint, with the exact
    neighbour counts, bit-identically from run to run, in single-cell items,
    runs of small cells and split tail items."""
    s, ref, G, gref = clustered_ref
    for sw in ("density", "adjoint"):
        ctx.set_param("sym_self", 1, sw)
        ctx.set_param("group", group, sw)
        ctx.set_param("chunk", chunk, sw)
        ctx.set_param("tail_parts", parts, sw)
    try:
        _flush(f"symmetric own cell group={group} chunk={chunk} parts={parts}")
        c1, out = run_density(ctx, s, "sorted")
        compare_density(out, ref, label=f"sym group {group} chunk {chunk}")
        _, out2 = run_density(ctx, s, "sorted", cells=c1)
        for x, y in zip(out, out2):
            assert np.array_equal(x, y)
        g = torch.from_numpy(G).to(dev())
        gp, gh = ctx.density_backward(c1, g)
        gp2, gh2 = ctx.density_backward(c1, g)
        ctx.check()
        gp, gh = gp.cpu().numpy(), gh.cpu().numpy()
        assert np.array_equal(gp, gp2.cpu().numpy()) and np.array_equal(gh, gh2.cpu().numpy())
        ex = np.max(np.abs(gp - gref["gx"]) / np.maximum(gref["gx_abs"], 1e-300))
        eh = np.max(np.abs(gh - gref["gh"]) / np.maximum(gref["gh_abs"], 1e-300))
        assert ex < 1e-5 and eh < 1e-5, (ex, eh)
        # translation invariance of the adjoint (the symmetric update adds
        # opposite forces to the two particles of a pair)
        tot = np.abs(gp.astype(np.float64).sum(0))
        assert np.all(tot < 1e-5 * gref["gx_abs"].sum(0))
    finally:
        for sw in ("density", "adjoint"):
            ctx.set_param("sym_self", 0, sw)
            ctx.set_param("group", 0, sw)
            ctx.set_param("chunk", 256, sw)
            ctx.set_param("tail_parts", 2, sw)


@pytest.mark.parametrize("hmode", ["lognormal", "const"])
def test_symmetric_own_cell_uniform_and_mixed_masses(ctx, hmode):
    """Uniform sets (one cell per item) with the symmetric own cell: exact
    counts and oracle parity; with mixed masses the density keeps the
    gathered own cell and still matches."""
    s = uniform_set(60000, 91, hmode=hmode)
    ref = oracle_for(s).density()
    ctx.set_param("sym_self", 1, "density")
    try:
        _, out = run_density(ctx, s, "sorted")
        compare_density(out, ref, label=f"sym uniform {hmode}")
        rng = np.random.Generator(np.random.PCG64(92))
        s.m = (s.m * rng.uniform(0.5, 1.5, s.n)).astype(np.float32)
        _, out = run_density(ctx, s, "sorted")
        compare_density(out, oracle_for(s).density(), label=f"sym mixed masses {hmode}")
    finally:
        ctx.set_param("sym_self", 0, "density")
