"""Batched boxes: independent periodic boxes of different sizes, particle counts
and clustering in one cell structure, swept by one persistent work-queue launch
per stage (density, adjoint), compared with the fp64 oracle box by box, with
the same boxes run one at a time, and through a captured HIP graph."""
import numpy as np
import pytest
import torch

from gpu_common import compare_density, dev, oracle_for
from synth import uniform_set, plummer_set, lattice_set, finest_grid

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_1804_06231_amd as pvl
    c = pvl.Context(0)
    yield c
    c.close()


def _boxes():
    """Nine boxes: uniform with lognormal / jittered / constant h, clustered,
    a lattice, boxes of edge 0.5 and 2, a box with no particles."""
    sets = [
        uniform_set(3000, 21, hmode="lognormal"),
        plummer_set(9000, 22, n_spheres=3),
        uniform_set(1000, 23, hmode="jitter", L=0.5),
        uniform_set(20000, 24, hmode="const"),
        None,                                             # empty box
        plummer_set(4000, 25, n_spheres=1, frac_uniform=0.3),
        lattice_set(10, 1.5),
        uniform_set(7000, 26, hmode="lognormal", L=2.0),
        uniform_set(1200, 27, hmode="const"),
    ]
    grids = [3 if s is None else max(3, finest_grid(s.h, s.box[0])) for s in sets]
    # one box on a coarser grid than its finest (more particles per cell)
    grids[3] = max(3, grids[3] // 2)
    return sets, grids


def _concat(sets):
    ns = [0 if s is None else s.n for s in sets]
    off = np.zeros(len(sets) + 1, dtype=np.int64)
    off[1:] = np.cumsum(ns)
    cat = lambda f, shape: np.concatenate([np.zeros(shape, np.float32) if s is None else f(s)
                                           for s in sets])
    pos = cat(lambda s: s.pos, (0, 3))
    h = cat(lambda s: s.h, (0,))
    m = cat(lambda s: s.m, (0,))
    boxes = [(1.0, 1.0, 1.0) if s is None else s.box for s in sets]
    d = dev()
    return off, [torch.from_numpy(np.ascontiguousarray(a)).to(d) for a in (pos, h, m)], boxes


def _seeded_g(n, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal(n).astype(np.float32)


def _run(ctx, off, arrs, boxes, grids, G, cells=None):
    pos, h, m = arrs
    cells = ctx.build_cells_batched(off, pos, h, m, boxes, grids, cells)
    ctx.sort_cells(cells)
    out = ctx.density(cells, "sorted")
    g = torch.from_numpy(G).to(dev())
    gp, gh = ctx.density_backward(cells, g)
    ctx.check()
    torch.cuda.synchronize()
    return cells, [t.cpu().numpy() for t in out], gp.cpu().numpy(), gh.cpu().numpy()


def test_batched_matches_oracle_per_box(ctx):
    sets, grids = _boxes()
    off, arrs, boxes = _concat(sets)
    G = _seeded_g(int(off[-1]), 31)
    cells, out, gp, gh = _run(ctx, off, arrs, boxes, grids, G)
    info = cells.info()
    assert info["nbox"] == len(sets) and info["n"] == off[-1]
    assert info["ncell"] == sum(g ** 3 for g in grids)
    for b, s in enumerate(sets):
        if s is None:
            continue
        sl = slice(int(off[b]), int(off[b + 1]))
        o = oracle_for(s, grids[b])
        compare_density([a[sl] for a in out], o.density(), label=f"box {b} density")
        ref = o.grad(G[sl].astype(np.float64))
        ex = np.max(np.abs(gp[sl] - ref["gx"]) / np.maximum(ref["gx_abs"], 1e-300))
        eh = np.max(np.abs(gh[sl] - ref["gh"]) / np.maximum(ref["gh_abs"], 1e-300))
        assert ex < 1e-5 and eh < 1e-5, (b, ex, eh)


def test_batched_equals_one_box_at_a_time(ctx):
    """A box's results do not depend on the other boxes of the batch: each
    item of the queue is computed the same way whichever workgroup takes it,
    and runs of small cells are formed within each box's own rows.  Bit for
    bit with the tail split off and a fixed run length (the split set is
    chosen by cell index within the whole structure, and the automatic run
    length by its cell count, so either may differ between the batch and the
    box alone, which changes the summation order); within rounding with the
    split on."""
    sets, grids = _boxes()
    off, arrs, boxes = _concat(sets)
    G = _seeded_g(int(off[-1]), 32)
    for parts in (1, 2):
        for sw in ("density", "adjoint"):
            ctx.set_param("tail_parts", parts, sw)
            ctx.set_param("group", 4, sw)
        try:
            _, out, gp, gh = _run(ctx, off, arrs, boxes, grids, G)
            for b, s in enumerate(sets):
                if s is None:
                    continue
                sl = slice(int(off[b]), int(off[b + 1]))
                o1, a1, _ = _concat([s])
                _, out1, gp1, gh1 = _run(ctx, o1, a1, [s.box], [grids[b]], G[sl].copy())
                if parts == 1:
                    for k in range(4):
                        assert np.array_equal(out[k][sl], out1[k]), (b, k)
                    assert np.array_equal(gp[sl], gp1) and np.array_equal(gh[sl], gh1), b
                else:
                    assert np.array_equal(out[3][sl], out1[3]), b          # counts
                    for k in range(2):
                        assert np.allclose(out[k][sl], out1[k], rtol=2e-6, atol=0), (b, k)
                    scale = np.max(np.abs(out1[2]))          # drho_dh: signed sums
                    assert np.allclose(out[2][sl], out1[2], rtol=2e-6, atol=1e-6 * scale), b
        finally:
            for sw in ("density", "adjoint"):
                ctx.set_param("tail_parts", 2, sw)
                ctx.set_param("group", 0, sw)


def test_batched_auto_grid(ctx):
    """Without grids every box gets its own finest legal grid."""
    sets, _ = _boxes()
    sets = [s for s in sets if s is not None]
    off, (pos, h, m), boxes = _concat(sets)
    cells = ctx.build_cells_batched(off, pos, h, m, boxes)
    want = sum(finest_grid(s.h, s.box[0]) ** 3 for s in sets)
    assert cells.info()["ncell"] == want


def test_graph_replay_matches_eager(ctx):
    """build + sort + density + adjoint of the whole batch captured once and
    replayed; every replay (with eager work between) equals the eager run."""
    sets, grids = _boxes()
    off, arrs, boxes = _concat(sets)
    n = int(off[-1])
    G = torch.from_numpy(_seeded_g(n, 33)).to(dev())
    pos, h, m = arrs
    d = dev()
    rho, wc, dh = (torch.empty(n, device=d) for _ in range(3))
    nc = torch.empty(n, dtype=torch.int32, device=d)
    gp, gh = torch.empty((n, 3), device=d), torch.empty(n, device=d)

    cells = ctx.build_cells_batched(off, pos, h, m, boxes, grids)

    def step():
        ctx.build_cells_batched(off, pos, h, m, boxes, grids, cells)
        ctx.sort_cells(cells)
        ctx.density(cells, "sorted", (rho, wc, dh, nc))
        ctx.density_backward(cells, G, (gp, gh))

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step()
    torch.cuda.current_stream().wait_stream(side)
    ctx.check()
    torch.cuda.synchronize()
    eager = [t.clone() for t in (rho, wc, dh, nc, gp, gh)]

    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        step()
    torch.cuda.synchronize()
    for rep in range(3):
        for t in (rho, wc, dh, gp, gh):
            t.fill_(float("nan"))
        nc.fill_(-1)
        graph.replay()
        torch.cuda.synchronize()
        for k, (a, b) in enumerate(zip((rho, wc, dh, nc, gp, gh), eager)):
            assert torch.equal(a, b), (rep, k)
        ctx.check()                      # eager work between replays
        _ = (rho * 2).sum().item()
    del graph
