"""Reuse of the sorted lists over several steps (pv_drift): after moving the
particles, density and adjoint must equal the fp64 oracle's at the moved
positions, with the projected bounds widened by the displacements."""
import numpy as np
import pytest
import torch

from gpu_common import compare_density, dev, upload
from synth import drift_set

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_1804_06231_amd as pvl
    c = pvl.Context(0)
    yield c
    c.close()


def _oracle(s, x):
    from oracle import Oracle
    return Oracle(np.mod(x, s.box[0]), s.h, s.m, s.box)


def test_drift_reuses_sorted_lists(ctx):
    s = drift_set(20000, 71, 3, 4e-4)
    pos, h, m = upload(s)
    cells = ctx.build_cells(pos, h, m, s.box)
    ctx.sort_cells(cells)
    G = np.random.Generator(np.random.PCG64(72)).standard_normal(s.n).astype(np.float32)
    g = torch.from_numpy(G).to(dev())
    for k, d in enumerate(s.extra["disp"]):
        ctx.drift(cells, torch.from_numpy(d).to(dev()))
        o = _oracle(s, s.extra["positions"][k + 1])
        ref = o.density()
        for algo in ("sorted", "plain"):
            out = [t.cpu().numpy() for t in ctx.density(cells, algo)]
            ctx.check()
            compare_density(out, ref, label=f"step {k + 1} {algo}")
        gp, gh = ctx.density_backward(cells, g)
        ctx.check()
        gr = o.grad(G.astype(np.float64))
        ex = np.max(np.abs(gp.cpu().numpy() - gr["gx"]) / np.maximum(gr["gx_abs"], 1e-300))
        eh = np.max(np.abs(gh.cpu().numpy() - gr["gh"]) / np.maximum(gr["gh_abs"], 1e-300))
        assert ex < 1e-5 and eh < 1e-5, (k, ex, eh)
    import paper_1804_06231_amd as pvl
    with pytest.raises(pvl.PVError) as e:
        ctx.sort_cells(cells)                 # moved cells are rebuilt, not re-sorted
    assert e.value.status == pvl.PV_ESTATE


def test_drift_beyond_the_cell_room_is_reported(ctx):
    import paper_1804_06231_amd as pvl
    s = drift_set(20000, 73, 1, 4e-4)
    pos, h, m = upload(s)
    cells = ctx.build_cells(pos, h, m, s.box)
    ctx.sort_cells(cells)
    edge = 1.0 / cells.info()["grid"][0]
    room = edge - float(cells.info()["hmax"])
    big = np.zeros((s.n, 3), dtype=np.float32)
    big[:, 0] = 0.75 * room                  # every particle moves by 0.75 of the room
    ctx.drift(cells, torch.from_numpy(big).to(dev()))
    ctx.density(cells, "sorted")
    with pytest.raises(pvl.PVError) as e:
        ctx.check()
    assert e.value.status == pvl.PV_ESTATE
    # a rebuild from the moved positions is valid again
    moved = torch.from_numpy(np.mod(s.pos.astype(np.float64) + big, 1.0).astype(np.float32)).to(dev())
    cells = ctx.build_cells(moved, h, m, s.box)
    ctx.sort_cells(cells)
    ctx.density(cells, "sorted")
    ctx.check()
