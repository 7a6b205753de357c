"""pv_density_static, the entry point that allocates nothing: its output
equals that of pv_build_cells (same grid) + pv_sort_cells + pv_density on the
same inputs, on two calls in a row (the second smaller), through the C ABI.
The fp64 oracle checks the first call as well."""
import numpy as np
import pytest
import torch

import paper_1804_06231_amd as pvl
from synth import uniform_set
from tests.gpu_common import RTOL, compare_density, oracle_for, upload

pytestmark = pytest.mark.gpu


def _finest(s):
    hmax = float(np.max(s.h)) * 1.825742
    return int(np.floor(1.0 / (hmax * (1 + 4e-6))))


def _existing(ctx, pos, h, m, box, grid, algo):
    cells = ctx.build_cells(pos, h, m, box, grid)
    if algo == "sorted":
        ctx.sort_cells(cells)
    out = ctx.density(cells, algo)
    ctx.check()
    torch.cuda.synchronize()
    res = [t.cpu().numpy() for t in out]
    cells.free()
    return res


def _same(a, b, label):
    rho, wc, dh, nc = a
    rho2, wc2, dh2, nc2 = b
    assert np.array_equal(nc, nc2), f"{label}: neighbour counts differ"
    assert np.max(np.abs(rho - rho2) / rho2) < RTOL, f"{label}: rho"
    assert np.max(np.abs(wc - wc2) / wc2) < RTOL, f"{label}: wcount"
    # drho_dh is a signed sum: compared at RTOL of its scale (3 rho / h bounds
    # the self and neighbour terms' magnitudes)
    assert np.max(np.abs(dh - dh2)) <= RTOL * np.max(np.abs(dh2)) + 1e-30, f"{label}: drho_dh"


@pytest.mark.parametrize("algo", ["sorted", "plain"])
def test_static_entry_point_equals_allocating_path(algo):
    ctx = pvl.Context(0)
    sets = [uniform_set(40000, 31, hmode="lognormal"), uniform_set(9000, 32, hmode="lognormal")]
    for k, s in enumerate(sets):
        g = _finest(s)
        grid = (g, g, g)
        pos, h, m = upload(s)
        print(f"[no-alloc] {algo} call {k}: n={s.n} grid={grid}", flush=True)
        out = ctx.density_static(pos, h, m, s.box, grid, algo)
        ctx.check()
        torch.cuda.synchronize()
        got = [t.cpu().numpy() for t in out]
        ref = _existing(ctx, pos, h, m, s.box, grid, algo)
        _same(got, ref, f"{algo} call {k} (n={s.n})")
        if k == 0:
            o = oracle_for(s, grid).density()
            compare_density(got, o, label=f"{algo} call {k} vs oracle")
    ctx.close()


def test_static_entry_point_limits_and_empty_input():
    ctx = pvl.Context(0)
    d = torch.device("cuda", 0)
    e = torch.empty((0, 3), device=d)
    z = torch.empty(0, device=d)
    rho, wc, dh, nc = ctx.density_static(e, z, z, (1.0, 1.0, 1.0), (4, 4, 4))
    ctx.check()
    assert rho.numel() == 0 and nc.numel() == 0
    big = torch.zeros((pvl.PV_STATIC_MAX_N + 1, 3), device=d)
    hb = torch.full((pvl.PV_STATIC_MAX_N + 1,), 0.01, device=d)
    with pytest.raises(pvl.PVError, match="static scratch"):
        ctx.density_static(big, hb, hb, (1.0, 1.0, 1.0), (8, 8, 8))
    with pytest.raises(pvl.PVError):
        ctx.density_static(big[:10], hb[:10], hb[:10], (1.0, 1.0, 1.0), (64, 64, 64))
    ctx.close()
