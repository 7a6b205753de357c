"""GPU h-iteration (pv_solve_h) against the fp64 oracle's per-particle
bisection of rho_i(h_i) h_i^3 = m_i eta^3, through the C ABI."""
import numpy as np
import pytest
import torch

from gpu_common import dev
from synth import uniform_set, plummer_set, h_for_neighbours

pytestmark = pytest.mark.gpu

TOL_H = 1e-5     # relative, on h (fp32 density, residual target 1e-6)


@pytest.fixture(scope="module")
def ctx():
    import paper_1804_06231_amd as pvl
    c = pvl.Context(0)
    yield c
    c.close()


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dev())


def _oracle_h(s, h0, up=2.5):
    from oracle import solve_h_fp64, eta_for_neighbours
    # bracket wide enough for the densest cores (contrast ~80: h / 4.3) and the
    # emptiest background; independent of the GPU result
    return solve_h_fp64(s.pos, s.m, h0 / 8.0, up * h0, eta_for_neighbours(48.0), s.box)


@pytest.mark.parametrize("kind", ["clustered", "lognormal"])
def test_solve_h_matches_oracle(ctx, kind):
    if kind == "clustered":
        s = plummer_set(8192, 91, n_spheres=64)
    else:
        s = uniform_set(20000, 92, hmode="lognormal")
    h0 = h_for_neighbours(s.n)
    h = _t(np.full(s.n, h0))                  # constant start, far from the solution
    it, res = ctx.solve_h(_t(s.pos), _t(s.m), h, s.box, ngb=48.0, tol=1e-6, max_iter=40)
    print(f"{kind}: {it} iterations, residual {res:.2e}", flush=True)
    assert res <= 1e-6 and it < 40
    hg = h.cpu().numpy().astype(np.float64)
    ho = _oracle_h(s, h0)
    err = np.max(np.abs(hg - ho) / ho)
    print(f"{kind}: max rel err of h {err:.2e}", flush=True)
    assert err < TOL_H


def test_solve_h_batched_boxes(ctx):
    sets = [uniform_set(6000, 93, hmode="jitter"), plummer_set(5000, 94, n_spheres=64),
            uniform_set(3000, 95, hmode="lognormal", L=0.5)]
    off = np.zeros(len(sets) + 1, dtype=np.int64)
    off[1:] = np.cumsum([s.n for s in sets])
    h0 = [h_for_neighbours(s.n, L=s.box[0]) for s in sets]
    pos = _t(np.concatenate([s.pos for s in sets]))
    m = _t(np.concatenate([s.m for s in sets]))
    h = _t(np.concatenate([np.full(s.n, h0[k]) for k, s in enumerate(sets)]))
    it, res = ctx.solve_h(pos, m, h, offsets=list(off), boxes=[s.box for s in sets],
                          tol=1e-6, max_iter=40)
    assert res <= 1e-6
    hg = h.cpu().numpy().astype(np.float64)
    for k, s in enumerate(sets):
        ho = _oracle_h(s, h0[k], up=2.0)
        err = np.max(np.abs(hg[off[k]:off[k + 1]] - ho) / ho)
        assert err < TOL_H, (k, err)


def test_solve_h_reports_grid_errors(ctx):
    import paper_1804_06231_amd as pvl
    s = uniform_set(100, 96, hmode="const", guard=False)   # H(48 ngb) > 1/3 of the box
    h = _t(np.full(s.n, h_for_neighbours(s.n)))
    with pytest.raises(pvl.PVError) as e:
        ctx.solve_h(_t(s.pos), _t(s.m), h, s.box)
    assert e.value.status == pvl.PV_EGRID
    # an iteration budget that is too small leaves the residual above tol
    s = plummer_set(4096, 97, n_spheres=64)
    h = _t(np.full(s.n, h_for_neighbours(s.n)))
    it, res = ctx.solve_h(_t(s.pos), _t(s.m), h, s.box, tol=1e-7, max_iter=2)
    assert it == 2 and res > 1e-7
