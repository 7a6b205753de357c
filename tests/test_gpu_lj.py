"""Second workload through the same sweep: Lennard-Jones forces and energies
(pv_lj) against the fp64 oracle, through the C ABI."""
import numpy as np
import pytest
import torch

from gpu_common import dev, upload, oracle_for
from synth import lj_set

pytestmark = pytest.mark.gpu

TOL = 1e-5   # of the sum of the terms' magnitudes (signed sums)


@pytest.fixture(scope="module")
def ctx():
    import paper_1804_06231_amd as pvl
    c = pvl.Context(0)
    yield c
    c.close()


def _check(f, e, ref, idx=None, label=""):
    if idx is not None:
        f, e = f[idx], e[idx]
    ef = np.max(np.abs(f - ref["force"]) / np.maximum(ref["f_abs"], 1e-300))
    ee = np.max(np.abs(e - ref["energy"]) / np.maximum(ref["e_abs"], 1e-300))
    assert ef < TOL and ee < TOL, (label, ef, ee)
    return ef, ee


@pytest.mark.parametrize("M,rc", [(24, 2.5), (32, 2.2)])
def test_lj_matches_oracle(ctx, M, rc):
    s = lj_set(M, 50 + M, jitter=0.2, rc_over_a=rc)
    sigma, eps = s.extra["sigma"], 1.3
    pos, h, m = upload(s)
    cells = ctx.build_cells(pos, h, m, s.box)
    ctx.sort_cells(cells)
    f, e = ctx.lj(cells, eps, sigma)
    ctx.check()
    f, e = f.cpu().numpy().astype(np.float64), e.cpu().numpy().astype(np.float64)
    ref = oracle_for(s).lj(eps, sigma)
    print(f"lj M={M}: max err force/energy", _check(f, e, ref, label=f"M={M}"), flush=True)
    assert np.all(np.abs(f.sum(0)) < 1e-5 * np.abs(f).sum(0))      # third law


def test_lj_1m_sampled(ctx):
    """10^6 particles (100^3 jittered lattice, r_c = 2.5 a): 2000 sampled
    receivers against the oracle, third law over all."""
    s = lj_set(100, 77, jitter=0.2, rc_over_a=2.5)
    sigma, eps = s.extra["sigma"], 1.0
    pos, h, m = upload(s)
    cells = ctx.build_cells(pos, h, m, s.box)
    ctx.sort_cells(cells)
    f, e = ctx.lj(cells, eps, sigma)
    ctx.check()
    f, e = f.cpu().numpy().astype(np.float64), e.cpu().numpy().astype(np.float64)
    idx = np.sort(np.random.Generator(np.random.PCG64(78)).choice(s.n, 2000, replace=False))
    ref = oracle_for(s).lj(eps, sigma, idx)
    print("lj-1m: max err force/energy", _check(f, e, ref, idx, "lj-1m"), flush=True)
    assert np.all(np.abs(f.sum(0)) < 1e-5 * np.abs(f).sum(0))


def test_grid_autotune(ctx):
    """The grid autotuner returns a legal grid no finer than the finest, at least
    as fast, and the results on it still match the oracle (any legal grid gives
    the same pairs)."""
    s = lj_set(40, 79, jitter=0.2, rc_over_a=2.5)
    pos, h, m = upload(s)
    (g,), t_finest, t_best = ctx.autotune_grid(pos, h, m, s.box, reps=2)
    finest = int(1.0 / (float(h[0]) * 1.825742 * (1 + 4e-6)))
    print(f"grid autotune: finest {finest}^3 {t_finest:.3f} ms -> {g} {t_best:.3f} ms", flush=True)
    assert 3 <= g[0] <= finest and t_best <= t_finest
    cells = ctx.build_cells(pos, h, m, s.box, g)
    ctx.sort_cells(cells)
    f, e = ctx.lj(cells, 1.0, s.extra["sigma"])
    ctx.check()
    ref = oracle_for(s).lj(1.0, s.extra["sigma"])
    _check(f.cpu().numpy().astype(np.float64), e.cpu().numpy().astype(np.float64), ref,
           label="tuned grid")
