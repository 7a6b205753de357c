"""Full-size GPU parity, in the launch configuration the bench times.

The oracle computes sampled receivers one by one (fp64 cell list); properties
that hold at any size (sorted == plain counts, translation invariance of the
adjoint) are checked on every particle.
  * uniform-1m-lognormal: 2^20 uniform particles, lognormal h (sigma 0.2)
  * clustered-4m: 2^22 particles, half uniform, half in 64 Plummer spheres,
    h solved for 48 neighbours, cell occupancy from a few to ~3000
  * adjoint-1m: 2^20 uniform particles, h jittered +-20%, loss against the
    density of a perturbed copy; gradients checked against fp64 central
    differences on 1000 sampled particles
  * batched-256: 256 boxes of 4096..262144 particles, half uniform (lognormal
    h), half clustered (kNN h), each on its finest grid, one launch per stage
"""
import numpy as np
import pytest
import torch

from gpu_common import compare_density, oracle_for, run_density, upload, dev
from synth import workload, GAMMA

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_1804_06231_amd as pvl
    c = pvl.Context(0)
    yield c
    c.close()


def _sample(n, k, seed):
    return np.sort(np.random.Generator(np.random.PCG64(seed)).choice(n, k, replace=False))


def test_uniform_1m_lognormal(ctx):
    print("uniform-1m-lognormal: generating", flush=True)
    s = workload("uniform-1m-lognormal")
    cells, srt = run_density(ctx, s, "sorted")
    _, pln = run_density(ctx, s, "plain", cells=cells)
    assert np.array_equal(srt[3], pln[3])
    assert np.max(np.abs(srt[0] - pln[0]) / pln[0]) < 2e-5
    o = oracle_for(s)
    idx = _sample(s.n, 20000, 1)
    # add the extremes of the lognormal tail (largest and smallest h)
    order = np.argsort(s.h)
    idx = np.unique(np.concatenate([idx, order[:200], order[-200:]]))
    e = compare_density(srt, o.density(idx), idx, "uniform-1m sorted")
    print("uniform-1m-lognormal max rel err rho/wcount/dh:", e, flush=True)


def test_clustered_4m(ctx):
    print("clustered-4m: generating", flush=True)
    s = workload("clustered-4m")
    cells, srt = run_density(ctx, s, "sorted")
    info = cells.info()
    assert info["max_occupancy"] > 1024          # the chunked work items are exercised
    _, pln = run_density(ctx, s, "plain", cells=cells)
    assert np.array_equal(srt[3], pln[3])
    assert np.all(srt[3] >= 46) and np.all(srt[3] <= 50)   # h solved for 48 neighbours
    o = oracle_for(s)
    # random receivers plus those of the most crowded cells
    g = info["grid"][0]
    c = np.floor(s.pos.astype(np.float64) * g).astype(np.int64)
    cid = (c[:, 0] * g + c[:, 1]) * g + c[:, 2]
    occ = np.bincount(cid, minlength=g ** 3)
    dense = np.nonzero(occ[cid] >= np.sort(occ)[-5])[0]
    idx = np.unique(np.concatenate([_sample(s.n, 8000, 2), dense[:: max(1, dense.size // 3000)]]))
    e = compare_density(srt, o.density(idx), idx, "clustered-4m sorted")
    print("clustered-4m max rel err rho/wcount/dh:", e, flush=True)


def test_adjoint_1m_against_fd(ctx):
    from oracle import Oracle
    print("adjoint-1m: generating", flush=True)
    s = workload("adjoint-1m")
    o = oracle_for(s)
    t = Oracle(s.extra["pos_target"], s.h, s.m, s.box).density()["rho"]
    pos, h, m = upload(s)
    pos.requires_grad_(True)
    h.requires_grad_(True)
    import paper_1804_06231_amd as pvl
    rho, _, _, _ = pvl.density(pos, m, h)
    tt = torch.from_numpy(t.astype(np.float32)).to(dev())
    loss = ((rho - tt) ** 2).sum()
    loss.backward()
    torch.cuda.synchronize()
    gp = pos.grad.cpu().numpy().astype(np.float64)
    gh = h.grad.cpu().numpy().astype(np.float64)
    # the upstream gradient exactly as the GPU formed it (fp32), and in fp64
    G32 = (2.0 * (rho.detach() - tt)).cpu().numpy().astype(np.float64)
    rho64 = o.density()["rho"]
    G64 = 2.0 * (rho64 - t)
    ks = _sample(s.n, 1000, 3)
    ref32 = o.grad(G32, ks)
    ref64 = o.grad(G64, ks)
    # parity with the oracle's adjoint for the same upstream gradient
    ex = np.max(np.abs(gp[ks] - ref32["gx"]) / ref32["gx_abs"])
    eh = np.max(np.abs(gh[ks] - ref32["gh"]) / ref32["gh_abs"])
    assert ex < 1e-5 and eh < 1e-5, (ex, eh)
    # fp64 central finite differences of L = sum (rho - t)^2 itself
    kk = np.repeat(ks, 4)
    comps = np.tile(np.arange(4), ks.size)
    row = np.repeat(np.arange(ks.size), 4)
    Hk = GAMMA * s.h[kk].astype(np.float64)
    eps = np.where(comps < 3, 1e-4 * Hk, 1e-4 * s.h[kk])
    # Richardson-extrapolated central differences; |fd(e) - fd(e/2)| bounds the
    # truncation left (the loss is quadratic, so where rho ~ t its curvature
    # term dominates the small gradient)
    fd1 = o.fd_loss(t, kk, comps, eps)
    fd2 = o.fd_loss(t, kk, comps, eps / 2)
    fd = (4.0 * fd2 - fd1) / 3.0
    trunc = 0.1 * np.abs(fd1 - fd2)
    pick = lambda r: np.where(comps < 3, r["gx"][row, np.minimum(comps, 2)], r["gh"][row])
    scale = np.where(comps < 3, ref64["gx_abs"][row, np.minimum(comps, 2)], ref64["gh_abs"][row])
    # the oracle's own adjoint agrees with its differences ...
    assert np.max(np.abs(pick(ref64) - fd) / (1e-6 * scale + trunc)) < 1.0
    # ... and the GPU's, up to 1e-5 plus what rounding G to fp32 changes
    gpu = np.where(comps < 3, gp[kk, np.minimum(comps, 2)], gh[kk])
    allow = 1e-5 * scale + np.abs(pick(ref64) - pick(ref32)) + trunc
    efd = np.max(np.abs(gpu - fd) / allow)
    print(f"adjoint-1m: parity err x {ex:.2e} h {eh:.2e}; FD err / allowance {efd:.2f}", flush=True)
    assert efd < 1.0
    # translation invariance over all particles
    tot = np.abs(gp.sum(0))
    assert np.all(tot < 1e-4 * np.abs(gp).sum(0))


def test_batched_256(ctx):
    """256 boxes of 4096..262144 particles (~15.4M), uniform and clustered, each
    on its finest grid, through one launch per stage; 24 sampled receivers per
    box against the oracle of that box, for the density and the adjoint."""
    from synth import workload
    print("batched-256: generating", flush=True)
    b = workload("batched-256", progress=lambda m: print("batched-256:", m, flush=True))
    d = dev()
    pos, h, m = (torch.from_numpy(x).to(d) for x in (b.pos, b.h, b.m))
    off = [int(x) for x in b.offsets]
    print("batched-256: running", flush=True)
    cells = ctx.build_cells_batched(off, pos, h, m, b.boxes, b.grids)
    ctx.sort_cells(cells)
    out = ctx.density(cells, "sorted")
    G = np.random.Generator(np.random.PCG64(6)).standard_normal(b.n).astype(np.float32)
    gp, gh = ctx.density_backward(cells, torch.from_numpy(G).to(d))
    ctx.check()
    torch.cuda.synchronize()
    out = [t.cpu().numpy() for t in out]
    gp, gh = gp.cpu().numpy(), gh.cpu().numpy()
    assert cells.info()["ncell"] == sum(g ** 3 for g in b.grids)
    rng = np.random.Generator(np.random.PCG64(7))
    worst = np.zeros(5)
    for k, s in enumerate(b.sets):
        sl = slice(off[k], off[k + 1])
        idx = np.sort(rng.choice(s.n, 24, replace=False))
        o = oracle_for(s, b.grids[k])
        e = compare_density([a[sl] for a in out], o.density(idx), idx, f"batched box {k}")
        ref = o.grad(G[sl].astype(np.float64), idx)
        ex = np.max(np.abs(gp[sl][idx] - ref["gx"]) / np.maximum(ref["gx_abs"], 1e-300))
        eh = np.max(np.abs(gh[sl][idx] - ref["gh"]) / np.maximum(ref["gh_abs"], 1e-300))
        assert ex < 1e-5 and eh < 1e-5, (k, ex, eh)
        worst = np.maximum(worst, [*e, ex, eh])
    print("batched-256 max rel err rho/wcount/dh/gx/gh:", worst, flush=True)
