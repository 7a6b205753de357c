"""GPU parity of the density adjoint (dL/dx, dL/dh) against the fp64 oracle's
analytic adjoint and fp64 finite differences, through the C ABI and through
torch.autograd."""
import numpy as np
import pytest
import torch

from gpu_common import dev, upload, oracle_for
from synth import uniform_set, plummer_set, adjoint_set

pytestmark = pytest.mark.gpu

TOL = 1e-5   # of the sum of absolute terms per component


@pytest.fixture(scope="module")
def ctx():
    import paper_1804_06231_amd as pvl
    c = pvl.Context(0)
    yield c
    c.close()


def _gpu_grad(ctx, s, G):
    pos, h, m = upload(s)
    cells = ctx.build_cells(pos, h, m, s.box)
    ctx.sort_cells(cells)
    g = torch.from_numpy(G.astype(np.float32)).to(dev())
    gp, gh = ctx.density_backward(cells, g)
    ctx.check()
    torch.cuda.synchronize()
    return gp.cpu().numpy(), gh.cpu().numpy()


def _check(gp, gh, ref, idx=None, label=""):
    if idx is not None:
        gp, gh = gp[idx], gh[idx]
    ex = np.max(np.abs(gp - ref["gx"]) / np.maximum(ref["gx_abs"], 1e-300))
    eh = np.max(np.abs(gh - ref["gh"]) / np.maximum(ref["gh_abs"], 1e-300))
    assert ex < TOL, f"{label}: dL/dx err {ex}"
    assert eh < TOL, f"{label}: dL/dh err {eh}"
    return ex, eh


@pytest.mark.parametrize("hmode", ["jitter", "lognormal"])
def test_adjoint_uniform_small(ctx, hmode):
    s = uniform_set(12000, 3, hmode=hmode)
    o = oracle_for(s)
    rho = o.density()["rho"]
    rng = np.random.Generator(np.random.PCG64(4))
    t = rho * (1 + 0.05 * rng.standard_normal(s.n))
    G = (2 * (rho - t)).astype(np.float32)
    gp, gh = _gpu_grad(ctx, s, G)
    ref = o.grad(G.astype(np.float64))
    _check(gp, gh, ref, label=hmode)
    # translation invariance: the position gradients sum to zero
    tot = np.abs(gp.astype(np.float64).sum(0))
    assert np.all(tot < 1e-5 * ref["gx_abs"].sum(0))


def test_adjoint_clustered(ctx):
    s = plummer_set(40000, 5, n_spheres=16)
    o = oracle_for(s)
    rng = np.random.Generator(np.random.PCG64(6))
    G = rng.standard_normal(s.n).astype(np.float32)
    gp, gh = _gpu_grad(ctx, s, G)
    _check(gp, gh, o.grad(G.astype(np.float64)), label="clustered")


def test_autograd_matches_abi(ctx):
    import paper_1804_06231_amd as pvl
    s = uniform_set(8000, 9, hmode="jitter")
    pos, h, m = upload(s)
    pos.requires_grad_(True)
    h.requires_grad_(True)
    rho, wc, dh, nc = pvl.density(pos, m, h)
    t = torch.from_numpy(oracle_for(s).density()["rho"].astype(np.float32) * 1.01).to(dev())
    loss = ((rho - t) ** 2).sum()
    loss.backward()
    G = (2 * (rho.detach() - t)).cpu().numpy()
    gp, gh = _gpu_grad(ctx, s, G)
    assert np.array_equal(pos.grad.cpu().numpy(), gp)
    assert np.array_equal(h.grad.cpu().numpy(), gh)
    assert not wc.requires_grad and not nc.requires_grad
    # dL/dh = G drho_dh with the forward drho_dh (summed in another order)
    ref = oracle_for(s).density()
    assert np.all(np.abs(h.grad.cpu().numpy() - G * dh.detach().cpu().numpy())
                  <= 2e-5 * np.abs(G) * ref["dh_abs"])


def test_adjoint_against_finite_differences(ctx):
    """fp32 GPU gradient of L = sum (rho - t)^2 against fp64 central
    differences of the oracle's L on sampled particles and coordinates; the
    allowance adds what rounding the upstream gradient to fp32 changes."""
    s = adjoint_set(20000, 8)
    o = oracle_for(s)
    from oracle import Oracle
    t = Oracle(s.extra["pos_target"], s.h, s.m, s.box).density()["rho"]
    rho = o.density()["rho"]
    G64 = 2 * (rho - t)
    G32 = G64.astype(np.float32)
    gp, gh = _gpu_grad(ctx, s, G32)
    rng = np.random.Generator(np.random.PCG64(10))
    ks = np.sort(rng.choice(s.n, 200, replace=False))
    kk = np.repeat(ks, 4)
    comps = np.tile(np.arange(4), ks.size)
    row = np.repeat(np.arange(ks.size), 4)
    H = 1.825742 * s.h[kk].astype(np.float64)
    eps = np.where(comps < 3, 1e-4 * H, 1e-4 * s.h[kk])
    # Richardson-extrapolated central differences; |fd(e) - fd(e/2)| bounds the
    # truncation left (the loss is quadratic, so where rho ~ t its curvature
    # term dominates the small gradient)
    fd1 = o.fd_loss(t, kk, comps, eps)
    fd2 = o.fd_loss(t, kk, comps, eps / 2)
    fd = (4.0 * fd2 - fd1) / 3.0
    trunc = 0.1 * np.abs(fd1 - fd2)
    r32 = o.grad(G32.astype(np.float64), ks)
    r64 = o.grad(G64, ks)
    pick = lambda r: np.where(comps < 3, r["gx"][row, np.minimum(comps, 2)], r["gh"][row])
    scale = np.where(comps < 3, r64["gx_abs"][row, np.minimum(comps, 2)], r64["gh_abs"][row])
    gpu = np.where(comps < 3, gp[kk, np.minimum(comps, 2)], gh[kk])
    _check(gp, gh, r32, ks, label="fd-set")
    allow = 1e-5 * scale + np.abs(pick(r64) - pick(r32)) + trunc
    err = np.abs(gpu - fd) / allow
    assert np.max(err) < 1.0, f"max FD err / allowance {np.max(err)}"


def test_adjoint_with_coincident_particles(ctx):
    """Distinct particles at one position: each is the other's neighbour at
    r = 0, so it adds 3 w(0) m_j to drho_dh (and dL/dh = G drho_dh) but nothing
    to dL/dx.  Copies take the original's h as well, so every pair keeps the
    generator's distance from the cut-offs."""
    from gpu_common import compare_density, run_density
    s = uniform_set(6000, 12, hmode="jitter")
    rng = np.random.Generator(np.random.PCG64(13))
    src = rng.choice(s.n // 2, 8, replace=False)
    dst = s.n // 2 + src
    s.pos[dst] = s.pos[src]
    s.h[dst] = s.h[src]
    o = oracle_for(s)
    ref = o.density()
    assert np.all(ref["ncount"][dst] >= 1)
    _, got = run_density(ctx, s)
    compare_density(got, ref, label="coincident density")
    G = rng.standard_normal(s.n).astype(np.float32)
    gp, gh = _gpu_grad(ctx, s, G)
    _check(gp, gh, o.grad(G.astype(np.float64)), label="coincident adjoint")
