"""Shared helpers of the GPU parity tests: upload a particle set, run the HIP
path through the C ABI, compare with the fp64 oracle."""
import numpy as np
import torch

from oracle import Oracle

RTOL = 1e-5   # relative tolerance for rho, wcount; drho_dh and gradients use
              # 1e-5 of the sum of absolute terms (signed sums cancel)


def dev():
    return torch.device("cuda", 0)


def upload(s):
    d = dev()
    return (torch.from_numpy(np.ascontiguousarray(s.pos)).to(d),
            torch.from_numpy(np.ascontiguousarray(s.h)).to(d),
            torch.from_numpy(np.ascontiguousarray(s.m)).to(d))


def run_density(ctx, s, algo="sorted", grid=None, cells=None):
    pos, h, m = upload(s)
    cells = ctx.build_cells(pos, h, m, s.box, grid, cells)
    if algo == "sorted":
        ctx.sort_cells(cells)
    out = ctx.density(cells, algo)
    ctx.check()
    torch.cuda.synchronize()
    return cells, [t.cpu().numpy() for t in out]


def compare_density(gpu, ref, idx=None, label=""):
    """gpu = [rho, wcount, drho_dh, ncount] (full arrays); ref = oracle dict for
    receivers idx (all when None).  Returns the worst relative errors."""
    rho, wc, dh, nc = gpu
    if idx is not None:
        rho, wc, dh, nc = rho[idx], wc[idx], dh[idx], nc[idx]
    bad = np.nonzero(nc != ref["ncount"])[0]
    assert bad.size == 0, f"{label}: {bad.size} neighbour counts differ, e.g. receiver " \
                          f"{bad[:5]} gpu {nc[bad[:5]]} ref {ref['ncount'][bad[:5]]}"
    e_rho = np.max(np.abs(rho - ref["rho"]) / ref["rho"]) if rho.size else 0.0
    e_wc = np.max(np.abs(wc - ref["wcount"]) / ref["wcount"]) if wc.size else 0.0
    e_dh = np.max(np.abs(dh - ref["drho_dh"]) / ref["dh_abs"]) if dh.size else 0.0
    assert e_rho < RTOL, f"{label}: rho rel err {e_rho}"
    assert e_wc < RTOL, f"{label}: wcount rel err {e_wc}"
    assert e_dh < RTOL, f"{label}: drho_dh err {e_dh} (of sum |terms|)"
    return e_rho, e_wc, e_dh


def oracle_for(s, grid=None):
    return Oracle(s.pos, s.h, s.m, s.box, grid)
