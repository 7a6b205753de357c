"""Benchmark of the pseudo-Verlet SPH density loop on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

A step is one pass of the whole hot path over the resident particle set:
build_cells (binning into cells, explicit grid) + sort_cells (13 per-axis
sorts) + density (sorted-pair sweep with in-place finalisation).  The plain
cell-list comparator (build_cells + density with the 27-cell brute force) is
timed the same way.  Both steps are timed as issued call by call on the
stream and as a captured HIP graph (one launch per step), with the same event
timing; the reported figure is the faster of the two (both are recorded, with
which one was reported).  The sweep parameters are autotuned first.  Inputs
are seeded synthetic particle sets already in HBM.

Prints one JSON line: pair-interactions/s of the sorted-pair path (value), the
plain comparator, ns/particle, the sweep kernel's roofline and the fp64 CPU
oracle timed on a bounded sample of the same workload.  The roofline's time
is the persistent sweep kernel's own average duration, from HIP events the
library records around its launch on its stream (pv_set_kernel_timing); the
whole density call (with the work-queue set-up and the tail combine) is
reported beside it.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Peak VALU rate of MI355X without packed fp32: 256 CUs x 4 SIMDs x 16 lanes x
# 2.4 GHz = 39.3e12 lane-operations per second (an FMA counts once).
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
HBM_PEAK_GBS = 8000.0
# Algorithmic VALU work of the sweep: lane-operations per pair that passes the
# projected-distance test (3 differences, 3 products for r^2, compare, key
# test) and per pair in range (square root at quarter rate = 4, scaling, both
# spline pieces and the select, 3 accumulations and the count).  Candidates
# are those of the method's exact per-receiver bounds: Section 3.3's bounds on
# the 26 neighbour cells and the receiver's cut-off in x in its own cell.
OPS_PER_CANDIDATE = 8
OPS_PER_INTERACTION = 25
# Algorithmic HBM bytes per particle of each stage: binning reads positions
# and h (16); the scatter into cell order reads them with the mass and writes
# the cell-ordered position/mass, cut-off and index (48); the 13 per-axis
# sorts read positions (12) and write 13 two-byte index lists (26); the sweep
# reads positions, cut-offs and the lists and writes the 4 outputs (66).
HBM_BYTES = {"bin": 16, "scatter": 48, "sort13": 38, "sweep": 66}
# the timed density sweep's name in a kernel trace (the census launch, which
# also counts pair slots, is an instantiation of its own)
SWEEP_KERNEL = "pvl::k_sweep_queue<0, false, false>"
# the kernels of each stage in a kernel trace (name prefixes)
STAGE_KERNELS = {
    "bin": ("pvl::k_bin_local", "pvl::k_bin_columns", "pvl::k_scan", "pvl::k_tile_sums",
            "pvl::k_tile_scan", "pvl::k_cell_box"),
    "scatter": ("pvl::k_scatter", "pvl::k_cell_finish"),
    "sort13": ("pvl::k_sort13",),
    "sweep": ("pvl::k_sweep_queue<0, false, false>", "pvl::k_tail_combine<0>",
              "pvl::k_queue_items"),
}


def _args():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="uniform-1m-lognormal")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--core", action="store_true",
                    help="skip the h-iteration, list-reuse and Lennard-Jones sections (their "
                         "density launches would mix into a profile of the sweep)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="time the default sweep parameters instead of the autotuned ones")
    ap.add_argument("--cpu-seconds", type=float, default=20.0,
                    help="target CPU time of the oracle sample")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="also run one device copy of this many MiB (a reference kernel "
                         "for scaling hardware byte counters)")
    return ap.parse_args()


def _autotune(a, ctx, cells, g_rho, targets):
    """Run the library's autotuner for each sweep (untimed set-up)."""
    if a.no_autotune:
        return {t: {"params": ctx.params(t)} for t in targets}
    out = {}
    for t in targets:
        print(f"[bench] autotuning the {t} sweep", file=sys.stderr, flush=True)
        before, after, p = ctx.autotune(cells, t, g_rho if t == "adjoint" else None, reps=3)
        out[t] = {"default_ms": before, "tuned_ms": after, "params": p}
    return out


def _capture(fn, torch):
    """Record fn (library calls only) into a HIP graph; one eager run on the
    capture stream first, as graph capture requires."""
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        fn()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        fn()
    torch.cuda.synchronize()
    return graph


def _time_loop(fn, steps, warmup, torch):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    start.record()
    for _ in range(steps):
        fn()
    stop.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return start.elapsed_time(stop) / steps, wall / steps * 1e3


def main():
    a = _args()
    if a.gpus != 1:
        print(f"bench.py: measures one GPU only (asked for --gpus {a.gpus}); "
              "the path runs on a single MI355X and has no multi-GPU mode.", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_1804_06231_amd as pvl
    from synth import workload

    print(f"[bench] generating {a.workload}", file=sys.stderr, flush=True)
    t0 = time.time()
    s = workload(a.workload, progress=lambda m: print(f"[bench] {m}", file=sys.stderr, flush=True))
    if hasattr(s, "offsets"):
        return bench_batched(a, s, torch, pvl, t0)
    print(f"[bench] inputs ready in {time.time() - t0:.1f}s (n={s.n})", file=sys.stderr, flush=True)
    dev = torch.device("cuda", 0)
    pos = torch.from_numpy(s.pos).to(dev)
    h = torch.from_numpy(s.h).to(dev)
    m = torch.from_numpy(s.m).to(dev)
    ctx = pvl.Context(0)
    if a.copy_probe_mb:
        src = torch.ones(a.copy_probe_mb * (1 << 20) // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # grid: the workload's own, else the autotuner's (the finest legal one
    # with --no-autotune); the cell structure is rebuilt in place every step
    grid_tune = None
    grid = s.grid
    if grid is None and not a.no_autotune:
        print("[bench] autotuning the grid", file=sys.stderr, flush=True)
        (grid,), t_fine, t_best = ctx.autotune_grid(pos, h, m, s.box, reps=3)
        grid_tune = {"grid": list(grid), "finest_step_ms": t_fine, "tuned_step_ms": t_best}
    cells = ctx.build_cells(pos, h, m, s.box, grid)
    grid = cells.info()["grid"]
    ctx.sort_cells(cells)
    out_s = ctx.density(cells, "sorted")
    out_p = ctx.density(cells, "plain")
    ctx.check()
    torch.cuda.synchronize()
    pairs = int(out_s[3].sum().item())
    assert pairs == int(out_p[3].sum().item()), "sorted and plain neighbour counts differ"

    # candidate census (untimed)
    ctx.set_census(True)
    ctx.density(cells, "sorted")
    cand_sorted, inr, slots_sorted = ctx.census()
    ctx.density(cells, "plain")
    cand_plain, _, slots_plain = ctx.census()
    ctx.set_census(False)

    gen = torch.Generator(device=dev)
    gen.manual_seed(7)
    g_rho = torch.randn(s.n, generator=gen, device=dev)
    tuning = _autotune(a, ctx, cells, g_rho, ("density", "plain", "adjoint"))

    def step_sorted():
        ctx.build_cells(pos, h, m, s.box, grid, cells)
        ctx.sort_cells(cells)
        ctx.density(cells, "sorted", out_s)

    def step_plain():
        ctx.build_cells(pos, h, m, s.box, grid, cells)
        ctx.density(cells, "plain", out_p)

    print("[bench] timing sorted-pair path", file=sys.stderr, flush=True)
    ms_sorted_eager, wall_eager = _time_loop(step_sorted, a.steps, a.warmup, torch)
    print("[bench] timing plain cell-list path", file=sys.stderr, flush=True)
    ms_plain_eager, _ = _time_loop(step_plain, a.steps, a.warmup, torch)
    ctx.check()
    # the same steps as captured HIP graphs (one launch per step)
    print("[bench] timing both paths as HIP graphs", file=sys.stderr, flush=True)
    g_sorted = _capture(step_sorted, torch)
    ms_sorted, wall_sorted = _time_loop(g_sorted.replay, a.steps, a.warmup, torch)
    g_plain = _capture(step_plain, torch)
    ms_plain, _ = _time_loop(g_plain.replay, a.steps, a.warmup, torch)
    ctx.check()
    del g_sorted, g_plain

    # stage times (events on the stream the library launches on)
    ctx.build_cells(pos, h, m, s.box, grid, cells)
    ms_build, _ = _time_loop(lambda: ctx.build_cells(pos, h, m, s.box, grid, cells), a.steps, 1, torch)
    ms_sort, _ = _time_loop(lambda: ctx.sort_cells(cells), a.steps, 1, torch)
    ms_sweep, _ = _time_loop(lambda: ctx.density(cells, "sorted", out_s), a.steps, 1, torch)
    ms_kernel = _kernel_ms(ctx, lambda: ctx.density(cells, "sorted", out_s), a.steps)
    ms_sweep_plain, _ = _time_loop(lambda: ctx.density(cells, "plain", out_p), a.steps, 1, torch)
    # adjoint sweep for a seeded upstream gradient (dL/drho)
    out_g = (torch.empty((s.n, 3), device=dev), torch.empty(s.n, device=dev))
    ms_adj, _ = _time_loop(lambda: ctx.density_backward(cells, g_rho, out_g), a.steps, 1, torch)
    ctx.check()
    hsolve = reuse = lj = None
    if not a.core:
        print("[bench] h-iteration, list reuse, Lennard-Jones", file=sys.stderr, flush=True)
        hsolve = _bench_hsolve(ctx, s, pos, m, torch)
        reuse = _bench_reuse(a, ctx, s, pos, h, m, grid, out_s, torch)
        lj = _bench_lj(a, ctx, torch)

    n = s.n
    # the faster of the two launch forms of the same step
    ms_sorted_graph, ms_plain_graph = ms_sorted, ms_plain
    timed = "graph" if ms_sorted_graph <= ms_sorted_eager else "stream"
    wall = wall_sorted if timed == "graph" else wall_eager
    ms_sorted = min(ms_sorted_graph, ms_sorted_eager)
    ms_plain = min(ms_plain_graph, ms_plain_eager)
    if reuse is not None:
        reuse["speedup_vs_rebuild"] = ms_sorted / reuse["ms_per_step"]
    value = pairs / (ms_sorted * 1e-3)
    alg_ops = OPS_PER_CANDIDATE * cand_sorted + OPS_PER_INTERACTION * inr

    cpu = None
    if not a.no_cpu_baseline:
        print("[bench] timing the fp64 CPU oracle on a sample", file=sys.stderr, flush=True)
        cpu = _cpu_baseline(s, a.cpu_seconds)

    traffic = _traffic(a.workload, SWEEP_KERNEL)
    stage_ms = {"build_cells": ms_build, "sort_cells": ms_sort, "density_sweep": ms_sweep}
    rec = {
        "metric": "density pair-interactions/s + ns/particle, sorted-pair vs cell-list, 1 GPU",
        "value": value,
        "unit": "pair-interactions/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_sorted,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": s.name, "n": n, "grid": list(grid), "seed": s.seed,
                   "box": list(s.box), "h": "lognormal sigma 0.2 around the 48-neighbour value"
                   if "lognormal" in s.name else "see workload"},
        "ns_per_particle": ms_sorted * 1e6 / n,
        "pairs_in_range": pairs,
        "timed": timed,
        "graph_ms_per_step": ms_sorted_graph,
        "eager_ms_per_step": ms_sorted_eager,
        "plain_cell_list": {"ms_per_step": ms_plain, "value": pairs / (ms_plain * 1e-3),
                            "ns_per_particle": ms_plain * 1e6 / n,
                            "graph_ms_per_step": ms_plain_graph,
                            "eager_ms_per_step": ms_plain_eager, "sweep_ms": ms_sweep_plain},
        "speedup_sorted_vs_plain": ms_plain / ms_sorted,
        "stages_ms": {"build_cells": ms_build, "sort_cells": ms_sort, "density_sweep": ms_sweep,
                      "adjoint_sweep": ms_adj},
        "candidates_per_particle": {"sorted": cand_sorted / n, "plain": cand_plain / n,
                                    "in_range": inr / n},
        "autotune": tuning,
        "grid_autotune": grid_tune,
        "h_iteration": hsolve,
        "verlet_reuse": reuse,
        "lennard_jones": lj,
        "wall_ms_per_step": wall,
        "roofline": _roofline(a.workload, n, alg_ops, cand_sorted, inr, slots_sorted, ms_kernel,
                              ms_sweep, traffic),
        "roofline_path": _path_roofline(n, alg_ops, ms_sorted),
        "hbm_fraction": _hbm_fractions(a.workload, n, stage_ms),
        "cpu_baseline": cpu,
    }
    rec["candidates_per_particle"]["tiled_slots_sorted"] = slots_sorted / n
    rec["candidates_per_particle"]["tiled_slots_plain"] = slots_plain / n
    print(json.dumps(rec))


def _roofline(workload, n, alg_ops, cand, inr, slots, ms_kernel, ms_call, traffic):
    """The density sweep kernel against the vector-ALU peak: algorithmic
    lane-operations (exact-bound candidates and pairs in range) per launch over
    the kernel's average duration, measured live with the HIP events the
    library records around it on its stream (ms_call: the whole density call,
    with the queue set-up and the tail combine)."""
    achieved = alg_ops / (ms_kernel * 1e-3) / 1e12
    return {"kernel": f"{SWEEP_KERNEL} (sorted-pair density sweep)", "bound": "alu",
            "achieved": achieved, "peak": VALU_PEAK_TOPS, "unit": "TOP/s",
            "frac": achieved / VALU_PEAK_TOPS, "traffic": traffic,
            "kernel_ms": ms_kernel, "density_call_ms": ms_call,
            "frac_of_density_call": alg_ops / (ms_call * 1e-3) / 1e12 / VALU_PEAK_TOPS,
            "work": f"{OPS_PER_CANDIDATE} lane-ops per candidate of the exact per-receiver "
                    f"bounds ({cand / n:.1f} per particle) + {OPS_PER_INTERACTION} per pair in "
                    f"range ({inr / n:.1f}) = {alg_ops / n:.0f} lane-ops per particle",
            "executed_pair_slots_per_particle": slots / n,
            "slot_efficiency": inr / slots if slots else None}


def _kernel_ms(ctx, fn, steps):
    """Mean duration (ms) of the persistent sweep kernel over `steps` calls of
    fn, from the HIP events the library records around each launch on its
    stream (one warm-up call first)."""
    fn()
    ctx.set_kernel_timing(True)
    for _ in range(steps):
        fn()
    ts = ctx.kernel_times(steps)
    ctx.set_kernel_timing(False)
    return sum(ts) / len(ts)


def _path_roofline(n, alg_ops, ms_step):
    """The whole step (build + sort + sweep) against its binding roof: the
    larger of the vector-ALU floor of the sweep's algorithmic work and the HBM
    floor of the step's algorithmic bytes."""
    alu_ms = alg_ops / (VALU_PEAK_TOPS * 1e12) * 1e3
    hbm_bytes = sum(HBM_BYTES.values()) * n
    hbm_ms = hbm_bytes / (HBM_PEAK_GBS * 1e9) * 1e3
    bound = "alu" if alu_ms >= hbm_ms else "hbm"
    return {"bound": bound, "floor_alu_ms": alu_ms, "floor_hbm_ms": hbm_ms,
            "hbm_bytes_per_particle": sum(HBM_BYTES.values()), "ms_per_step": ms_step,
            "frac": max(alu_ms, hbm_ms) / ms_step,
            "hbm_frac_whole_step": hbm_ms / ms_step}


def _hbm_fractions(workload, n, stage_ms):
    """Algorithmic HBM bytes over time for the bandwidth-bound stages: from
    the stage times measured here (several launches each), and per stage from
    the kernel durations of the committed rocprofv3 summary of this workload
    when it was taken on the current library sources."""
    live = {}
    for stage, key, b in (("build (bin + scatter)", "build_cells", HBM_BYTES["bin"] +
                           HBM_BYTES["scatter"]),
                          ("sort13", "sort_cells", HBM_BYTES["sort13"]),
                          ("sweep", "density_sweep", HBM_BYTES["sweep"])):
        tbs = b * n / (stage_ms[key] * 1e-3) / 1e12
        live[stage] = {"bytes_per_particle": b, "ms": stage_ms[key], "achieved_TB_s": tbs,
                       "frac": tbs / (HBM_PEAK_GBS / 1e3)}
    out = {"peak_TB_s": HBM_PEAK_GBS / 1e3, "stages_live": live, "kernels_profiled": None}
    prof = _profile(workload)
    if prof is not None:
        per = {}
        for stage, names in STAGE_KERNELS.items():
            us = 0.0
            used = []
            for k, v in prof["kernels"].items():
                if k.startswith(names):
                    # kernels launched once per step of the profiled command
                    us += v["avg_us"]
                    used.append(k)
            if us > 0:
                tbs = HBM_BYTES[stage] * n / (us * 1e-6) / 1e12
                per[stage] = {"kernels": sorted(used), "us": us,
                              "bytes_per_particle": HBM_BYTES[stage], "achieved_TB_s": tbs,
                              "frac": tbs / (HBM_PEAK_GBS / 1e3)}
        out["kernels_profiled"] = per
    return out


def _profile(workload):
    """The committed rocprofv3 summary of this workload, if it was taken on
    the current library sources."""
    from paper_1804_06231_amd.rocprof_summary import source_hash
    path = os.path.join(ROOT, "profiles", f"{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_hash") != source_hash():
        return None
    return rec


def bench_batched(a, b, torch, pvl, t0):
    """Many boxes: one step = build_cells + sort_cells + density + adjoint over
    every box.  Timed as one captured HIP graph, as the same calls issued
    eagerly, and as a loop that runs each box on its own."""
    print(f"[bench] inputs ready in {time.time() - t0:.1f}s (n={b.n}, {b.nbox} boxes)",
          file=sys.stderr, flush=True)
    dev = torch.device("cuda", 0)
    pos = torch.from_numpy(b.pos).to(dev)
    h = torch.from_numpy(b.h).to(dev)
    m = torch.from_numpy(b.m).to(dev)
    n = b.n
    off = [int(x) for x in b.offsets]
    gen = torch.Generator(device=dev)
    gen.manual_seed(7)
    g_rho = torch.randn(n, generator=gen, device=dev)
    ctx = pvl.Context(0)
    rho, wc, dh = (torch.empty(n, device=dev) for _ in range(3))
    nc = torch.empty(n, dtype=torch.int32, device=dev)
    gp, gh = torch.empty((n, 3), device=dev), torch.empty(n, device=dev)

    grids = b.grids
    grid_tune = None
    if not a.no_autotune:
        print("[bench] autotuning the grids", file=sys.stderr, flush=True)
        grids, t_fine, t_best = ctx.autotune_grid(pos, h, m, reps=2, offsets=off, boxes=b.boxes)
        grid_tune = {"finest_step_ms": t_fine, "tuned_step_ms": t_best,
                     "grids_per_side": [min(g[0] for g in grids), max(g[0] for g in grids)]}
    cells = ctx.build_cells_batched(off, pos, h, m, b.boxes, grids)
    ctx.sort_cells(cells)
    ctx.density(cells, "sorted", (rho, wc, dh, nc))
    ctx.check()
    pairs = int(nc.sum().item())
    ctx.set_census(True)
    ctx.density(cells, "sorted")
    cand, inr, slots = ctx.census()
    ctx.set_census(False)
    tuning = _autotune(a, ctx, cells, g_rho, ("density", "adjoint"))

    def step():
        ctx.build_cells_batched(off, pos, h, m, b.boxes, grids, cells)
        ctx.sort_cells(cells)
        ctx.density(cells, "sorted", (rho, wc, dh, nc))
        ctx.density_backward(cells, g_rho, (gp, gh))

    # the same work box by box, each box with its own cell structure
    boxes = []
    for k in range(b.nbox):
        sl = slice(off[k], off[k + 1])
        c = ctx.build_cells(pos[sl], h[sl], m[sl], b.boxes[k], grids[k])
        boxes.append((c, sl))

    def step_loop():
        for k, (c, sl) in enumerate(boxes):
            ctx.build_cells(pos[sl], h[sl], m[sl], b.boxes[k], grids[k], c)
            ctx.sort_cells(c)
            ctx.density(c, "sorted", (rho[sl], wc[sl], dh[sl], nc[sl]))
            ctx.density_backward(c, g_rho[sl], (gp[sl], gh[sl]))

    print("[bench] timing the eager batched step", file=sys.stderr, flush=True)
    ms_eager, _ = _time_loop(step, a.steps, a.warmup, torch)
    print("[bench] capturing and timing the graph", file=sys.stderr, flush=True)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        step()
    ms_graph, wall_graph = _time_loop(graph.replay, a.steps, a.warmup, torch)
    ctx.check()
    print("[bench] timing the per-box loop", file=sys.stderr, flush=True)
    ms_loop, _ = _time_loop(step_loop, max(1, a.steps // 4), 1, torch)
    ctx.check()
    # stage times of the batched structure
    ms_build, _ = _time_loop(lambda: ctx.build_cells_batched(off, pos, h, m, b.boxes, grids, cells),
                             a.steps, 1, torch)
    ms_sort, _ = _time_loop(lambda: ctx.sort_cells(cells), a.steps, 1, torch)
    ms_sweep, _ = _time_loop(lambda: ctx.density(cells, "sorted", (rho, wc, dh, nc)), a.steps, 1, torch)
    ms_kernel = _kernel_ms(ctx, lambda: ctx.density(cells, "sorted", (rho, wc, dh, nc)), a.steps)
    ms_adj, _ = _time_loop(lambda: ctx.density_backward(cells, g_rho, (gp, gh)), a.steps, 1, torch)
    ctx.check()
    del graph

    alg_ops = OPS_PER_CANDIDATE * cand + OPS_PER_INTERACTION * inr
    cpu = None
    if not a.no_cpu_baseline:
        print("[bench] timing the fp64 CPU oracle on a sample", file=sys.stderr, flush=True)
        cpu = _cpu_baseline_batched(b, a.cpu_seconds)
    rec = {
        "metric": "density pair-interactions/s + ns/particle, sorted-pair vs cell-list, 1 GPU",
        "value": pairs / (ms_graph * 1e-3),
        "unit": "pair-interactions/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_graph,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": b.name, "n": n, "nbox": b.nbox, "seed": b.seed,
                   "particles_per_box": [min(np.diff(b.offsets).tolist()),
                                         max(np.diff(b.offsets).tolist())],
                   "grids_per_side": [min(g[0] for g in grids) if grid_tune else min(b.grids),
                                      max(g[0] for g in grids) if grid_tune else max(b.grids)],
                   "step": "build_cells + sort_cells + density + adjoint over all boxes, "
                           "one HIP graph launch"},
        "ns_per_particle": ms_graph * 1e6 / n,
        "pairs_in_range": pairs,
        "eager_batched_ms": ms_eager,
        "per_box_loop_ms": ms_loop,
        "speedup_graph_vs_per_box_loop": ms_loop / ms_graph,
        "stages_ms": {"build_cells": ms_build, "sort_cells": ms_sort, "density_sweep": ms_sweep,
                      "adjoint_sweep": ms_adj},
        "candidates_per_particle": {"sorted": cand / n, "in_range": inr / n},
        "autotune": tuning,
        "grid_autotune": grid_tune,
        "wall_ms_per_step": wall_graph,
        "roofline": _roofline(b.name, n, alg_ops, cand, inr, slots, ms_kernel, ms_sweep,
                              _traffic(b.name, SWEEP_KERNEL)),
        "cpu_baseline": cpu,
    }
    print(json.dumps(rec))


def _bench_reuse(a, ctx, s, pos, h, m, grid, out, torch):
    """Steps that keep the cells and their sorted lists (Section 2's reuse with
    bounds widened by the displacement): drift every particle by a fixed small
    step, then the sorted-pair density.  The step length leaves room in the
    cells for all the steps timed here."""
    cells = ctx.build_cells(pos, h, m, s.box, grid)
    ctx.sort_cells(cells)
    info = cells.info()
    room = min(s.box) / max(info["grid"]) - info["hmax"]
    nstep = a.warmup + 2 * (a.steps + 1) + 4
    dx = room / (4.0 * nstep)
    gen = torch.Generator(device=pos.device)
    gen.manual_seed(11)
    d = torch.randn((s.n, 3), generator=gen, device=pos.device)
    d = d / d.norm(dim=1, keepdim=True) * dx

    def step():
        ctx.drift(cells, d)
        ctx.density(cells, "sorted", out)

    ms_eager, _ = _time_loop(step, a.steps, a.warmup, torch)
    graph = _capture(step, torch)
    ms, _ = _time_loop(graph.replay, a.steps, 0, torch)
    ctx.check()
    del graph
    return {"ms_per_step": ms, "eager_ms_per_step": ms_eager, "displacement_per_step": dx,
            "step": "drift + sorted-pair density on kept cells and sorted lists"}


def _bench_lj(a, ctx, torch):
    """Second workload through the same sweep: Lennard-Jones forces and energies
    on 10^6 particles (jittered 100^3 lattice, cut-off 2.5 spacings); a step is
    build_cells + sort_cells + the force sweep, timed as a HIP graph."""
    from synth import workload
    s = workload("lj-1m")
    dev = torch.device("cuda", 0)
    pos, h, m = (torch.from_numpy(x).to(dev) for x in (s.pos, s.h, s.m))
    grid_tune = None
    grid = None
    if not a.no_autotune:
        (grid,), t_fine, t_best = ctx.autotune_grid(pos, h, m, s.box, reps=3)
        grid_tune = {"finest_step_ms": t_fine, "tuned_step_ms": t_best}
    cells = ctx.build_cells(pos, h, m, s.box, grid)
    grid = cells.info()["grid"]
    ctx.sort_cells(cells)
    _, _, _, nc = ctx.density(cells, "sorted")
    pairs = int(nc.sum().item())
    f = torch.empty((s.n, 3), device=dev)
    e = torch.empty(s.n, device=dev)
    sigma, eps = s.extra["sigma"], 1.0

    def step():
        ctx.build_cells(pos, h, m, s.box, grid, cells)
        ctx.sort_cells(cells)
        ctx.lj(cells, eps, sigma, (f, e))

    graph = _capture(step, torch)
    ms, _ = _time_loop(graph.replay, a.steps, a.warmup, torch)
    ms_sweep, _ = _time_loop(lambda: ctx.lj(cells, eps, sigma, (f, e)), a.steps, 1, torch)
    ctx.check()
    del graph
    return {"workload": s.name, "n": s.n, "grid": list(grid), "pairs_in_range": pairs,
            "ms_per_step": ms, "pair_interactions_per_s": pairs / (ms * 1e-3),
            "force_sweep_ms": ms_sweep, "grid_autotune": grid_tune,
            "step": "build_cells + sort_cells + Lennard-Jones sweep, one HIP graph launch"}


def _bench_hsolve(ctx, s, pos, m, torch):
    """h-iteration on the workload's positions: Newton on rho h^3 = m eta^3 to
    a relative residual of 1e-6, from a constant 48-neighbour start on uniform
    workloads.  On clustered ones a constant start puts thousands of
    particles in a dense cell (above the cell limit), so they start from
    their own h scaled by a seeded U(0.95, 1.05) factor per particle; an
    iteration that still crowds a cell is reported, not timed.  The context
    keeps the solver's working set between calls: the first call (which
    allocates it) is timed apart from a second, steady-state one."""
    from paper_1804_06231_amd import PVError
    from synth import h_for_neighbours
    if s.name.startswith("uniform"):
        start = "constant h of 48 neighbours at the mean density"
        h = torch.full((s.n,), h_for_neighbours(s.n, L=s.box[0]), dtype=torch.float32,
                       device=pos.device)
    else:
        start = "the workload's h times U(0.95, 1.05) (seed 7)"
        f = np.random.Generator(np.random.PCG64(7)).uniform(0.95, 1.05, s.n).astype(np.float32)
        h = torch.from_numpy(s.h * f).to(pos.device)
    times = []
    for _ in range(2):
        hh = h.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        try:
            it, res = ctx.solve_h(pos, m, hh, s.box, ngb=48.0, tol=1e-6, max_iter=40)
        except PVError as e:
            return {"start": start, "error": str(e)}
        torch.cuda.synchronize()
        times.append((time.perf_counter() - t0) * 1e3)
    ms = times[1]
    return {"iterations": it, "residual": res, "ms": ms, "ms_per_iteration": ms / max(it, 1),
            "first_call_ms": times[0], "start": start, "tol": 1e-6}


def _cpu_baseline_batched(b, target_seconds):
    """fp64 oracle on every receiver of boxes taken in a seeded random order."""
    from oracle import Oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    rng = np.random.Generator(np.random.PCG64(123))
    dt = 0.0
    pairs = nrecv = 0
    used = 0
    for k in rng.permutation(b.nbox):
        s = b.sets[k]
        o = Oracle(s.pos, s.h, s.m, s.box, b.grids[k])
        t0 = time.perf_counter()
        d = o.density()
        dt += time.perf_counter() - t0
        pairs += int(d["ncount"].sum())
        nrecv += s.n
        used += 1
        if dt > 0.4 * target_seconds:
            break
    return {"value": pairs / dt, "unit": "pair-interactions/s", "cores": threads, "kind": "oracle",
            "sample": f"all {nrecv} receivers of {used} of the {b.nbox} boxes (seeded random "
                      f"order), fp64 27-cell brute force, {dt:.2f}s",
            "ns_per_particle": dt * 1e9 / nrecv}


def _traffic(workload, kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary of this workload, if it was taken on the current library sources."""
    rec = _profile(workload)
    if rec is None:
        return None
    t = rec.get("traffic", {}).get(kernel)
    if not t:
        return None
    return t["fetch_bytes"] + t["write_bytes"]


def _omp_threads(k):
    """Set the OpenMP thread count of this process (the oracle's parallel
    loops) and return the previous one."""
    import ctypes
    gomp = ctypes.CDLL("libgomp.so.1")
    prev = gomp.omp_get_max_threads()
    gomp.omp_set_num_threads(int(k))
    return prev


def _cpu_baseline(s, target_seconds):
    """fp64 oracle (C + OpenMP cell-list brute force) on a sample of receivers:
    the median of 5 runs on all host threads (the paper's timing takes the
    median of 5 runs), and one run on one thread over an eighth of the sample
    (the paper's figures are single-thread)."""
    from oracle import Oracle
    o = Oracle(s.pos, s.h, s.m, s.box)
    threads = _omp_threads(0) or 1
    _omp_threads(threads)
    rng = np.random.Generator(np.random.PCG64(123))
    per_run = target_seconds / 8.0     # 5 runs + the one-thread run ~ 8 runs' time
    k = 16384
    while True:
        idx = np.sort(rng.choice(s.n, min(k, s.n), replace=False))
        t0 = time.perf_counter()
        d = o.density(idx)
        dt = time.perf_counter() - t0
        if dt > 0.5 * per_run or k >= s.n:
            break
        k = min(s.n, int(k * max(2.0, 0.7 * per_run / max(dt, 1e-3))))
    pairs = int(d["ncount"].sum())
    runs = [dt]
    for _ in range(4):
        t0 = time.perf_counter()
        o.density(idx)
        runs.append(time.perf_counter() - t0)
    med = float(np.median(runs))
    sub = idx[: max(1, idx.size // 8)]
    prev = _omp_threads(1)
    try:
        t0 = time.perf_counter()
        d1 = o.density(sub)
        dt1 = time.perf_counter() - t0
    finally:
        _omp_threads(prev)
    pairs1 = int(d1["ncount"].sum())
    return {"value": pairs / med, "unit": "pair-interactions/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{idx.size} of {s.n} receivers (uniform random), full 27-cell fp64 "
                      f"brute force, median of 5 runs ({min(runs):.2f}-{max(runs):.2f}s)",
            "ns_per_particle": med * 1e9 / idx.size,
            "runs_s": runs,
            "one_thread": {"value": pairs1 / dt1, "unit": "pair-interactions/s", "cores": 1,
                           "sample": f"{sub.size} receivers (the first eighth of the sample), "
                                     f"{dt1:.2f}s", "ns_per_particle": dt1 * 1e9 / sub.size}}


if __name__ == "__main__":
    main()
