"""Summarise rocprofv3 CSV output for the density path.

    python -m paper_1804_06231_amd.rocprof_summary \
        --trace DIR [--fetch DIR --write DIR --copy-mib 256] \
        --workload NAME --command "the profiled command" \
        --out-md profiles/NAME.md [--out-json profiles/NAME.json]

--trace    a `rocprofv3 --kernel-trace --stats --output-format csv` directory
--fetch    a `rocprofv3 --pmc FETCH_SIZE --output-format csv` directory
--write    a `rocprofv3 --pmc WRITE_SIZE --output-format csv` directory
--sq       a `rocprofv3 --pmc SQ_INSTS_VALU SQ_ACTIVE_INST_VALU
           SQ_THREAD_CYCLES_VALU SQ_INSTS_SALU SQ_INSTS_LDS SQ_WAVES
           --output-format csv` directory (vector-ALU use per kernel)

The byte counters are calibrated against the device copy of --copy-mib MiB
that `bench.py --copy-probe-mb` performs in the same run: the factor
(known bytes / counted bytes) of that copy scales every kernel's count.  The
JSON records, per kernel, the average duration, the scaled HBM bytes per
launch, and a hash of the library sources the numbers belong to.
"""
from __future__ import annotations

import argparse
import collections
import csv
import glob
import hashlib
import json
import os

PKG = os.path.dirname(os.path.abspath(__file__))


def source_hash() -> str:
    """Hash of the HIP sources and headers (numbers go stale when it changes)."""
    h = hashlib.sha256()
    files = sorted(glob.glob(os.path.join(PKG, "csrc", "*")))
    files.append(os.path.join(os.path.dirname(PKG), "include", "pvl.h"))
    for f in files:
        with open(f, "rb") as fh:
            h.update(os.path.basename(f).encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


def _short(name: str) -> str:
    name = name.replace("void ", "")
    base = name.split("(")[0]
    return base


def _col(row, *names):
    for n in names:
        for k in row:
            if k.strip().lower() == n.lower():
                return row[k]
    raise KeyError(names)


def kernel_stats(trace_dir):
    f = glob.glob(os.path.join(trace_dir, "**", "*kernel_stats.csv"), recursive=True)
    if not f:
        raise FileNotFoundError(f"no kernel_stats.csv under {trace_dir}")
    out = []
    for r in csv.DictReader(open(f[0])):
        out.append(dict(kernel=_short(_col(r, "Name")), calls=int(_col(r, "Calls")),
                        avg_us=float(_col(r, "AverageNs", "Average (nsec)", "Average (Nsec)")) / 1e3,
                        min_us=float(_col(r, "MinNs", "Min (nsec)", "Min (Nsec)")) / 1e3,
                        max_us=float(_col(r, "MaxNs", "Max (nsec)", "Max (Nsec)")) / 1e3,
                        share=float(_col(r, "Percentage", "Percent (Inc)"))))
    return out


def counter_per_dispatch(pmc_dir, counter):
    """{kernel: [value per dispatch]} for one counter."""
    f = glob.glob(os.path.join(pmc_dir, "**", "*counter_collection.csv"), recursive=True)
    if not f:
        raise FileNotFoundError(f"no counter_collection.csv under {pmc_dir}")
    per = collections.defaultdict(lambda: collections.defaultdict(float))
    for r in csv.DictReader(open(f[0])):
        if _col(r, "Counter_Name") != counter:
            continue
        per[_short(_col(r, "Kernel_Name"))][int(_col(r, "Dispatch_Id"))] += float(_col(r, "Counter_Value"))
    return {k: list(v.values()) for k, v in per.items()}


SQ_COUNTERS = ("SQ_INSTS_VALU", "SQ_ACTIVE_INST_VALU", "SQ_THREAD_CYCLES_VALU", "SQ_INSTS_SALU",
               "SQ_INSTS_LDS", "SQ_WAVES")
# MI355X: 256 compute units x 4 SIMDs, 2.4 GHz peak engine clock; a wave64
# vector instruction occupies a 16-lane SIMD for 4 cycles
SIMDS = 1024
CLOCK_HZ = 2.4e9


def sq_summary(sq_dir, stats):
    """Per kernel: counter averages per dispatch and two derived figures,
    the vector-ALU issue fraction (VALU instructions x 4 cycles over the
    SIMD-cycles of the kernel's average duration at the peak clock) and the
    active-lane fraction of a VALU instruction (SQ_THREAD_CYCLES_VALU over
    64 x SQ_ACTIVE_INST_VALU, the definition of rocprof's VALUUtilization)."""
    dur = {x["kernel"]: x["avg_us"] for x in stats}
    out = {}
    per = {c: counter_per_dispatch(sq_dir, c) for c in SQ_COUNTERS}
    for k in set().union(*[set(v) for v in per.values()]):
        avg = {c: (sum(per[c][k]) / len(per[c][k]) if per[c].get(k) else 0.0) for c in SQ_COUNTERS}
        rec = dict(avg)
        if k in dur and dur[k] > 0:
            rec["valu_issue_frac"] = avg["SQ_INSTS_VALU"] * 4.0 / (SIMDS * dur[k] * 1e-6 * CLOCK_HZ)
        if avg["SQ_ACTIVE_INST_VALU"] > 0:
            rec["valu_lane_frac"] = avg["SQ_THREAD_CYCLES_VALU"] / (64.0 * avg["SQ_ACTIVE_INST_VALU"])
        out[k] = rec
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--trace", required=True)
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--sq")
    ap.add_argument("--sq-command", default="")
    ap.add_argument("--copy-mib", type=float, default=256.0)
    ap.add_argument("--workload", required=True)
    ap.add_argument("--command", required=True)
    ap.add_argument("--out-md", required=True)
    ap.add_argument("--out-json")
    a = ap.parse_args(argv)

    stats = kernel_stats(a.trace)
    traffic = {}
    if a.fetch and a.write:
        fetch = counter_per_dispatch(a.fetch, "FETCH_SIZE")
        write = counter_per_dispatch(a.write, "WRITE_SIZE")
        copy_bytes = a.copy_mib * (1 << 20)
        # the calibration copy: the dispatch whose counts are largest among the
        # runtime's copy kernels / torch's copy kernels
        cands = [k for k in set(fetch) | set(write) if "copy" in k.lower()]
        best = max(cands, key=lambda k: max(write.get(k, [0])))
        fc = max(fetch.get(best, [0])) * 1024.0
        wc = max(write.get(best, [0])) * 1024.0
        f_fac = copy_bytes / fc if fc > 0 else None
        w_fac = copy_bytes / wc if wc > 0 else None
        for k in set(fetch) | set(write):
            fv = fetch.get(k, [])
            wv = write.get(k, [])
            fb = (sum(fv) / len(fv)) * 1024.0 if fv else 0.0
            wb = (sum(wv) / len(wv)) * 1024.0 if wv else 0.0
            traffic[k] = dict(fetch_bytes=fb * (f_fac or 1.0), write_bytes=wb * (w_fac or 1.0),
                              raw_fetch_kib=fb / 1024.0, raw_write_kib=wb / 1024.0)
        traffic["_calibration"] = dict(kernel=best, copy_bytes=copy_bytes, fetch_factor=f_fac,
                                       write_factor=w_fac)

    lines = [f"# Kernel profile: {a.workload}", "",
             "Command (from the repository root, one MI355X):", "", "```", a.command, "```", ""]
    if traffic:
        cal = traffic["_calibration"]
        lines += [f"HBM bytes: FETCH_SIZE and WRITE_SIZE (two separate `--pmc` runs of the "
                  f"same command), scaled by the factor that maps the counts of a "
                  f"{a.copy_mib:.0f} MiB device copy (`{cal['kernel']}`) onto its known size: "
                  f"fetch x{cal['fetch_factor']:.3f}, write x{cal['write_factor']:.3f}.", ""]
    lines += ["| kernel | calls | avg (us) | min (us) | max (us) | share | HBM read / launch | HBM write / launch |",
              "|---|---|---|---|---|---|---|---|"]
    for s in stats:
        t = traffic.get(s["kernel"])
        rd = f"{t['fetch_bytes'] / 1e6:.2f} MB" if t else ""
        wr = f"{t['write_bytes'] / 1e6:.2f} MB" if t else ""
        name = s["kernel"] if len(s["kernel"]) < 64 else s["kernel"][:61] + "..."
        lines.append(f"| `{name}` | {s['calls']} | {s['avg_us']:.1f} | {s['min_us']:.1f} | "
                     f"{s['max_us']:.1f} | {s['share']:.1f}% | {rd} | {wr} |")
    sq = sq_summary(a.sq, stats) if a.sq else {}
    if sq:
        lines += ["", "Vector-ALU use (one `--pmc` run with the counters "
                  + ", ".join(SQ_COUNTERS) + (f": `{a.sq_command}`" if a.sq_command else "")
                  + "). Issue fraction: VALU instructions x 4 cycles over 1024 SIMDs x the "
                  "kernel's average duration at 2.4 GHz. Lane fraction: SQ_THREAD_CYCLES_VALU / "
                  "(64 x SQ_ACTIVE_INST_VALU).", "",
                  "| kernel | VALU instr / launch | SALU instr | LDS instr | waves | VALU issue | active lanes |",
                  "|---|---|---|---|---|---|---|"]
        for st in stats:
            r = sq.get(st["kernel"])
            if not r or r["SQ_INSTS_VALU"] < 1e5:
                continue
            name = st["kernel"] if len(st["kernel"]) < 64 else st["kernel"][:61] + "..."
            lines.append(f"| `{name}` | {r['SQ_INSTS_VALU'] / 1e6:.1f}M | "
                         f"{r['SQ_INSTS_SALU'] / 1e6:.1f}M | {r['SQ_INSTS_LDS'] / 1e6:.2f}M | "
                         f"{r['SQ_WAVES']:.0f} | {100 * r.get('valu_issue_frac', 0):.1f}% | "
                         f"{100 * r.get('valu_lane_frac', 0):.1f}% |")
    lines += ["", f"Library source hash: `{source_hash()}`", ""]
    os.makedirs(os.path.dirname(os.path.abspath(a.out_md)), exist_ok=True)
    with open(a.out_md, "w") as f:
        f.write("\n".join(lines))
    if a.out_json:
        rec = dict(workload=a.workload, command=a.command, source_hash=source_hash(),
                   kernels={s["kernel"]: dict(avg_us=s["avg_us"], calls=s["calls"]) for s in stats},
                   traffic=traffic, sq=sq)
        with open(a.out_json, "w") as f:
            json.dump(rec, f, indent=1, sort_keys=True)
    print("\n".join(lines))


if __name__ == "__main__":
    main()
