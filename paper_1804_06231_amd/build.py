"""Build libpvl.so (the HIP library behind include/pvl.h) for gfx950, in-tree.

    python -m paper_1804_06231_amd.build            # compile every source
    python -m paper_1804_06231_amd.build --jobs 8

Each .hip file is compiled to an object in parallel, then linked into
paper_1804_06231_amd/libpvl.so.  Packed fp32 instructions are disabled for all
device code, and multiply-add fusion happens only where the source asks
for it (fmaf).
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import glob
import json
import os
import re
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libpvl.so")
ARCH = os.environ.get("PVL_OFFLOAD_ARCH", "gfx950")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CFLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # no implicit multiply-add fusion: cell origins and cell-pair shifts must be
    # rounded exactly as written for the differences taken from them to be
    # exact; every intended fused multiply-add is an explicit fmaf
    "-ffp-contract=off",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
    "-Wall", "-Wno-unused-function",
]


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


# The compiler's per-kernel resource report (registers, scratch, occupancy),
# kept beside the objects: a kernel that spills registers to scratch memory
# is slower by a wide margin, so the build records it and the CPU tests check.
RESOURCES = os.path.join(BUILD, "resources.json")
_REMARK = re.compile(r"remark:\s+(Function Name|VGPRs|AGPRs|ScratchSize \[bytes/lane\]|"
                     r"Occupancy \[waves/SIMD\]|LDS Size \[bytes/block\]):\s+(\S+)")


def _resources(stderr: str) -> dict:
    """{kernel: {field: value}} from the resource-usage remarks of one compile."""
    out, cur = {}, None
    for line in stderr.splitlines():
        m = _REMARK.search(line)
        if not m:
            continue
        key, val = m.group(1), m.group(2)
        if key == "Function Name":
            cur = out.setdefault(val, {})
        elif cur is not None:
            cur[key.split(" ")[0]] = int(val)
    return out


def _compile(src: str):
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [HIPCC, *CFLAGS, "-Rpass-analysis=kernel-resource-usage", "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    return obj, _resources(r.stderr)


def build(jobs: int = 8, verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    with cf.ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        done = list(ex.map(_compile, srcs))
    objs = [o for o, _ in done]
    res = {}
    for _, r in done:
        res.update(r)
    with open(RESOURCES, "w") as f:
        json.dump(res, f, indent=1, sort_keys=True)
    spills = sorted(k for k, v in res.items() if v.get("ScratchSize", 0) > 0)
    if spills:
        print("build: kernels using scratch memory (register spills): " + ", ".join(spills),
              file=sys.stderr)
    tmp = LIB + f".tmp{os.getpid()}"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB} from {len(srcs)} sources")
    return LIB


# Host code built with AddressSanitizer (device code as usual), for the CPU
# tests of the C ABI: load it with the sanitizer runtime preloaded.
ASAN_DIR = os.path.join(BUILD, "asan")
ASAN_LIB = os.path.join(ASAN_DIR, "libpvl.so")
ASAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer"]


def asan_runtime() -> str:
    """Path of the compiler's AddressSanitizer runtime (empty if absent)."""
    r = subprocess.run([HIPCC, "-print-file-name=libclang_rt.asan-x86_64.so"],
                       capture_output=True, text=True)
    p = r.stdout.strip()
    return p if r.returncode == 0 and os.path.isabs(p) and os.path.exists(p) else ""


def build_asan(jobs: int = 8) -> str:
    os.makedirs(ASAN_DIR, exist_ok=True)
    flags = [f if f != "-O3" else "-O1" for f in CFLAGS] + ["-g"] + ASAN_FLAGS

    def one(src):
        obj = os.path.join(ASAN_DIR, os.path.basename(src) + ".o")
        r = subprocess.run([HIPCC, *flags, "-c", src, "-o", obj], capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
        return obj

    with cf.ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        objs = list(ex.map(one, sources()))
    tmp = ASAN_LIB + f".tmp{os.getpid()}"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *ASAN_FLAGS, "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, ASAN_LIB)
    return ASAN_LIB


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=8)
    ap.add_argument("--asan", action="store_true",
                    help="also build the host-sanitizer library for the CPU tests")
    a = ap.parse_args(argv)
    build(a.jobs, verbose=True)
    if a.asan:
        print(f"built {build_asan(a.jobs)}")


if __name__ == "__main__":
    sys.exit(main())
