"""The compiler's resource report of the last build (registers, scratch,
occupancy per kernel), written by paper_1804_06231_amd.build: no kernel of
the library spills registers to scratch memory, and the sweeps keep the
waves per SIMD their launch bounds ask for (a spill or a lost wave shows up
as a large slowdown, not as a wrong result)."""
import json
import os

import pytest

from paper_1804_06231_amd.build import RESOURCES


@pytest.fixture(scope="module")
def report():
    if not os.path.exists(RESOURCES):
        pytest.skip("no build report (python -m paper_1804_06231_amd.build)")
    with open(RESOURCES) as f:
        return json.load(f)


def _pvl(report):
    return {k: v for k, v in report.items() if k.startswith("_ZN3pvl")}


def test_report_covers_the_kernels(report):
    names = " ".join(_pvl(report))
    for k in ("k_sweep_queue", "k_sort13_small", "k_bin_local", "k_scatter", "k_cell_finish_small"):
        assert k in names, k


# At five waves per SIMD the adjoint sweep and the density sweep (whose row
# loop is built twice, for equal and for differing masses) keep a few
# loop-invariant lane values in scratch memory, reloaded once per work item
# outside the row loop; both measured faster so than at four waves without.
# Those are the spills allowed.
ALLOWED_SCRATCH = {
    "_ZN3pvl13k_sweep_queueILi2ELb0ELb0EEEvNS_9SweepArgsE": 16,
    "_ZN3pvl13k_sweep_queueILi0ELb0ELb0EEEvNS_9SweepArgsE": 40,
    "_ZN3pvl13k_sweep_queueILi0ELb0ELb1EEEvNS_9SweepArgsE": 40,
}


def test_no_kernel_spills(report):
    spills = {k: v["ScratchSize"] for k, v in _pvl(report).items()
              if v.get("ScratchSize", 0) > ALLOWED_SCRATCH.get(k, 0)}
    assert not spills, spills


def test_sweep_occupancy(report):
    # five waves per SIMD (five persistent workgroups per compute unit), four
    # for the symmetric own-cell forms
    for k, v in _pvl(report).items():
        if "k_sweep_queue" in k:
            sym = "Lb1ELb0E" in k
            assert v["Occupancy"] >= (4 if sym else 5), (k, v)
