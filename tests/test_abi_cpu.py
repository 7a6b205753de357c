"""The C-ABI library on a host without a GPU: it loads, exports exactly what
include/pvl.h declares, and validates arguments before touching a device."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pvl.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(pv_[a-z_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    from paper_1804_06231_amd.pvl import load_library, LIB_PATH
    if not os.path.exists(LIB_PATH):
        pytest.fail("libpvl.so is not built (python -m paper_1804_06231_amd.build)")
    return load_library()


def test_header_and_binding_agree():
    from paper_1804_06231_amd.pvl import EXPORTS
    assert sorted(EXPORTS) == _declared()


def test_every_declared_symbol_is_exported(lib):
    for name in _declared():
        assert hasattr(lib, name), name


def test_null_context_is_rejected(lib):
    assert lib.pv_sort_cells(None, None) == -1
    assert lib.pv_density(None, None, 0, None, None, None, None) == -1
    assert lib.pv_check(None) == -1
    assert lib.pv_create(0, None, None) == -1


@pytest.fixture()
def vctx(lib):
    h = C.c_void_p()
    assert lib.pv_create(-1, None, C.byref(h)) == 0
    yield h
    lib.pv_destroy(h)


def _build(lib, ctx, n, box=(1.0, 1.0, 1.0), grid=None, ptrs=True):
    off = (C.c_int64 * 2)(0, n)
    b = (C.c_double * 3)(*box)
    g = None if grid is None else (C.c_int * 3)(*grid)
    fake = C.c_void_p(0x1000) if ptrs else None
    cells = C.c_void_p()
    return lib.pv_build_cells_batched(ctx, 1, off, fake, fake, fake, b, g, C.byref(cells))


def test_argument_validation_without_gpu(lib, vctx):
    assert lib.pv_build_cells(vctx, -1, None, None, None, None, None, None) == -1     # n < 0
    assert _build(lib, vctx, 10, box=(1.0, 0.0, 1.0)) == -1                           # box <= 0
    assert _build(lib, vctx, 10, box=(1.0, float("nan"), 1.0)) == -1
    assert _build(lib, vctx, 10, ptrs=False) == -1                                    # NULL arrays
    assert _build(lib, vctx, 10, grid=(2, 4, 4)) == -4                                # grid < 3
    assert _build(lib, vctx, 10, grid=(4, 4, 5000)) == -4                             # grid too big
    assert _build(lib, vctx, 10, grid=(4, 4, 4)) == -6                                # valid: no device
    assert b"no device" in lib.pv_last_error(vctx)
    off = (C.c_int64 * 3)(0, 5, 3)                                                    # decreasing
    cells = C.c_void_p()
    assert lib.pv_build_cells_batched(vctx, 2, off, None, None, None, (C.c_double * 6)(*[1.0] * 6),
                                      None, C.byref(cells)) == -1
    off = (C.c_int64 * 2)(1, 5)                                                       # offsets[0] != 0
    assert lib.pv_build_cells_batched(vctx, 1, off, None, None, None, (C.c_double * 3)(1, 1, 1),
                                      None, C.byref(cells)) == -1
    assert lib.pv_build_cells_batched(vctx, 0, off, None, None, None, None, None,
                                      C.byref(cells)) == -1                           # nbox < 1
    assert lib.pv_sort_cells(vctx, None) == -1
    assert lib.pv_density(vctx, None, 0, None, None, None, None) == -1
    assert lib.pv_check(vctx) == 0


def test_python_binding_refuses_without_library(tmp_path):
    from paper_1804_06231_amd import pvl
    saved = pvl._lib
    pvl._lib = None
    try:
        with pytest.raises(RuntimeError, match="not found"):
            pvl.load_library(str(tmp_path / "missing.so"))
    finally:
        pvl._lib = saved


def test_tuning_parameters_without_gpu(lib, vctx):
    """Parameters are validated and kept per sweep (density / adjoint)."""
    from paper_1804_06231_amd.pvl import PARAMS, PV_PARAM_ADJOINT, PV_PARAM_PLAIN
    v = C.c_int()
    defaults = {"reach_order": 0, "task_sort": 1, "queue_wgs": 5, "chunk": 256,
                "tail_parts": 2, "tail_cells": 0, "group": 0, "sym_self": 0,
                "xcd_ranges": 0, "tail_split": 0}
    for name, p in PARAMS.items():
        for off in (0, PV_PARAM_ADJOINT, PV_PARAM_PLAIN):
            assert lib.pv_get_param(vctx, p + off, C.byref(v)) == 0
            assert v.value == defaults[name], (name, off)
    assert lib.pv_set_param(vctx, PARAMS["chunk"], 128) == 0
    assert lib.pv_get_param(vctx, PARAMS["chunk"], C.byref(v)) == 0 and v.value == 128
    assert lib.pv_get_param(vctx, PARAMS["chunk"] + PV_PARAM_ADJOINT, C.byref(v)) == 0
    assert v.value == 256                                         # the adjoint's is separate
    assert lib.pv_get_param(vctx, PARAMS["chunk"] + PV_PARAM_PLAIN, C.byref(v)) == 0
    assert v.value == 256
    for bad in (16, 100, 272, 0):
        assert lib.pv_set_param(vctx, PARAMS["chunk"], bad) == -1
    assert lib.pv_get_param(vctx, PARAMS["chunk"], C.byref(v)) == 0 and v.value == 128
    assert lib.pv_set_param(vctx, PARAMS["queue_wgs"], 0) == -1
    assert lib.pv_set_param(vctx, PARAMS["queue_wgs"], 9) == -1
    assert lib.pv_set_param(vctx, PARAMS["queue_wgs"], 8) == 0
    for bad in (0, 3, 8):
        assert lib.pv_set_param(vctx, PARAMS["tail_parts"], bad) == -1
    assert lib.pv_set_param(vctx, PARAMS["tail_parts"], 4) == 0
    assert lib.pv_set_param(vctx, PARAMS["tail_cells"], 2049) == -1
    assert lib.pv_set_param(vctx, PARAMS["tail_cells"], -1) == -1
    assert lib.pv_set_param(vctx, PARAMS["tail_cells"], 2048) == 0
    assert lib.pv_get_param(vctx, PARAMS["tail_cells"], C.byref(v)) == 0 and v.value == 2048
    for bad in (9, -1):
        assert lib.pv_set_param(vctx, PARAMS["group"], bad) == -1
    assert lib.pv_set_param(vctx, PARAMS["group"] + PV_PARAM_ADJOINT, 3) == 0
    assert lib.pv_get_param(vctx, PARAMS["group"] + PV_PARAM_ADJOINT, C.byref(v)) == 0
    assert v.value == 3
    assert lib.pv_get_param(vctx, PARAMS["group"], C.byref(v)) == 0 and v.value == 0
    assert lib.pv_set_param(vctx, 11, 1) == -1                    # unknown
    assert lib.pv_get_param(vctx, 11, C.byref(v)) == -1
    # the autotuner validates before it needs a device
    t = (C.c_float * 2)()
    assert lib.pv_autotune(vctx, None, 0, None, 3, t) == -1
    assert lib.pv_autotune(None, None, 0, None, 3, t) == -1


def test_kernel_timing_argument_checks_without_gpu(lib, vctx):
    """Kernel timing needs a device context; its read-back checks its
    arguments first."""
    n = C.c_int(4)
    ms = (C.c_float * 4)()
    assert lib.pv_set_kernel_timing(None, 1) == -1
    assert lib.pv_kernel_times(None, ms, C.byref(n)) == -1
    assert lib.pv_kernel_times(vctx, ms, None) == -1
    assert lib.pv_kernel_times(vctx, None, C.byref(n)) == -1     # ms NULL with count > 0
    bad = C.c_int(-1)
    assert lib.pv_kernel_times(vctx, ms, C.byref(bad)) == -1
    assert lib.pv_set_kernel_timing(vctx, 1) == -6                # no device (PV_ESTATE)
    assert lib.pv_kernel_times(vctx, ms, C.byref(n)) == -6


def test_bench_refuses_more_than_one_gpu():
    """The benchmark measures one GPU: asked for more it exits with a message
    (before touching a device)."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_static_density_argument_checks_without_gpu(lib, vctx):
    """pv_density_static checks its limits before touching a device."""
    from paper_1804_06231_amd.pvl import PV_STATIC_MAX_N, PV_STATIC_MAX_CELLS
    fake = C.c_void_p(0x1000)
    box = (C.c_double * 3)(1.0, 1.0, 1.0)

    def call(n, grid, b=box, ptr=fake, algo=0):
        g = None if grid is None else (C.c_int * 3)(*grid)
        return lib.pv_density_static(vctx, n, ptr, ptr, ptr, b, g, algo, fake, fake, fake, fake)

    assert call(100, (4, 4, 4)) == -6                                      # valid: no device
    assert call(-1, (4, 4, 4)) == -1
    assert call(PV_STATIC_MAX_N + 1, (4, 4, 4)) == -1                      # above the scratch
    assert b"static scratch" in lib.pv_last_error(vctx)
    assert call(PV_STATIC_MAX_N, (4, 4, 4)) == -6
    assert call(100, None) == -1                                            # grid required
    assert call(100, (2, 4, 4)) == -4
    assert call(100, (33, 32, 32)) == -1                                    # > 32768 cells
    assert 32 * 32 * 32 == PV_STATIC_MAX_CELLS and call(100, (32, 32, 32)) == -6
    assert call(100, (4, 4, 4), b=(C.c_double * 3)(1.0, -1.0, 1.0)) == -1
    assert call(100, (4, 4, 4), ptr=None) == -1
    assert call(0, (4, 4, 4), ptr=None) == -6                               # empty input
    assert call(100, (4, 4, 4), algo=7) == -1
    assert lib.pv_density_static(None, 10, fake, fake, fake, box, (C.c_int * 3)(4, 4, 4), 0,
                                 None, None, None, None) == -1
