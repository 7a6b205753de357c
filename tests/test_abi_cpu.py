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
        pytest.fail("libpvl.so is not built (run __graft_entry__.build())")
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
