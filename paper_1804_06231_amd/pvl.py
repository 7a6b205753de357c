"""ctypes binding of libpvl.so (include/pvl.h).

Argument marshalling only: every step of the density loop runs in the HIP
library.  PyTorch provides device memory and the stream; tensors must be
contiguous fp32 (int32 for counts) on the context's GPU.  If the library is
not built, loading fails with an error -- there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import json
import math
import os
from typing import Optional, Sequence

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
# the in-tree build; PVL_LIBRARY names another build of the same library (the
# host-sanitizer build of the CPU tests)
LIB_PATH = os.environ.get("PVL_LIBRARY") or os.path.join(_PKG, "libpvl.so")

PV_OK, PV_EINVAL, PV_ENOMEM, PV_EHIP, PV_EGRID, PV_EOVERFLOW, PV_ESTATE = 0, -1, -2, -3, -4, -5, -6
PV_SORTED_PAIR, PV_PLAIN_CELL = 0, 1
PV_MAX_CELL = 8192
PV_MAX_GRID = 1024
ALGOS = {"sorted": PV_SORTED_PAIR, "plain": PV_PLAIN_CELL}

# every symbol the header declares (checked by the CPU tests)
EXPORTS = (
    "pv_create", "pv_destroy", "pv_set_stream", "pv_last_error", "pv_build_cells",
    "pv_build_cells_batched", "pv_sort_cells", "pv_density", "pv_density_backward",
    "pv_check", "pv_cells_info", "pv_cells_export", "pv_set_census", "pv_census",
    "pv_free_cells", "pv_set_param", "pv_get_param", "pv_autotune", "pv_solve_h", "pv_drift",
    "pv_lj", "pv_autotune_grid", "pv_density_static", "pv_set_kernel_timing",
    "pv_kernel_times",
)
PV_KTIME_RING = 64
PV_STATIC_MAX_N = 131072
PV_STATIC_MAX_CELLS = 32768
PARAMS = {"reach_order": 1, "task_sort": 2, "queue_wgs": 3, "chunk": 4, "tail_parts": 5,
          "tail_cells": 6, "group": 7, "sym_self": 8,
          "xcd_ranges": 9, "tail_split": 10}
PV_PARAM_ADJOINT = 16
PV_PARAM_PLAIN = 32
TUNE_TARGETS = {"density": 0, "adjoint": 1, "plain": 2}
_SET_OFFSET = {"density": 0, "adjoint": PV_PARAM_ADJOINT, "plain": PV_PARAM_PLAIN}

_STATUS = {
    PV_EINVAL: "PV_EINVAL", PV_ENOMEM: "PV_ENOMEM", PV_EHIP: "PV_EHIP",
    PV_EGRID: "PV_EGRID", PV_EOVERFLOW: "PV_EOVERFLOW", PV_ESTATE: "PV_ESTATE",
}


class PVError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libpvl.so and declare its signatures.  Raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libpvl.so not found at {path}: build it with "
                           "`python -m paper_1804_06231_amd.build`")
    lib = C.CDLL(path)
    P, i32, i64 = C.c_void_p, C.c_int, C.c_int64
    sig = {
        "pv_create": ([i32, P, P], i32),
        "pv_destroy": ([P], None),
        "pv_set_stream": ([P, P], i32),
        "pv_last_error": ([P], C.c_char_p),
        "pv_build_cells": ([P, i64, P, P, P, P, P, P], i32),
        "pv_build_cells_batched": ([P, i32, P, P, P, P, P, P, P], i32),
        "pv_sort_cells": ([P, P], i32),
        "pv_density": ([P, P, i32, P, P, P, P], i32),
        "pv_density_backward": ([P, P, P, P, P], i32),
        "pv_check": ([P], i32),
        "pv_cells_info": ([P, P, P, P, P, P, P, P], i32),
        "pv_cells_export": ([P, P, P, P, P], i32),
        "pv_set_census": ([P, i32], i32),
        "pv_census": ([P, P], i32),
        "pv_free_cells": ([P, P], i32),
        "pv_set_param": ([P, i32, i32], i32),
        "pv_get_param": ([P, i32, P], i32),
        "pv_autotune": ([P, P, i32, P, i32, P], i32),
        "pv_solve_h": ([P, i32, P, P, P, P, P, C.c_float, C.c_float, i32, P, P], i32),
        "pv_drift": ([P, P, P], i32),
        "pv_lj": ([P, P, C.c_float, C.c_float, P, P], i32),
        "pv_autotune_grid": ([P, i32, P, P, P, P, P, i32, P, P], i32),
        "pv_density_static": ([P, i64, P, P, P, P, P, i32, P, P, P, P], i32),
        "pv_set_kernel_timing": ([P, i32], i32),
        "pv_kernel_times": ([P, P, P], i32),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


def _dev_f32(t, n, cols, name, device):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.device != device:
        raise ValueError(f"{name} is on {t.device}, expected {device}")
    if t.dtype != torch.float32:
        raise TypeError(f"{name} must be float32")
    shape = (n, cols) if cols else (n,)
    if tuple(t.shape) != shape:
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {shape}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


class Cells:
    """A pv_cells handle (library-owned device memory)."""

    def __init__(self, ctx: "Context", handle, n: int, nbox: int):
        self.ctx = ctx
        self.handle = handle
        self.n = n
        self.nbox = nbox
        self.sorted = False

    def info(self):
        g = (C.c_int * 3)()
        nc = C.c_int64()
        occ = C.c_int32()
        hm = C.c_float()
        nb = C.c_int()
        n = C.c_int64()
        self.ctx._call("pv_cells_info", self.handle, g, C.byref(nc), C.byref(occ), C.byref(hm),
                       C.byref(nb), C.byref(n))
        return dict(grid=tuple(g), ncell=nc.value, max_occupancy=occ.value, hmax=hm.value,
                    nbox=nb.value, n=n.value)

    def export(self):
        """(cell_start, order, sorted) device tensors describing the layout."""
        info = self.info()
        dev = self.ctx.device
        cs = torch.empty(info["ncell"] + 1, dtype=torch.int32, device=dev)
        order = torch.empty(self.n, dtype=torch.int32, device=dev)
        srt = torch.empty((13, self.n), dtype=torch.int16, device=dev) if self.sorted else None
        self.ctx._sync_stream()
        self.ctx._call("pv_cells_export", self.handle, _ptr(cs), _ptr(order), _ptr(srt))
        return cs, order, srt

    def free(self):
        if self.handle is not None and self.ctx.handle is not None:
            load_library().pv_free_cells(self.ctx.handle, self.handle)
        self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Context:
    """A pv_ctx bound to one GPU; calls are issued on torch's current stream."""

    def __init__(self, device: Optional[int] = None):
        lib = load_library()
        if device is None:
            device = torch.cuda.current_device()
        self.device = torch.device("cuda", device)
        h = C.c_void_p()
        st = lib.pv_create(device, C.c_void_p(torch.cuda.current_stream(self.device).cuda_stream),
                           C.byref(h))
        if st != PV_OK:
            raise PVError(st, f"pv_create(device={device}) failed")
        self.handle = h

    # -- plumbing --------------------------------------------------------
    def _sync_stream(self):
        s = torch.cuda.current_stream(self.device).cuda_stream
        load_library().pv_set_stream(self.handle, C.c_void_p(s))

    def _call(self, name, *args):
        st = getattr(load_library(), name)(self.handle, *args)
        if st != PV_OK:
            msg = load_library().pv_last_error(self.handle)
            raise PVError(st, (msg or b"").decode())

    def close(self):
        if getattr(self, "handle", None) is not None:
            load_library().pv_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- entry points ----------------------------------------------------
    def build_cells(self, pos, h, mass, box=(1.0, 1.0, 1.0), grid=None,
                    cells: Optional[Cells] = None) -> Cells:
        n = int(pos.shape[0])
        _dev_f32(pos, n, 3, "pos", self.device)
        _dev_f32(h, n, 0, "h", self.device)
        _dev_f32(mass, n, 0, "mass", self.device)
        return self.build_cells_batched([0, n], pos, h, mass, [box], None if grid is None else [grid],
                                        cells)

    def build_cells_batched(self, offsets: Sequence[int], pos, h, mass, boxes, grids=None,
                            cells: Optional[Cells] = None) -> Cells:
        nbox = len(offsets) - 1
        n = int(offsets[-1])
        _dev_f32(pos, n, 3, "pos", self.device)
        _dev_f32(h, n, 0, "h", self.device)
        _dev_f32(mass, n, 0, "mass", self.device)
        off = (C.c_int64 * (nbox + 1))(*[int(x) for x in offsets])
        bx = []
        for b in boxes:
            bx.extend([float(b)] * 3 if isinstance(b, (int, float)) else [float(x) for x in b])
        if len(bx) != 3 * nbox:
            raise ValueError("boxes must give 3 edges per box")
        barr = (C.c_double * (3 * nbox))(*bx)
        garr = None
        if grids is not None:
            gl = []
            for g in grids:
                gl.extend([int(g)] * 3 if isinstance(g, (int,)) else [int(x) for x in g])
            if len(gl) != 3 * nbox:
                raise ValueError("grids must give 3 counts per box")
            garr = (C.c_int * (3 * nbox))(*gl)
        handle = C.c_void_p(cells.handle.value if cells is not None else None)
        self._sync_stream()
        self._call("pv_build_cells_batched", nbox, off, _ptr(pos), _ptr(h), _ptr(mass), barr,
                   garr, C.byref(handle))
        if cells is not None:
            cells.handle = handle
            cells.n = n
            cells.nbox = nbox
            cells.sorted = False
            return cells
        return Cells(self, handle, n, nbox)

    def sort_cells(self, cells: Cells) -> None:
        self._sync_stream()
        self._call("pv_sort_cells", cells.handle)
        cells.sorted = True

    def density(self, cells: Cells, algo: str = "sorted", out=None):
        """(rho, wcount, drho_dh, ncount) in original particle order."""
        n = cells.n
        if out is None:
            rho = torch.empty(n, dtype=torch.float32, device=self.device)
            wc = torch.empty_like(rho)
            dh = torch.empty_like(rho)
            nc = torch.empty(n, dtype=torch.int32, device=self.device)
        else:
            rho, wc, dh, nc = out
        self._sync_stream()
        self._call("pv_density", cells.handle, ALGOS[algo], _ptr(rho), _ptr(wc), _ptr(dh), _ptr(nc))
        return rho, wc, dh, nc

    def density_static(self, pos, h, mass, box, grid, algo: str = "sorted", out=None):
        """(rho, wcount, drho_dh, ncount) of one box by pv_density_static: build,
        sort and sweep in one call that allocates no device memory (the cells
        live in the library's static scratch; n <= PV_STATIC_MAX_N, an explicit
        grid of at most PV_STATIC_MAX_CELLS cells).  Output tensors are
        allocated here unless given in `out`."""
        n = int(pos.shape[0])
        _dev_f32(pos, n, 3, "pos", self.device)
        _dev_f32(h, n, 0, "h", self.device)
        _dev_f32(mass, n, 0, "mass", self.device)
        if out is None:
            rho = torch.empty(n, dtype=torch.float32, device=self.device)
            wc = torch.empty_like(rho)
            dh = torch.empty_like(rho)
            nc = torch.empty(n, dtype=torch.int32, device=self.device)
        else:
            rho, wc, dh, nc = out
        bx = [float(box)] * 3 if isinstance(box, (int, float)) else [float(x) for x in box]
        gl = [int(grid)] * 3 if isinstance(grid, int) else [int(x) for x in grid]
        self._sync_stream()
        self._call("pv_density_static", n, _ptr(pos), _ptr(h), _ptr(mass),
                   (C.c_double * 3)(*bx), (C.c_int * 3)(*gl), ALGOS[algo], _ptr(rho), _ptr(wc),
                   _ptr(dh), _ptr(nc))
        return rho, wc, dh, nc

    def autotune_grid(self, pos, h, mass, box=(1.0, 1.0, 1.0), reps: int = 3, offsets=None,
                      boxes=None):
        """Fastest cells-per-axis for build + sort + density (pv_autotune_grid):
        returns (grids, ms at the finest grid, ms at the chosen one); grids is
        one (gx, gy, gz) per box."""
        n = int(pos.shape[0])
        _dev_f32(pos, n, 3, "pos", self.device)
        _dev_f32(h, n, 0, "h", self.device)
        _dev_f32(mass, n, 0, "mass", self.device)
        if offsets is None:
            offsets, boxes = [0, n], [box]
        nbox = len(offsets) - 1
        off = (C.c_int64 * (nbox + 1))(*[int(x) for x in offsets])
        bx = []
        for b in boxes:
            bx.extend([float(b)] * 3 if isinstance(b, (int, float)) else [float(x) for x in b])
        barr = (C.c_double * (3 * nbox))(*bx)
        g = (C.c_int * (3 * nbox))()
        t = (C.c_float * 2)()
        self._sync_stream()
        self._call("pv_autotune_grid", nbox, off, _ptr(pos), _ptr(h), _ptr(mass), barr,
                   int(reps), g, t)
        grids = [tuple(g[3 * b:3 * b + 3]) for b in range(nbox)]
        return grids, float(t[0]), float(t[1])

    def lj(self, cells: Cells, eps: float, sigma: float, out=None):
        """Lennard-Jones (force (n, 3), energy (n,)) over each particle's
        cut-off (pv_lj)."""
        n = cells.n
        if out is None:
            f = torch.empty((n, 3), dtype=torch.float32, device=self.device)
            e = torch.empty(n, dtype=torch.float32, device=self.device)
        else:
            f, e = out
        self._sync_stream()
        self._call("pv_lj", cells.handle, float(eps), float(sigma), _ptr(f), _ptr(e))
        return f, e

    def set_kernel_timing(self, enable: bool) -> None:
        """Record HIP events around every persistent sweep kernel launch
        (pv_set_kernel_timing); clears the record."""
        self._sync_stream()
        self._call("pv_set_kernel_timing", 1 if enable else 0)

    def kernel_times(self, count: int = PV_KTIME_RING):
        """Durations (ms) of the most recent timed sweep kernel launches, oldest
        first (pv_kernel_times; synchronises the stream)."""
        ms = (C.c_float * max(1, count))()
        k = C.c_int(count)
        self._sync_stream()
        self._call("pv_kernel_times", ms, C.byref(k))
        return [float(ms[i]) for i in range(k.value)]

    def drift(self, cells: Cells, disp) -> None:
        """Move the cells' particles by disp (n x 3, input order) keeping the
        sorted lists (pv_drift)."""
        _dev_f32(disp, cells.n, 3, "disp", self.device)
        self._sync_stream()
        self._call("pv_drift", cells.handle, _ptr(disp))

    def density_backward(self, cells: Cells, grad_rho, out=None):
        n = cells.n
        _dev_f32(grad_rho, n, 0, "grad_rho", self.device)
        if out is None:
            gp = torch.empty((n, 3), dtype=torch.float32, device=self.device)
            gh = torch.empty(n, dtype=torch.float32, device=self.device)
        else:
            gp, gh = out
        self._sync_stream()
        self._call("pv_density_backward", cells.handle, _ptr(grad_rho), _ptr(gp), _ptr(gh))
        return gp, gh

    def solve_h(self, pos, mass, h, box=(1.0, 1.0, 1.0), ngb: float = 48.0, tol: float = 1e-6,
                max_iter: int = 30, offsets=None, boxes=None):
        """Solve rho_i(h_i) h_i^3 = m_i eta^3 (eta from the weighted neighbour
        number ngb) in place in h (pv_solve_h).  One box, or several with
        offsets/boxes as in build_cells_batched.  Returns (iterations, largest
        relative residual)."""
        n = int(pos.shape[0])
        _dev_f32(pos, n, 3, "pos", self.device)
        _dev_f32(mass, n, 0, "mass", self.device)
        _dev_f32(h, n, 0, "h", self.device)
        if offsets is None:
            offsets, boxes = [0, n], [box]
        nbox = len(offsets) - 1
        off = (C.c_int64 * (nbox + 1))(*[int(x) for x in offsets])
        bx = []
        for b in boxes:
            bx.extend([float(b)] * 3 if isinstance(b, (int, float)) else [float(x) for x in b])
        barr = (C.c_double * (3 * nbox))(*bx)
        it = C.c_int()
        res = C.c_float()
        self._sync_stream()
        self._call("pv_solve_h", nbox, off, _ptr(pos), _ptr(mass), _ptr(h), barr, float(ngb),
                   float(tol), int(max_iter), C.byref(it), C.byref(res))
        return it.value, res.value

    def check(self) -> None:
        self._sync_stream()
        self._call("pv_check")

    def set_param(self, name: str, value: int, sweep: str = "density") -> None:
        """Tuning parameter (see pv_param in include/pvl.h) of one sweep:
        "density" (sorted pair), "adjoint" or "plain"."""
        self._call("pv_set_param", PARAMS[name] + _SET_OFFSET[sweep], int(value))

    def get_param(self, name: str, sweep: str = "density") -> int:
        v = C.c_int()
        self._call("pv_get_param", PARAMS[name] + _SET_OFFSET[sweep], C.byref(v))
        return v.value

    def params(self, sweep: str = "density") -> dict:
        return {k: self.get_param(k, sweep) for k in PARAMS}

    def autotune(self, cells: Cells, target: str = "density", grad_rho=None, reps: int = 3,
                 cache: Optional["TuneCache"] = None):
        """Pick the fastest parameters of one sweep ("density", "adjoint" or
        "plain") for these cells (pv_autotune).  Returns (ms before, ms after,
        chosen parameters).  With a cache, parameters already tuned for the
        same device architecture and size class (see tune_key) are applied
        without timing (both times are then NaN), and new results are stored."""
        if target == "adjoint":
            _dev_f32(grad_rho, cells.n, 0, "grad_rho", self.device)
        key = None
        if cache is not None:
            info = cells.info()
            arch = torch.cuda.get_device_properties(self.device).gcnArchName
            key = tune_key(arch, target, info["n"], info["ncell"], info["nbox"])
            hit = cache.get(key)
            if hit is not None:
                for name, v in hit.items():
                    self.set_param(name, v, target)
                return float("nan"), float("nan"), self.params(target)
        t = (C.c_float * 2)()
        self._sync_stream()
        self._call("pv_autotune", cells.handle, TUNE_TARGETS[target],
                   _ptr(grad_rho) if target == "adjoint" else None, int(reps), t)
        chosen = self.params(target)
        if cache is not None:
            cache.put(key, chosen)
        return float(t[0]), float(t[1]), chosen

    def set_census(self, on: bool) -> None:
        self._call("pv_set_census", 1 if on else 0)

    def census(self):
        """(pairs tested under the exact per-receiver bounds, pairs in range,
        pair slots of the tiled sweep) of the last density call made with the
        census on."""
        v = (C.c_int64 * 3)()
        self._sync_stream()
        self._call("pv_census", v)
        return int(v[0]), int(v[1]), int(v[2])


def tune_key(arch: str, target: str, n: int, ncell: int, nbox: int) -> str:
    """Size class of a tuned sweep: the device architecture, the sweep, the
    particle count and the particles per cell, each to the nearest power of
    two (the tuned settings follow the work per item and the items per
    workgroup), and whether the structure holds one box or several."""
    def p2(x: float) -> int:
        return int(round(math.log2(x))) if x > 0 else -1
    return f"{arch}|{target}|n{p2(n)}|ppc{p2(n / max(ncell, 1))}|{'one' if nbox == 1 else 'many'}"


class TuneCache:
    """Tuned sweep parameters kept in a JSON file across processes, keyed by
    tune_key.  Entries hold the parameter names of PARAMS and their values;
    the file is rewritten whole on every store."""

    def __init__(self, path: str):
        self.path = path
        self._data = {}
        if os.path.exists(path):
            with open(path) as f:
                self._data = json.load(f)

    def get(self, key: str):
        v = self._data.get(key)
        if v is None or set(v) - set(PARAMS):
            return None
        return {k: int(x) for k, x in v.items()}

    def put(self, key: str, params: dict) -> None:
        self._data[key] = {k: int(v) for k, v in params.items() if k in PARAMS}
        tmp = f"{self.path}.tmp{os.getpid()}"
        with open(tmp, "w") as f:
            json.dump(self._data, f, indent=1, sort_keys=True)
        os.replace(tmp, self.path)


_contexts = {}


def context(device: Optional[int] = None) -> Context:
    """Process-wide context for a device (created on first use)."""
    if device is None:
        device = torch.cuda.current_device()
    if device not in _contexts:
        _contexts[device] = Context(device)
    return _contexts[device]


# -- high-level, differentiable ------------------------------------------------
class _DensityFn(torch.autograd.Function):
    @staticmethod
    def forward(fctx, pos, h, mass, box, grid, algo):
        ctx = context(pos.device.index)
        cells = ctx.build_cells(pos.detach(), h.detach(), mass.detach(), box, grid)
        if algo == "sorted" or pos.requires_grad or h.requires_grad:
            ctx.sort_cells(cells)
        rho, wc, dh, nc = ctx.density(cells, algo)
        # device-detected errors (a cut-off above the cell edge of an explicit
        # grid, a crowded cell) raise here rather than leave the context's
        # error word set for later calls
        ctx.check()
        fctx.cells = cells
        fctx.mark_non_differentiable(wc, dh, nc)
        return rho, wc, dh, nc

    @staticmethod
    def backward(fctx, g_rho, g_wc, g_dh, g_nc):
        cells = fctx.cells
        ctx = cells.ctx
        if g_rho is None:
            return None, None, None, None, None, None
        gp, gh = ctx.density_backward(cells, g_rho.contiguous().float())
        ctx.check()
        need_p, need_h = fctx.needs_input_grad[0], fctx.needs_input_grad[1]
        return (gp if need_p else None), (gh if need_h else None), None, None, None, None


def density(pos, mass, h, box=(1.0, 1.0, 1.0), algo: str = "sorted", grid=None):
    """SPH density of every particle: (rho, wcount, drho_dh, ncount).

    Differentiable in pos and h through rho (the adjoint runs in the library);
    wcount, drho_dh and ncount carry no gradient."""
    if algo not in ALGOS:
        raise ValueError(f"algo must be one of {sorted(ALGOS)}")
    return _DensityFn.apply(pos, h, mass, tuple(box) if not isinstance(box, (int, float)) else (box,) * 3,
                            grid, algo)
