"""ctypes front end of the C cell-list oracle (pv_oracle.c).

TEST INFRASTRUCTURE ONLY (see the package docstring).  The shared object is
built with gcc into oracle/_build/ by build_oracle_lib(), which the repository's
build entry point also calls.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pv_oracle.c")
_OUT = os.path.join(_HERE, "_build", "liboracle.so")
_lib = None

ORACLE_GAMMA = 1.825742


def build_oracle_lib(force: bool = True) -> str:
    os.makedirs(os.path.dirname(_OUT), exist_ok=True)
    if force or not os.path.exists(_OUT) or os.path.getmtime(_OUT) < os.path.getmtime(_SRC):
        tmp = _OUT + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _OUT)
    return _OUT


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_OUT) or os.path.getmtime(_OUT) < os.path.getmtime(_SRC):
        build_oracle_lib(force=True)
    lib = C.CDLL(_OUT)
    P = C.c_void_p
    i64 = C.c_int64
    lib.or_kernel.argtypes = [C.c_double, C.POINTER(C.c_double), C.POINTER(C.c_double)]
    lib.or_kernel.restype = None
    lib.or_gamma.restype = C.c_double
    lib.or_grid_build.argtypes = [i64, P, P, P, P, P]
    lib.or_grid_build.restype = P
    lib.or_grid_free.argtypes = [P]
    lib.or_density.argtypes = [P, P, i64, P, P, P, P, P]
    lib.or_density_grad.argtypes = [P, P, P, i64, P, P, P, P]
    lib.or_fd_loss.argtypes = [P, P, i64, C.c_int, C.c_double]
    lib.or_fd_loss.restype = C.c_double
    lib.or_fd_loss_many.argtypes = [P, P, P, P, P, i64, P]
    lib.or_solve_h.argtypes = [P, C.c_double, P, P]
    lib.or_solve_h.restype = i64
    lib.or_lj.argtypes = [P, C.c_double, C.c_double, P, i64, P, P, P, P]
    lib.or_lj.restype = None
    lib.or_lj_energy_moved.argtypes = [P, C.c_double, C.c_double, i64, C.c_int, C.c_double]
    lib.or_lj_energy_moved.restype = C.c_double
    _lib = lib
    return lib


def kernel_w(u: float):
    """(w(u), w'(u)) of the oracle's cubic spline."""
    lib = _load()
    w = C.c_double()
    dw = C.c_double()
    lib.or_kernel(float(u), C.byref(w), C.byref(dw))
    return w.value, dw.value


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


class Oracle:
    """Cell list over fp64 copies of (pos, h, m).  grid=None picks the finest
    legal cells-per-side floor(L / H_max) on each axis."""

    def __init__(self, pos, h, m, box=(1.0, 1.0, 1.0), grid=None):
        self.lib = _load()
        self.x = np.ascontiguousarray(np.asarray(pos, dtype=np.float64).reshape(-1, 3))
        self.h = np.ascontiguousarray(np.asarray(h, dtype=np.float64))
        self.m = np.ascontiguousarray(np.asarray(m, dtype=np.float64))
        self.n = self.x.shape[0]
        self.L = np.ascontiguousarray(np.asarray(box, dtype=np.float64).reshape(3))
        Hmax = ORACLE_GAMMA * float(self.h.max()) if self.n else 0.0
        if grid is None:
            g = [max(3, int(math.floor(self.L[a] / Hmax))) if Hmax > 0 else 3 for a in range(3)]
            g = [min(x, 512) for x in g]
        elif np.isscalar(grid):
            g = [int(grid)] * 3
        else:
            g = [int(x) for x in grid]
        self.g = np.ascontiguousarray(np.asarray(g, dtype=np.int32))
        self.handle = self.lib.or_grid_build(self.n, _ptr(self.x), _ptr(self.h), _ptr(self.m),
                                             _ptr(self.L), _ptr(self.g))
        if not self.handle:
            raise ValueError(f"oracle: illegal grid {g} for H_max={Hmax}")

    def __del__(self):
        if getattr(self, "handle", None):
            self.lib.or_grid_free(self.handle)
            self.handle = None

    def density(self, recv=None):
        """dict of rho, wcount, drho_dh, ncount, dh_abs (fp64 / int64)."""
        if recv is None:
            k = self.n
            r = None
        else:
            r = np.ascontiguousarray(np.asarray(recv, dtype=np.int64))
            k = r.size
        out = {n: np.zeros(k) for n in ("rho", "wcount", "drho_dh", "dh_abs")}
        out["ncount"] = np.zeros(k, dtype=np.int64)
        self.lib.or_density(self.handle, _ptr(r), k, _ptr(out["rho"]), _ptr(out["wcount"]),
                            _ptr(out["drho_dh"]), _ptr(out["ncount"]), _ptr(out["dh_abs"]))
        return out

    def grad(self, G, recv=None):
        """Adjoint of rho for upstream dL/drho = G: dict of gx (k,3), gh, gx_abs, gh_abs."""
        G = np.ascontiguousarray(np.asarray(G, dtype=np.float64))
        if recv is None:
            k = self.n
            r = None
        else:
            r = np.ascontiguousarray(np.asarray(recv, dtype=np.int64))
            k = r.size
        out = {"gx": np.zeros((k, 3)), "gh": np.zeros(k), "gx_abs": np.zeros((k, 3)),
               "gh_abs": np.zeros(k)}
        self.lib.or_density_grad(self.handle, _ptr(G), _ptr(r), k, _ptr(out["gx"]),
                                 _ptr(out["gh"]), _ptr(out["gx_abs"]), _ptr(out["gh_abs"]))
        return out

    def lj(self, eps, sigma, recv=None):
        """Lennard-Jones force (k, 3), energy (k,) and the |term| sums f_abs
        (k, 3) and e_abs (k,) over pairs within each receiver's cut-off."""
        if recv is None:
            k, r = self.n, None
        else:
            r = np.ascontiguousarray(np.asarray(recv, dtype=np.int64))
            k = r.size
        out = {"force": np.zeros((k, 3)), "energy": np.zeros(k), "f_abs": np.zeros((k, 3)),
               "e_abs": np.zeros(k)}
        self.lib.or_lj(self.handle, float(eps), float(sigma), _ptr(r), k, _ptr(out["force"]),
                       _ptr(out["energy"]), _ptr(out["f_abs"]), _ptr(out["e_abs"]))
        return out

    def lj_energy_moved(self, eps, sigma, k, comp, delta):
        """Total Lennard-Jones energy with particle k's coordinate comp moved by delta."""
        return self.lib.or_lj_energy_moved(self.handle, float(eps), float(sigma), int(k),
                                           int(comp), float(delta))

    def fd_loss(self, target, ks, comps, eps):
        """Central differences of L = sum (rho - target)^2 for each (k, comp, eps)."""
        t = np.ascontiguousarray(np.asarray(target, dtype=np.float64))
        ks = np.ascontiguousarray(np.asarray(ks, dtype=np.int64))
        comps = np.ascontiguousarray(np.asarray(comps, dtype=np.int32))
        eps = np.ascontiguousarray(np.broadcast_to(np.asarray(eps, dtype=np.float64), ks.shape))
        out = np.zeros(ks.size)
        self.lib.or_fd_loss_many(self.handle, _ptr(t), _ptr(ks), _ptr(comps), _ptr(eps),
                                 ks.size, _ptr(out))
        return out


def solve_h_fp64(pos, m, h_lo, h_hi, eta, box=(1.0, 1.0, 1.0)):
    """Per-particle root of rho_i(h) h^3 = m_i eta^3 by fp64 bisection on
    [h_lo_i, h_hi_i] (pv_oracle.c: or_solve_h).  Raises if a bracket holds no
    root."""
    n = np.asarray(pos).reshape(-1, 3).shape[0]
    hi = np.broadcast_to(np.asarray(h_hi, dtype=np.float64), (n,))
    o = Oracle(pos, hi, m, box)
    lo = np.ascontiguousarray(np.broadcast_to(np.asarray(h_lo, dtype=np.float64), (n,)))
    out = np.zeros(o.n)
    bad = o.lib.or_solve_h(o.handle, float(eta), _ptr(lo), _ptr(out))
    if bad:
        raise ValueError(f"oracle: {bad} brackets hold no root")
    return out


def eta_for_neighbours(ngb: float) -> float:
    """eta with rho h^3 = m eta^3 equivalent to (4 pi / 3) H^3 wcount = ngb for
    equal masses: eta^3 = 3 ngb / (4 pi gamma^3)."""
    return (3.0 * ngb / (4.0 * math.pi * ORACLE_GAMMA ** 3)) ** (1.0 / 3.0)


def density_fp64(pos, h, m, box=(1.0, 1.0, 1.0), grid=None, recv=None):
    return Oracle(pos, h, m, box, grid).density(recv)


def grad_fp64(pos, h, m, G, box=(1.0, 1.0, 1.0), grid=None, recv=None):
    return Oracle(pos, h, m, box, grid).grad(G, recv)
