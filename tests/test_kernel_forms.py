"""CPU checks of the algebraic forms the GPU sweep evaluates in place of the
textbook cubic spline, against the oracle's spline (fp64).  The equal-mass
density step accumulates four cubic sums and combines them per receiver, which
is exact only if, with v = 1 - u and s = max(0, 1 - 2u),
    w(u) = 2 v^3 - s^3        and        u w'(u) = 6 u (s^2 - v^2)
on the whole support 0 <= u < 1; the general step uses t = min(0, 1 - 2u) with
    w(u) = 1 - 6u^2 + 6u^3 + t^3   and   u w'(u) = 18u^3 - 12u^2 - 6u t^2."""
import numpy as np

from oracle.cell_list import kernel_w


def _grid():
    # both pieces, the knot at 1/2 and the edge of the support
    u = np.concatenate([np.linspace(0.0, 0.999999, 4001), [0.5, np.nextafter(0.5, 0), 0.25, 0.75]])
    return u


def test_cubic_sum_form_matches_spline():
    for u in _grid():
        w, dw = kernel_w(u)
        v = 1.0 - u
        s = max(0.0, 1.0 - 2.0 * u)
        assert abs((2.0 * v ** 3 - s ** 3) - w) < 1e-12, u
        assert abs(6.0 * u * (s * s - v * v) - u * dw) < 1e-12, u


def test_select_free_form_matches_spline():
    for u in _grid():
        w, dw = kernel_w(u)
        t = min(0.0, 1.0 - 2.0 * u)
        # the sweep forms t as -clamp(2u - 1, 0, 1) and s as clamp(1 - 2u, 0, 1)
        assert t == -min(1.0, max(0.0, 2.0 * u - 1.0)), u
        assert max(0.0, 1.0 - 2.0 * u) == min(1.0, max(0.0, 1.0 - 2.0 * u)), u
        assert abs((1.0 - 6.0 * u * u + 6.0 * u ** 3 + t ** 3) - w) < 1e-12, u
        assert abs((18.0 * u ** 3 - 12.0 * u * u - 6.0 * u * t * t) - u * dw) < 1e-12, u


def test_cubic_sums_combine_to_the_density_sums():
    """Sums over random pairs: the per-receiver combination of the four sums
    equals the direct sums of w and u w'."""
    rng = np.random.Generator(np.random.PCG64(5))
    u = rng.random(2000) * 0.999
    v = 1.0 - u
    s = np.maximum(0.0, 1.0 - 2.0 * u)
    sw = sum(kernel_w(x)[0] for x in u)
    sdw = sum(x * kernel_w(x)[1] for x in u)
    assert abs((2.0 * np.sum(v ** 3) - np.sum(s ** 3)) - sw) < 1e-9 * abs(sw)
    assert abs(6.0 * (np.sum(u * s * s) - np.sum(u * v * v)) - sdw) < 1e-9 * abs(sdw)
