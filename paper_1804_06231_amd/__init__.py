"""pseudo-Verlet (sorted cell-pair) SPH density loop on AMD gfx950.

The computation lives in the HIP library libpvl.so (C ABI in include/pvl.h);
this package is its thin Python binding:

    from paper_1804_06231_amd import density, Context
    rho, wcount, drho_dh, ncount = density(pos, mass, h, box=(1, 1, 1))

Nothing here computes densities on the CPU; without the built library the
calls raise.
"""
from .pvl import (Cells, Context, PVError, context, density, load_library,  # noqa: F401
                  ALGOS, PV_MAX_CELL, PV_MAX_GRID, EXPORTS, LIB_PATH, PV_OK, PV_EINVAL,
                  PV_ENOMEM, PV_EHIP, PV_EGRID, PV_EOVERFLOW, PV_ESTATE, PV_STATIC_MAX_N,
                  PV_STATIC_MAX_CELLS)

__all__ = ["Cells", "Context", "PVError", "context", "density", "load_library"]
