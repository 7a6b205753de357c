"""FP64 CPU oracle for the pseudo-Verlet SPH density loop.

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
bench's CPU-baseline leg.  The GPU library (paper_1804_06231_amd) never imports
it, and it never imports the GPU library.

  cell_list  -- plain cell-list brute force in C (pv_oracle.c), fp64, OpenMP;
                also the per-particle bisection solve of rho h^3 = m eta^3
  allpairs   -- O(N^2) numpy brute force for tiny inputs (pins the cell list)
  census     -- candidate census of the sorted-projection pruning (pins the
                paper's in-range fractions)
"""
from .cell_list import (Oracle, build_oracle_lib, kernel_w, density_fp64,  # noqa: F401
                        grad_fp64, solve_h_fp64, eta_for_neighbours, ORACLE_GAMMA)
