"""CPU oracle for the GMG-preconditioned FGMRES Poisson solve.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link this package: only the test-suite, the smoke check and the benchmark's
CPU-baseline leg use it.  It shares no code with the HIP library.

A plain, slow, FP64 (or, for the mixed-precision preconditioner, FP32) NumPy
implementation of what the paper computes, written step by step from the
paper:

* ``operator``  -- the finite-volume operator of eq. e18 (Sec. 2.2) with the
  plate and side boundary conditions of Sec. 1, and its right-side lifting;
* ``multigrid`` -- the level hierarchy, red-black Gauss-Seidel smoother,
  transfers, direct coarse solve, the zero-guess V-cycle and the full
  multigrid cycle used as preconditioners (Sec. 3.2, Appendix A);
* ``fgmres``    -- FGMRES(m) of Algorithm 1 (Sec. 3.1) with the stopping rule
  of eq. criterion (Sec. 5.2);
* ``adjoint``   -- gradient of a loss through the solve (derived from e18);
* ``semi_implicit`` -- coefficient and right side of the elliptic problem of
  a semi-implicit step, and E = -grad phi (Sec. 2.1-2.2);
* ``krylov``    -- the other Krylov methods of the comparison in Sec. 5.3
  (GMRES, CG, FCG, CGS, BiCGSTAB) with any preconditioner;
* ``chebyshev`` -- the paper's Chebyshev(2)+SSOR smoother (Sec. 3.2, eq.
  qntn), its Arnoldi bound estimate and the V-cycle that uses it;
* ``exact``     -- independent exact references (spectral DCT/DST solve for
  constant a, sparse direct solve, manufactured solution) used to pin the
  pieces above.

Every reading of a point the paper leaves open is named in the docstring of
the function that takes it.
"""
from .operator import (  # noqa: F401
    face_coefficients,
    apply_operator,
    lifting,
    rhs,
    diagonal,
    assemble_dense,
    assemble_sparse,
)
from .multigrid import (  # noqa: F401
    level_shapes,
    build_hierarchy,
    coarsen_faces,
    rbgs_half_sweep,
    restrict,
    restrict_transpose,
    prolong,
    vcycle,
    Hierarchy,
)
from .fgmres import fgmres, FGMRESResult  # noqa: F401
from .adjoint import coefficient_gradient, solve_and_gradient  # noqa: F401
