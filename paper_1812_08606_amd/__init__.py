"""MI355X (gfx950) geometric-multigrid-preconditioned FGMRES solver for the
variable-coefficient Poisson-type equation -div(a grad phi) = f of the
semi-implicit streamer scheme (eq. e18; Algorithm 1; Sec. 3.2).

The solve runs in the HIP library ``libgmg.so`` behind the C ABI of
``include/gmg.h``; this package only marshals arguments.  Importing it
without the built library raises ImportError.
"""
from . import _lib

_lib.load()

from .solver import (  # noqa: E402,F401
    FP64,
    MIXED,
    GMGError,
    GMGPoisson,
    SemiImplicitStepper,
    SolveResult,
    StepInfo,
    fgmres_solve_static,
    poisson_solve,
)
