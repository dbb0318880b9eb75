"""FGMRES(m) with a V-cycle preconditioner: Algorithm 1 of Sec. 3.1, the
preconditioner application of Sec. 3.2 and the stopping rule of eq. criterion
(Sec. 5.2).

Readings of points the paper leaves open:

* Least squares (Algorithm 1, step "compute the residual"): only
  min_y || beta e_1 - Hbar_j y || is stated; the oracle solves it with a
  library least-squares routine on the unrotated Hessenberg matrix and takes
  the residual norm of that solution as the estimate r_j.
* Stopping: relative to ||b|| of the lifted right side (eq. criterion uses
  the full right side), tested on the estimate r_j inside a cycle; when a
  cycle ends, the true residual b - A x is recomputed (it is the next cycle's
  r_0) and decides convergence, otherwise the method restarts from x.
* Happy breakdown (not discussed): when h_{j+1,j} <= 1e-14 ||Hbar(:, j)||,
  v_{j+1} is not formed and the cycle ends after step j.
* Iterations are Arnoldi steps (preconditioner applications), counted across
  restarts; ``max_iter`` caps them.  With tol = 0 exactly ``max_iter`` steps
  run, which is how results are compared at a fixed step count.
* b = 0 returns phi = 0 after 0 steps (the criterion is undefined there).
* Residual history: entry 0 is ||r_0|| / ||b|| of the first cycle, then one
  estimate r_j / ||b|| per Arnoldi step.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .multigrid import build_hierarchy, fmg, vcycle
from .operator import apply_operator, rhs


@dataclass
class FGMRESResult:
    x: np.ndarray
    iterations: int
    converged: bool
    res_hist: list
    true_relres: float
    restarts: int
    # last cycle's bases, kept for checks of the Arnoldi relation
    V: list = field(default_factory=list)
    Z: list = field(default_factory=list)
    Hbar: np.ndarray | None = None


def fgmres(A, b, M, x0=None, tol=1e-8, restart=10, max_iter=200,
           breakdown_tol=1e-14):
    """Solve A x = b with right-preconditioned flexible GMRES(m).

    ``A(x)`` and ``M(v)`` are callables (M may change from call to call: the
    flexibility of Algorithm 1)."""
    b = np.asarray(b, dtype=np.float64)
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return FGMRESResult(x=np.zeros_like(b), iterations=0, converged=True,
                            res_hist=[0.0], true_relres=0.0, restarts=0)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    m = restart
    it = 0
    hist = []
    cycles = 0
    V, Z, Hbar = [], [], None
    while True:
        # step 2: r_0 = b - A x_0, beta = ||r_0||, v_1 = r_0 / beta
        r0 = b - A(x)
        beta = np.linalg.norm(r0)
        if not hist:
            hist.append(beta / bnorm)
        if beta < tol * bnorm:
            return FGMRESResult(x=x, iterations=it, converged=True,
                                res_hist=hist, true_relres=beta / bnorm,
                                restarts=max(cycles - 1, 0), V=V, Z=Z, Hbar=Hbar)
        if it >= max_iter:
            return FGMRESResult(x=x, iterations=it, converged=False,
                                res_hist=hist, true_relres=beta / bnorm,
                                restarts=max(cycles - 1, 0), V=V, Z=Z, Hbar=Hbar)
        cycles += 1
        V = [r0 / beta]
        Z = []
        Hbar = np.zeros((m + 1, m))
        e1 = np.zeros(m + 1)
        e1[0] = beta
        k = 0
        y = np.zeros(0)
        for j in range(m):
            if it >= max_iter:
                break
            z = M(V[j])  # preconditioning, z_j = M_j v_j
            Z.append(z)
            w = A(z)  # omega = A z_j
            for i in range(j + 1):  # modified Gram-Schmidt
                Hbar[i, j] = np.vdot(w, V[i])
                w = w - Hbar[i, j] * V[i]
            Hbar[j + 1, j] = np.linalg.norm(w)
            breakdown = Hbar[j + 1, j] <= breakdown_tol * np.linalg.norm(Hbar[: j + 2, j])
            if not breakdown:
                V.append(w / Hbar[j + 1, j])
            it += 1
            k = j + 1
            # r_j = min_y || beta e_1 - Hbar_j y ||, Hbar_j the (j+1) x j block
            Hj = Hbar[: j + 2, : j + 1]
            y, *_ = np.linalg.lstsq(Hj, e1[: j + 2], rcond=None)
            r_j = np.linalg.norm(e1[: j + 2] - Hj @ y)
            hist.append(r_j / bnorm)
            if r_j < tol * bnorm or breakdown:
                break
        # step 3: x_k = x_0 + Z_k y_k
        for i in range(k):
            x = x + y[i] * Z[i]
        # step 4: restart from x_k (the loop head re-checks the true residual)


def solve_poisson(a, f, h, phi_bot=0.0, phi_top=1.0, tol=1e-8, restart=10,
                  max_iter=200, nu_pre=2, nu_post=2, precision="fp64",
                  x0=None, coarse_max_cells=4096, cold="fmg", warm="vcycle",
                  restriction="mean"):
    """FGMRES(restart) with one multigrid cycle per step on A phi = f +
    lifting.

    The cycle of a solve without an initial guess (x0 None) is the full
    multigrid cycle when cold = "fmg", of a warm-started one when warm =
    "fmg", and a V-cycle otherwise (Sec. 3.2: FMG on the first time step,
    which starts from zero, V-cycles on the later, warm-started ones; the
    defaults).  The preconditioner acts on the Krylov vectors, so either
    cycle serves a warm start: it only changes M.

    precision "fp64": the whole cycle in float64;
    precision "mixed": the cycle (coefficients, smoother, transfers, coarse
    solve) in float32, its input v_j rounded to float32 and its output
    promoted exactly to float64; everything else in float64."""
    dtype = {"fp64": np.float64, "mixed": np.float32}[precision]
    if cold not in ("vcycle", "fmg") or warm not in ("vcycle", "fmg"):
        raise ValueError("cold and warm must be 'vcycle' or 'fmg'")
    hier = build_hierarchy(a, h, nu_pre=nu_pre, nu_post=nu_post,
                           coarse_max_cells=coarse_max_cells, dtype=dtype,
                           restriction=restriction)
    b = rhs(f, a, h, phi_bot, phi_top)
    cycle = fmg if (cold if x0 is None else warm) == "fmg" else vcycle

    def A(x):
        return apply_operator(x, a, h)

    def M(v):
        return cycle(hier, v.astype(dtype)).astype(np.float64)

    return fgmres(A, b, M, x0=x0, tol=tol, restart=restart, max_iter=max_iter)
