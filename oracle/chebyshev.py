"""The paper's own smoother, evaluated on the oracle only: a degree-2
Chebyshev polynomial preconditioned by one symmetric SSOR step (Sec. 3.2,
eq. qntn), with the eigenvalue bounds taken from 10 Arnoldi steps.  Test
infrastructure only: the product path never imports or calls this module
(the GPU path keeps red-black symmetric Gauss-Seidel, which needed fewer
FGMRES steps at half the smoothing cost on the workloads measured).

Readings of points the paper leaves open:

* "Quadratic polynomial": the smoother's error polynomial q_{n+1} of eq.
  qntn has degree 2 (two Chebyshev steps), the usual meaning of a degree-2
  Chebyshev smoother.
* The Chebyshev iteration is preconditioned by SSOR, so the polynomial acts
  on M^{-1} A_l (M the SSOR matrix) and the bounds of eq. qntn are those of
  M^{-1} A_l: lambda_max = 1.1 and lambda* = 0.1 times the largest Ritz value
  of the 10-step Arnoldi process applied to M^{-1} A_l (the paper's "Arnoldi
  without preconditioning" read as Algorithm 1 with z_j = v_j on the
  smoother's operator).  The Arnoldi start vector is an input.
* SSOR with relaxation factor 1 in its data-parallel red-black form: one
  symmetric sweep from zero, red, black, red (the forward sweep red-black
  followed by the backward sweep black-red; the repeated black half-sweep
  does nothing).
"""
from __future__ import annotations

import numpy as np

from .multigrid import Hierarchy, Level, coarse_solve, prolong, rbgs_half_sweep, restrict
from .operator import apply_faces


def ssor(lev: Level, r):
    """z = M^{-1} r: one symmetric red-black Gauss-Seidel sweep from zero."""
    z = np.zeros_like(r)
    rbgs_half_sweep(z, r, lev, 0)
    rbgs_half_sweep(z, r, lev, 1)
    rbgs_half_sweep(z, r, lev, 0)
    return z


def lambda_max_estimate(lev: Level, v0, m=10):
    """Largest real part of the Ritz values of m Arnoldi steps on M^{-1} A."""
    V = [np.asarray(v0, dtype=np.float64) / np.linalg.norm(v0)]
    H = np.zeros((m + 1, m))
    for j in range(m):
        w = ssor(lev, apply_faces(V[j], lev.faces, lev.h))
        for i in range(j + 1):
            H[i, j] = np.vdot(w, V[i])
            w = w - H[i, j] * V[i]
        H[j + 1, j] = np.linalg.norm(w)
        if H[j + 1, j] == 0.0:
            m = j + 1
            break
        V.append(w / H[j + 1, j])
    return float(np.linalg.eigvals(H[:m, :m]).real.max())


def chebyshev_smooth(x, b, lev: Level, lam_max, lam_star, steps=2):
    """x <- x + p(M^{-1} A) M^{-1} (b - A x) with error polynomial
    q(t) = T_steps((lam_max + lam_star - 2t)/(lam_max - lam_star)) /
           T_steps((lam_max + lam_star)/(lam_max - lam_star))   (eq. qntn),
    by the three-term Chebyshev recurrence."""
    theta = 0.5 * (lam_max + lam_star)
    delta = 0.5 * (lam_max - lam_star)
    sigma = theta / delta
    x = np.array(x, dtype=np.float64)
    z = ssor(lev, b - apply_faces(x, lev.faces, lev.h))
    d = z / theta
    x = x + d
    rho_prev = 1.0 / sigma
    for _ in range(steps - 1):
        z = ssor(lev, b - apply_faces(x, lev.faces, lev.h))
        rho = 1.0 / (2.0 * sigma - rho_prev)
        d = rho * rho_prev * d + (2.0 * rho / delta) * z
        x = x + d
        rho_prev = rho
    return x


def level_bounds(hier: Hierarchy, seed=0, m=10):
    """(lambda*, lambda_max) per smoothed level: 0.1 and 1.1 times the
    Arnoldi estimate, from a seeded uniform start vector."""
    rng = np.random.default_rng(seed)
    out = []
    for lev in hier.levels[:-1]:
        nx, ny, nz = lev.shape
        lam = lambda_max_estimate(lev, rng.uniform(-1.0, 1.0, (nz, ny, nx)), m)
        out.append((0.1 * lam, 1.1 * lam))
    return out


def vcycle_chebyshev(hier: Hierarchy, bounds, b, level=0, steps=2):
    """V-cycle from zero with the Chebyshev smoother before and after the
    coarse correction (same transfers and coarse solve as the V-cycle of
    ``oracle.multigrid``)."""
    lev = hier.levels[level]
    b = np.asarray(b, dtype=np.float64)
    if level == len(hier.levels) - 1:
        return coarse_solve(hier, b)
    lam_star, lam_max = bounds[level]
    x = chebyshev_smooth(np.zeros_like(b), b, lev, lam_max, lam_star, steps)
    r = b - apply_faces(x, lev.faces, lev.h)
    x = x + prolong(vcycle_chebyshev(hier, bounds, restrict(r), level + 1, steps))
    return chebyshev_smooth(x, b, lev, lam_max, lam_star, steps)
