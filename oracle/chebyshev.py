"""The paper's own smoother: a degree-2 Chebyshev polynomial preconditioned
by one symmetric SSOR step (Sec. 3.2, eq. qntn), with the eigenvalue bounds
taken from 10 Arnoldi steps.  Test infrastructure only: the product path
never imports or calls this module.

Readings of points the paper leaves open:

* "Quadratic polynomial": the smoother's error polynomial q_{n+1} of eq.
  qntn has degree 2 (two Chebyshev steps), the usual meaning of a degree-2
  Chebyshev smoother.  One application before and one after the coarse
  correction (``nu`` repeats it).
* The Chebyshev iteration is preconditioned by SSOR, so the polynomial acts
  on M^{-1} A_l (M the SSOR matrix) and the bounds of eq. qntn are those of
  M^{-1} A_l: lambda_max = 1.1 and lambda* = 0.1 times the largest real part
  of the Ritz values of the 10-step Arnoldi process applied to M^{-1} A_l
  (the paper's "Arnoldi without preconditioning" read as Algorithm 1 with
  z_j = v_j on the smoother's operator).
* The Arnoldi start vector is random; the paper does not say how it is
  drawn.  Here it comes from SplitMix64 (Steele, Lea and Flood 2014, with
  the output function of Vigna's reference version), a counter-based
  generator, so that any implementation can draw the same vector: cell c
  (natural index) of level l takes output c + 1 of the generator seeded with
  seed + l, mapped to [-1, 1) as 2 (z >> 11) 2^-53 - 1.
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


_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_MIX1 = np.uint64(0xBF58476D1CE4E5B9)
_MIX2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed, k):
    """Output k (k >= 1, an array) of SplitMix64 seeded with ``seed``: the
    state after k steps is seed + k * gamma (mod 2^64), passed through the
    output mix."""
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + np.asarray(k, dtype=np.uint64) * _GAMMA
        z = (z ^ (z >> np.uint64(30))) * _MIX1
        z = (z ^ (z >> np.uint64(27))) * _MIX2
    return z ^ (z >> np.uint64(31))


def start_vector(shape_zyx, seed):
    """Arnoldi start vector: cell c (natural index) = 2 (z >> 11) 2^-53 - 1
    with z = output c + 1 of SplitMix64 seeded with ``seed``."""
    n = int(np.prod(shape_zyx))
    z = splitmix64(seed, np.arange(1, n + 1, dtype=np.uint64))
    u = (z >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    return (2.0 * u - 1.0).reshape(shape_zyx)


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
    """(lambda*, lambda_max) per smoothed level l: 0.1 and 1.1 times the
    Arnoldi estimate from ``start_vector(level shape, seed + l)``."""
    out = []
    for li, lev in enumerate(hier.levels[:-1]):
        nx, ny, nz = lev.shape
        lam = lambda_max_estimate(lev, start_vector((nz, ny, nx), seed + li), m)
        out.append((0.1 * lam, 1.1 * lam))
    return out


def vcycle_chebyshev(hier: Hierarchy, bounds, b, level=0, steps=2, nu=1):
    """V-cycle from zero with ``nu`` applications of the Chebyshev smoother
    before and after the coarse correction (same transfers and coarse solve
    as the V-cycle of ``oracle.multigrid``)."""
    lev = hier.levels[level]
    b = np.asarray(b, dtype=np.float64)
    if level == len(hier.levels) - 1:
        return coarse_solve(hier, b)
    lam_star, lam_max = bounds[level]
    x = np.zeros_like(b)
    for _ in range(nu):
        x = chebyshev_smooth(x, b, lev, lam_max, lam_star, steps)
    r = b - apply_faces(x, lev.faces, lev.h)
    x = x + prolong(vcycle_chebyshev(hier, bounds, restrict(r), level + 1, steps, nu))
    for _ in range(nu):
        x = chebyshev_smooth(x, b, lev, lam_max, lam_star, steps)
    return x
