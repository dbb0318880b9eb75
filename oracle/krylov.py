"""The other Krylov methods the paper compares with FGMRES, each with the same
multigrid preconditioner (Sec. 5.3, Table t1): GMRES, CG, FCG, CGS and
BiCGSTAB.  Test infrastructure only: the product path never imports or
calls this module.

The paper names the methods and cites a textbook for them without giving
their steps; these are the textbook forms:

* GMRES(m), right-preconditioned: Arnoldi on A M, and at the end of a cycle
  x = x0 + M (V_m y_m) with y_m the least-squares solution (the same
  recurrences as Algorithm 1 with one fixed M; only the update differs).
* CG, preconditioned: the standard preconditioned conjugate gradient
  recurrence.  Its optimality assumes a fixed symmetric positive definite
  M.  The default V-cycle is not symmetric (its mean-of-8 restriction is not
  a multiple of the transpose of its trilinear prolongation; a test shows
  M != M^T), so with it CG is only a heuristic; the V-cycle built with the
  option ``restriction="transpose"`` (R = P^T / 8, equal pre- and
  post-smoothing counts) is symmetric.
* FCG: flexible CG with truncation to one previous direction (Notay's
  flexible CG): the new direction is z made A-orthogonal to the last one,
  p = z - ((z, A p_old) / (p_old, A p_old)) p_old.  With a fixed symmetric
  positive definite M it equals CG in exact arithmetic.
* CGS and BiCGSTAB, right-preconditioned: the usual recurrences with M
  applied to the search directions (two preconditioner and two operator
  applications per iteration).  BiCGSTAB stops half-way through an
  iteration when the intermediate residual s already meets the tolerance
  (its second half would divide 0 by 0).

Readings: the stopping test is the relative residual of eq. criterion on
the recursively updated residual, confirmed on the true residual b - A x;
if that fails the method restarts from x (as FGMRES does at the end of a
cycle).  Iterations count the methods' own iterations; ``precond`` counts
preconditioner applications.  ``M`` may be any callable; the comparison
uses the V-cycle from zero for every method.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class KrylovResult:
    x: np.ndarray
    iterations: int
    precond: int
    converged: bool
    true_relres: float
    res_hist: list


def _finish(A, b, x, bnorm):
    return np.linalg.norm(b - A(x)) / bnorm


def gmres(A, b, M, x0=None, tol=1e-8, restart=10, max_iter=200, breakdown_tol=1e-14):
    """Right-preconditioned GMRES(m)."""
    b = np.asarray(b, dtype=np.float64)
    bnorm = np.linalg.norm(b)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    it = nprec = 0
    hist = []
    if bnorm == 0.0:
        return KrylovResult(np.zeros_like(b), 0, 0, True, 0.0, [0.0])
    while True:
        r0 = b - A(x)
        beta = np.linalg.norm(r0)
        if not hist:
            hist.append(beta / bnorm)
        if beta < tol * bnorm or it >= max_iter:
            return KrylovResult(x, it, nprec, beta < tol * bnorm, beta / bnorm, hist)
        V = [r0 / beta]
        H = np.zeros((restart + 1, restart))
        e1 = np.zeros(restart + 1)
        e1[0] = beta
        k = 0
        y = np.zeros(0)
        for j in range(restart):
            if it >= max_iter:
                break
            w = A(M(V[j]))
            nprec += 1
            for i in range(j + 1):
                H[i, j] = np.vdot(w, V[i])
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            breakdown = H[j + 1, j] <= breakdown_tol * np.linalg.norm(H[: j + 2, j])
            if not breakdown:
                V.append(w / H[j + 1, j])
            it += 1
            k = j + 1
            y, *_ = np.linalg.lstsq(H[: j + 2, : j + 1], e1[: j + 2], rcond=None)
            r_j = np.linalg.norm(e1[: j + 2] - H[: j + 2, : j + 1] @ y)
            hist.append(r_j / bnorm)
            if r_j < tol * bnorm or breakdown:
                break
        if k > 0:
            u = np.zeros_like(b)
            for i in range(k):
                u = u + y[i] * V[i]
            x = x + M(u)
            nprec += 1


def cg(A, b, M, x0=None, tol=1e-8, max_iter=200, flexible=False):
    """Preconditioned CG; flexible=True gives FCG (one-direction truncation)."""
    b = np.asarray(b, dtype=np.float64)
    bnorm = np.linalg.norm(b)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    it = nprec = 0
    hist = []
    if bnorm == 0.0:
        return KrylovResult(np.zeros_like(b), 0, 0, True, 0.0, [0.0])
    while True:
        r = b - A(x)
        rn = np.linalg.norm(r)
        if not hist:
            hist.append(rn / bnorm)
        if rn < tol * bnorm or it >= max_iter:
            return KrylovResult(x, it, nprec, rn < tol * bnorm, rn / bnorm, hist)
        z = M(r)
        nprec += 1
        p = z.copy()
        rho = np.vdot(r, z)
        while it < max_iter:
            q = A(p)
            alpha = rho / np.vdot(p, q)
            x = x + alpha * p
            r = r - alpha * q
            it += 1
            rn = np.linalg.norm(r)
            hist.append(rn / bnorm)
            if rn < tol * bnorm:
                break
            z = M(r)
            nprec += 1
            rho_new = np.vdot(r, z)
            if flexible:
                beta = -np.vdot(z, q) / np.vdot(p, q)
            else:
                beta = rho_new / rho
            p = z + beta * p
            rho = rho_new
        # confirm on the true residual (the loop head), restart if needed


def cgs(A, b, M, x0=None, tol=1e-8, max_iter=200):
    """Right-preconditioned conjugate gradient squared."""
    b = np.asarray(b, dtype=np.float64)
    bnorm = np.linalg.norm(b)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    it = nprec = 0
    hist = []
    if bnorm == 0.0:
        return KrylovResult(np.zeros_like(b), 0, 0, True, 0.0, [0.0])
    while True:
        r = b - A(x)
        rn = np.linalg.norm(r)
        if not hist:
            hist.append(rn / bnorm)
        if rn < tol * bnorm or it >= max_iter:
            return KrylovResult(x, it, nprec, rn < tol * bnorm, rn / bnorm, hist)
        rs = r.copy()  # shadow residual
        rho = np.vdot(r, rs)
        p = r.copy()
        u = r.copy()
        while it < max_iter:
            ph = M(p)
            vh = A(ph)
            alpha = rho / np.vdot(vh, rs)
            q = u - alpha * vh
            uh = M(u + q)
            nprec += 2
            x = x + alpha * uh
            r = r - alpha * A(uh)
            it += 1
            rn = np.linalg.norm(r)
            hist.append(rn / bnorm)
            if rn < tol * bnorm:
                break
            rho_new = np.vdot(r, rs)
            beta = rho_new / rho
            u = r + beta * q
            p = u + beta * q + beta * beta * p
            rho = rho_new


def bicgstab(A, b, M, x0=None, tol=1e-8, max_iter=200):
    """Right-preconditioned BiCGSTAB."""
    b = np.asarray(b, dtype=np.float64)
    bnorm = np.linalg.norm(b)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    it = nprec = 0
    hist = []
    if bnorm == 0.0:
        return KrylovResult(np.zeros_like(b), 0, 0, True, 0.0, [0.0])
    while True:
        r = b - A(x)
        rn = np.linalg.norm(r)
        if not hist:
            hist.append(rn / bnorm)
        if rn < tol * bnorm or it >= max_iter:
            return KrylovResult(x, it, nprec, rn < tol * bnorm, rn / bnorm, hist)
        rs = r.copy()
        rho = alpha = omega = 1.0
        v = np.zeros_like(b)
        p = np.zeros_like(b)
        while it < max_iter:
            rho_new = np.vdot(rs, r)
            beta = (rho_new / rho) * (alpha / omega)
            p = r + beta * (p - omega * v)
            ph = M(p)
            v = A(ph)
            alpha = rho_new / np.vdot(rs, v)
            s = r - alpha * v
            nprec += 1
            if np.linalg.norm(s) < tol * bnorm:  # converged half-way: x from p alone
                x = x + alpha * ph
                r = s
                it += 1
                hist.append(np.linalg.norm(r) / bnorm)
                break
            sh = M(s)
            t = A(sh)
            nprec += 1
            omega = np.vdot(t, s) / np.vdot(t, t)
            x = x + alpha * ph + omega * sh
            r = s - omega * t
            rho = rho_new
            it += 1
            rn = np.linalg.norm(r)
            hist.append(rn / bnorm)
            if rn < tol * bnorm:
                break
