"""Gradient of a loss L(phi) through the solve of eq. e18.

With A(a) phi = b(f, a) (b = f + plate lifting) and A symmetric, the adjoint
lambda solves A lambda = dL/dphi with homogeneous plate values, and

    dL/df = lambda,
    dL/da = lambda^T db/da - lambda^T (dA/da) phi
          = - d/da [ lambda^T (A phi - lifting) ].

lambda^T (A phi - lifting) is a sum over faces of  w_f (d lambda)_f (d phi)_f
with (d u)_f the one-sided difference quotient across the face: for an
interior face (u_nb - u_c)/h_d with w_f = (a_c + a_nb)/2, for a plate face the
half-cell quotient (u_c - u_b)/(h_z/2) with w_f = a_c and the factor 1/2 that
the mirrored ghost brings.  Differentiating each face term gives, for every
cell c,

    dL/da_c = -1/2 * sum over the faces of c of (d phi)_f (d lambda)_f

(Neumann side faces carry no term).  This is derived from e18 and the
boundary readings of ``oracle.operator``; it is checked against finite
differences and a dense autograd solve in the tests.
"""
from __future__ import annotations

import numpy as np

from .fgmres import solve_poisson


def coefficient_gradient(phi, lam, h, phi_bot, phi_top):
    hx, hy, hz = h
    g = np.zeros_like(phi)
    for axis, hd in ((2, hx), (1, hy), (0, hz)):
        n = phi.shape[axis]
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        lo[axis] = slice(0, n - 1)
        hi[axis] = slice(1, n)
        lo, hi = tuple(lo), tuple(hi)
        dphi = (phi[hi] - phi[lo]) / hd
        dlam = (lam[hi] - lam[lo]) / hd
        t = 0.5 * dphi * dlam
        g[lo] -= t
        g[hi] -= t
    half = 0.5 * hz
    g[0] -= 0.5 * ((phi[0] - phi_bot) / half) * (lam[0] / half)
    g[-1] -= 0.5 * ((phi[-1] - phi_top) / half) * (lam[-1] / half)
    return g


def solve_and_gradient(a, f, h, phi_bot, phi_top, dL_dphi, tol=1e-8, **kw):
    """Forward solve, adjoint solve and both gradients.

    Returns (phi, dL/df, dL/da, forward result, adjoint result)."""
    fwd = solve_poisson(a, f, h, phi_bot, phi_top, tol=tol, **kw)
    adj = solve_poisson(a, dL_dphi, h, 0.0, 0.0, tol=tol, **kw)
    lam = adj.x
    return fwd.x, lam, coefficient_gradient(fwd.x, lam, h, phi_bot, phi_top), fwd, adj
