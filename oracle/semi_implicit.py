"""Elliptic side of one semi-implicit step, and the time step around it.
Test infrastructure only: the product path never imports or calls this
module.

The coefficient and right side of the variable-coefficient elliptic problem
that each time step solves (Sec. 2.1, eq. semi2 for the predictor of the
second-order scheme, eq. e15 for the first-order one; discretised in Sec.
2.2, eq. e18), and the electric field from its solution:

* coefficient ``P = eps0/e + tau_eff (mu_p n_p + mu_e n_e)`` per cell (the
  definition of P^n in Sec. 2.2), with ``tau_eff = tau/2`` in eq. semi2 and
  ``tau`` in eq. e15;
* right side ``n_p - n_e - tau_eff sum_d D_d / h_d^2 delta_d^2 n_e`` (the
  right side of eq. e18), ``delta_d^2`` the second central difference;
* ``E = -grad phi`` by central differences (Sec. 2.2, after eq. e18) and
  ``|E|``.

Readings of points the paper leaves open:

* Ghost cells of n_e: homogeneous Neumann on every boundary (Sec. 1 states
  that condition for n_e), i.e. the ghost equals the boundary cell, so the
  second difference at a boundary cell is one-sided.
* Ghost cells of phi for E: the same as the operator's (``oracle.operator``):
  mirrored through the plates, ``2 phi_b - phi_c``, equal to the boundary
  cell on the sides.

``time_step`` sequences one step of either scheme around the elliptic solve
(Sec. 2.1).  The transport operator -- drift, diffusion and source of the
density equations, discretised in the paper by MUSCL fluxes with the Koren
limiter -- is not part of the solver: the caller passes it as a function
``transport(n_e, n_p, E) -> (L_e, L_p)`` giving the time derivatives of the
two densities for a frozen field E = (E_x, E_y, E_z, |E|), so that each
density equation of eqs. e1, e2 and semi-implicit reads
``(n_new - n_base) / dt = L(n_eval, E)``.

* Second order (eqs. e1, e2, semi2): the elliptic problem with
  tau_eff = tau/2 from the densities at t_n gives phi^{n+1/2} and E^{n+1/2};
  the predictor n^{n+1/2} = n^n + tau/2 L(n^n, E^{n+1/2}) (eq. e1); the
  corrector n^{n+1} = n^n + tau L(n^{n+1/2}, E^{n+1/2}) (eq. e2), reusing
  E^{n+1/2}: one elliptic solve per step.
* First order (eqs. semi-implicit, e15): tau_eff = tau gives phi^{n+1},
  E^{n+1}; n^{n+1} = n^n + tau L(n^n, E^{n+1}).

The solve is warm-started from the previous step's phi when one is given
(Sec. 3.2), cold (full multigrid cycles) otherwise.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


def coefficient(n_e, n_p, eps0_over_e, tau_eff, mu_e, mu_p):
    """P = eps0/e + tau_eff (mu_p n_p + mu_e n_e), cell by cell."""
    n_e = np.asarray(n_e, dtype=np.float64)
    n_p = np.asarray(n_p, dtype=np.float64)
    return eps0_over_e + tau_eff * (mu_p * n_p + mu_e * n_e)


def second_difference(u, axis):
    """delta^2 u along ``axis`` with ghost cells equal to the boundary cells."""
    u = np.asarray(u, dtype=np.float64)
    lo = np.concatenate([np.take(u, [0], axis=axis), np.take(u, np.arange(u.shape[axis] - 1), axis=axis)],
                        axis=axis)
    hi = np.concatenate([np.take(u, np.arange(1, u.shape[axis]), axis=axis),
                         np.take(u, [u.shape[axis] - 1], axis=axis)], axis=axis)
    return hi - 2.0 * u + lo


def right_side(n_e, n_p, h, tau_eff, De):
    """n_p - n_e - tau_eff (D_x/hx^2 dxx n_e + D_y/hy^2 dyy n_e + D_z/hz^2 dzz n_e).

    Arrays are (nz, ny, nx); h = (hx, hy, hz), De = (D_x, D_y, D_z)."""
    n_e = np.asarray(n_e, dtype=np.float64)
    n_p = np.asarray(n_p, dtype=np.float64)
    hx, hy, hz = h
    dx, dy, dz = De
    diff = (dx / hx ** 2 * second_difference(n_e, 2) + dy / hy ** 2 * second_difference(n_e, 1)
            + dz / hz ** 2 * second_difference(n_e, 0))
    return n_p - n_e - tau_eff * diff


def electric_field(phi, h, phi_bot, phi_top):
    """(E_x, E_y, E_z, |E|) with E = -grad phi by central differences."""
    phi = np.asarray(phi, dtype=np.float64)
    hx, hy, hz = h
    # x and y: ghosts equal to the boundary cells
    px = np.concatenate([phi[:, :, :1], phi, phi[:, :, -1:]], axis=2)
    py = np.concatenate([phi[:, :1, :], phi, phi[:, -1:, :]], axis=1)
    # z: ghosts mirrored through the plates
    pz = np.concatenate([2.0 * phi_bot - phi[:1], phi, 2.0 * phi_top - phi[-1:]], axis=0)
    ex = -(px[:, :, 2:] - px[:, :, :-2]) / (2.0 * hx)
    ey = -(py[:, 2:, :] - py[:, :-2, :]) / (2.0 * hy)
    ez = -(pz[2:] - pz[:-2]) / (2.0 * hz)
    return ex, ey, ez, np.sqrt(ex * ex + ey * ey + ez * ez)


@dataclass
class StepParams:
    eps0_over_e: float
    mu_e: float
    mu_p: float
    De: tuple  # (D_x, D_y, D_z)


@dataclass
class StepResult:
    n_e: np.ndarray
    n_p: np.ndarray
    phi: np.ndarray  # phi^{n+1/2} (second order) or phi^{n+1} (first order)
    E: tuple  # the field of phi: (E_x, E_y, E_z, |E|)
    iterations: int


def time_step(n_e, n_p, h, prm: StepParams, tau, transport, phi_bot, phi_top, phi_prev=None,
              scheme="second", tol=1e-8, **solve_kw):
    """One time step of the second-order scheme (eqs. e1, e2 with the
    elliptic problem semi2) or of the first-order one (eqs. semi-implicit,
    e15).  solve_kw go to ``oracle.fgmres.solve_poisson``."""
    from .fgmres import solve_poisson

    if scheme not in ("second", "first"):
        raise ValueError("scheme must be 'second' or 'first'")
    n_e = np.asarray(n_e, dtype=np.float64)
    n_p = np.asarray(n_p, dtype=np.float64)
    tau_eff = 0.5 * tau if scheme == "second" else tau
    a = coefficient(n_e, n_p, prm.eps0_over_e, tau_eff, prm.mu_e, prm.mu_p)
    f = right_side(n_e, n_p, h, tau_eff, prm.De)
    sol = solve_poisson(a, f, h, phi_bot, phi_top, tol=tol, x0=phi_prev, **solve_kw)
    E = electric_field(sol.x, h, phi_bot, phi_top)
    le, lp = transport(n_e, n_p, E)
    if scheme == "first":
        return StepResult(n_e + tau * le, n_p + tau * lp, sol.x, E, sol.iterations)
    ne_h, np_h = n_e + 0.5 * tau * le, n_p + 0.5 * tau * lp  # predictor (eq. e1)
    le, lp = transport(ne_h, np_h, E)
    return StepResult(n_e + tau * le, n_p + tau * lp, sol.x, E, sol.iterations)  # corrector (eq. e2)
