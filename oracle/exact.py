"""Exact references that pin the oracle independently of its iteration.

* ``spectral_solve``: for constant a the operator of e18 separates; along z
  (mirrored-ghost Dirichlet plates) it is diagonalised by the DST-II basis
  sin(pi p (k+1/2)/N), p = 1..N, along x and y (Neumann sides) by the DCT-II
  basis cos(pi p (i+1/2)/N), p = 0..N-1, with 1-D eigenvalues
  4 a sin^2(pi p / (2N)) / h^2.  The orthonormal transforms of scipy.fft give
  the exact discrete solution.
* ``sparse_solve``: sparse direct solve (SuperLU) of the assembled matrix.
* ``manufactured``: a smooth solution meeting both boundary conditions and
  its analytic source, for the second-order convergence check.
"""
from __future__ import annotations

import numpy as np
import scipy.fft as sfft
import scipy.sparse.linalg as spla

from .operator import assemble_sparse, rhs


def spectral_eigenvalues(shape_zyx, h, a0=1.0):
    nz, ny, nx = shape_zyx
    hx, hy, hz = h
    px = np.arange(nx)
    py = np.arange(ny)
    pz = np.arange(1, nz + 1)
    lx = 4.0 * a0 * np.sin(np.pi * px / (2 * nx)) ** 2 / hx ** 2
    ly = 4.0 * a0 * np.sin(np.pi * py / (2 * ny)) ** 2 / hy ** 2
    lz = 4.0 * a0 * np.sin(np.pi * pz / (2 * nz)) ** 2 / hz ** 2
    return lz[:, None, None] + ly[None, :, None] + lx[None, None, :]


def spectral_solve(b, h, a0=1.0):
    """Exact solution of A phi = b for the constant coefficient a0."""
    lam = spectral_eigenvalues(b.shape, h, a0)
    bh = sfft.dct(b, type=2, axis=2, norm="ortho")
    bh = sfft.dct(bh, type=2, axis=1, norm="ortho")
    bh = sfft.dst(bh, type=2, axis=0, norm="ortho")
    ph = bh / lam
    ph = sfft.idst(ph, type=2, axis=0, norm="ortho")
    ph = sfft.idct(ph, type=2, axis=1, norm="ortho")
    ph = sfft.idct(ph, type=2, axis=2, norm="ortho")
    return ph


def sparse_solve(a, f, h, phi_bot=0.0, phi_top=0.0):
    """Exact discrete solution of e18 by a sparse direct solve."""
    A = assemble_sparse(a, h).tocsc()
    b = rhs(f, a, h, phi_bot, phi_top)
    return spla.spsolve(A, b.ravel()).reshape(a.shape)


def manufactured(n, phi_top=1.0):
    """phi = phi_top z + cos(pi x) cos(pi y) sin(pi z),
    a = 1 + cos(pi x) cos(pi y) cos(pi z) / 2, f = -div(a grad phi),
    sampled at the cell centres of an n^3 grid on the unit cube.
    phi meets phi(z=0) = 0, phi(z=1) = phi_top and d phi/dn = 0 on the sides;
    a has zero normal derivative on every face."""
    c = (np.arange(n) + 0.5) / n
    z, y, x = np.meshgrid(c, c, c, indexing="ij")
    pi = np.pi
    cx, sx = np.cos(pi * x), np.sin(pi * x)
    cy, sy = np.cos(pi * y), np.sin(pi * y)
    cz, sz = np.cos(pi * z), np.sin(pi * z)
    phi = phi_top * z + cx * cy * sz
    a = 1.0 + 0.5 * cx * cy * cz
    # gradients
    px, py, pz = -pi * sx * cy * sz, -pi * cx * sy * sz, phi_top + pi * cx * cy * cz
    ax, ay, az = -0.5 * pi * sx * cy * cz, -0.5 * pi * cx * sy * cz, -0.5 * pi * cx * cy * sz
    lap = -3.0 * pi ** 2 * cx * cy * sz
    f = -(a * lap + ax * px + ay * py + az * pz)
    return phi, a, f
