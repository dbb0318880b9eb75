"""Finite-volume operator of eq. e18 (Sec. 2.2) with the boundary conditions
of Sec. 1.

Grid: M_x x M_y x M_z uniform cells, spacing (hx, hy, hz) (Sec. 2.2).  Arrays
are (nz, ny, nx), x fastest.

Discrete operator, per cell c (eq. e18, with P -> a):

    (A phi)_c = sum over the faces of c of  w_f (phi_c - phi_nb) / h_d^2

where the face coefficient is the arithmetic mean of the two cells it
separates, w_f = (a_c + a_nb) / 2 (Sec. 2.2, definition of P_{i+1/2,j,k}).

Boundary readings (the paper states the conditions, Sec. 1, but not how the
cell-centred scheme imposes them):

* x and y sides, homogeneous Neumann: ghost value equals the cell value, so
  the side faces carry no flux;
* plates z=0 and z=1, Dirichlet phi_b: a ghost cell mirrored through the
  plate, phi_g = 2 phi_b - phi_c, with the face coefficient equal to the cell's
  own a_c (the coefficient itself has homogeneous Neumann ghosts, inherited
  from n_e and n_p, Sec. 1).  The plate face adds 2 a_c (phi_c - phi_b)/hz^2.

The linear system solved is A phi = b with A the operator above for phi_b = 0
(homogeneous) and b = f + lifting, lifting = 2 a_c phi_b / hz^2 on the first
and last z-layers.

The operator is stored by its face coefficients (``Faces``), so that the
coarse multigrid levels, whose coefficients live on faces, use the same code.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp


@dataclass
class Faces:
    """Face coefficients of one grid.

    wx[k,j,i]: face between cells i and i+1     (nz, ny, nx-1)
    wy[k,j,i]: face between cells j and j+1     (nz, ny-1, nx)
    wz[k,j,i]: face between layers k and k+1    (nz-1, ny, nx)
    bot[j,i], top[j,i]: plate faces of the first and last layers (ny, nx)."""

    wx: np.ndarray
    wy: np.ndarray
    wz: np.ndarray
    bot: np.ndarray
    top: np.ndarray

    def astype(self, dtype):
        return Faces(*(np.asarray(w, dtype=dtype) for w in
                       (self.wx, self.wy, self.wz, self.bot, self.top)))


def face_coefficients(a):
    """Faces of e18: w = (a_c + a_nb)/2 on interior faces, a_c on the plates."""
    return Faces(wx=0.5 * (a[:, :, 1:] + a[:, :, :-1]),
                 wy=0.5 * (a[:, 1:, :] + a[:, :-1, :]),
                 wz=0.5 * (a[1:, :, :] + a[:-1, :, :]),
                 bot=a[0].copy(), top=a[-1].copy())


def apply_faces(x, F: Faces, h):
    """Homogeneous operator A x (plate values 0) from face coefficients."""
    hx, hy, hz = h
    y = np.zeros_like(x)
    # flux through each interior face, w (x_nb - x_c) / h^2 seen from the
    # lower cell: it enters the lower cell with a minus sign and the upper
    # cell with a plus sign (the two terms of e18 for that direction).
    fx = F.wx * (x[:, :, 1:] - x[:, :, :-1]) / (hx * hx)
    y[:, :, :-1] -= fx
    y[:, :, 1:] += fx
    fy = F.wy * (x[:, 1:, :] - x[:, :-1, :]) / (hy * hy)
    y[:, :-1, :] -= fy
    y[:, 1:, :] += fy
    fz = F.wz * (x[1:, :, :] - x[:-1, :, :]) / (hz * hz)
    y[:-1, :, :] -= fz
    y[1:, :, :] += fz
    # plates: mirrored ghost -x_c, so the face term is w (x_c + x_c) / hz^2
    y[0] += 2.0 * F.bot * x[0] / (hz * hz)
    y[-1] += 2.0 * F.top * x[-1] / (hz * hz)
    return y


def lifting(a, h, phi_bot, phi_top):
    """Plate contributions moved to the right side: b - f."""
    hz = h[2]
    out = np.zeros_like(a)
    out[0] += 2.0 * a[0] * phi_bot / (hz * hz)
    out[-1] += 2.0 * a[-1] * phi_top / (hz * hz)
    return out


def apply_operator(x, a, h, phi_bot=0.0, phi_top=0.0):
    """Left side of eq. e18 evaluated on the cell values ``x`` with plate
    values ``phi_bot`` (z=0) and ``phi_top`` (z=1): A x - lifting.

    With phi_bot = phi_top = 0 this is the linear operator A; with the true
    plate values, apply_operator(phi) = f is the discrete problem itself."""
    y = apply_faces(x, face_coefficients(a), h)
    if phi_bot != 0.0 or phi_top != 0.0:
        y = y - lifting(a, h, phi_bot, phi_top)
    return y


def rhs(f, a, h, phi_bot, phi_top):
    """b = f + lifting: the right side of A phi = b."""
    return f + lifting(a, h, phi_bot, phi_top)


def diagonal(F: Faces, h):
    """Diagonal of A: sum of w_f / h_d^2 over the interior faces of each cell
    plus 2 w_plate / hz^2 for each plate face."""
    hx, hy, hz = h
    nz = F.wz.shape[0] + 1
    ny, nx = F.bot.shape
    d = np.zeros((nz, ny, nx), dtype=F.bot.dtype)
    d[:, :, :-1] += F.wx / (hx * hx)
    d[:, :, 1:] += F.wx / (hx * hx)
    d[:, :-1, :] += F.wy / (hy * hy)
    d[:, 1:, :] += F.wy / (hy * hy)
    d[:-1, :, :] += F.wz / (hz * hz)
    d[1:, :, :] += F.wz / (hz * hz)
    d[0] += 2.0 * F.bot / (hz * hz)
    d[-1] += 2.0 * F.top / (hz * hz)
    return d


def assemble_dense(F: Faces, h):
    """Dense matrix of A, column by column: A e_c for every unit vector e_c.

    Brute force, for small grids only (it applies the operator n times)."""
    shape = (F.wz.shape[0] + 1,) + F.bot.shape
    n = int(np.prod(shape))
    M = np.zeros((n, n), dtype=F.bot.dtype)
    e = np.zeros(shape, dtype=F.bot.dtype)
    for c in range(n):
        e.flat[c] = 1.0
        M[:, c] = apply_faces(e, F, h).ravel()
        e.flat[c] = 0.0
    return M


def assemble_sparse(a, h):
    """Sparse CSR matrix of A built face by face from the e18 stencil (cell
    index c = (k ny + j) nx + i).  Independent of ``apply_faces``; used for
    sparse direct reference solves on moderate grids."""
    nz, ny, nx = a.shape
    hx, hy, hz = h
    n = a.size
    idx = np.arange(n).reshape(a.shape)
    rows, cols, vals = [], [], []
    diag = np.zeros(n)
    for axis, hd in ((2, hx), (1, hy), (0, hz)):
        m = a.shape[axis]
        lo = np.take(idx, np.arange(m - 1), axis=axis).ravel()
        hi = np.take(idx, np.arange(1, m), axis=axis).ravel()
        c = 0.5 * (a.ravel()[lo] + a.ravel()[hi]) / (hd * hd)
        rows += [lo, hi]
        cols += [hi, lo]
        vals += [-c, -c]
        np.add.at(diag, lo, c)
        np.add.at(diag, hi, c)
    diag[idx[0].ravel()] += (2.0 * a[0] / (hz * hz)).ravel()
    diag[idx[-1].ravel()] += (2.0 * a[-1] / (hz * hz)).ravel()
    rows.append(np.arange(n))
    cols.append(np.arange(n))
    vals.append(diag)
    return sp.csr_matrix((np.concatenate(vals),
                          (np.concatenate(rows), np.concatenate(cols))),
                         shape=(n, n))
