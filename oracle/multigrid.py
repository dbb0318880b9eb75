"""Geometric multigrid V-cycle used as the FGMRES preconditioner
(Sec. 3.2, Fig. multigriddiagram, eq. eRichard, Appendix A).

Readings of points the paper leaves open (its figure with the transfer
operators is not available, and its smoother is replaced, see below):

* Hierarchy: cell-centred 2x2x2 agglomeration (the 4x4 -> 2x2 cell picture of
  Fig. multigriddiagram).  All three dimensions halve together while every
  one is even and >= 4; the last level must hold at most
  ``coarse_max_cells`` cells.  Level l has spacing 2^l h.
* Coarse operator: the 7-point form of e18 on every level, with the same
  boundary conditions (homogeneous on the plates, since every V-cycle level
  solves a residual equation).  Its face coefficients are averaged from the
  finer level: a coarse face coefficient is the mean of the 4 finer face
  coefficients lying on that coarse face, a coarse plate coefficient the mean
  of the 4 finer plate coefficients under it.  This operator is exactly half
  the Galerkin product R A P with piecewise-constant P and the mean-of-8 R.
  (Rediscretising e18 with a cell-mean coefficient converges 2-4x slower at
  the 1e3-1e4 coefficient contrasts of the filament workloads.)
* Smoother: red-black symmetric Gauss-Seidel, relaxation factor 1.  Colour =
  parity of i+j+k, red = even.  Pre-smoothing runs nu_pre times (red, black),
  post-smoothing nu_post times (black, red).  The paper's smoother is a
  degree-2 Chebyshev polynomial wrapped around one local SSOR step
  (Sec. 3.2); red-black symmetric Gauss-Seidel is the data-parallel form of
  that SSOR step.
* Restriction: mean of the residual over the 8 children (default).  That is
  not a multiple of the transpose of the trilinear prolongation, so the
  V-cycle is not a symmetric operator; CG (Sec. 5.3) assumes one.  Option
  ``restriction="transpose"``: R = P^T / 8, the transpose of the trilinear
  prolongation with its ghost rules folded back (full weighting over the 64
  fine cells around a coarse cell), which with nu_pre = nu_post makes the
  V-cycle symmetric (the pre-smoother red-black, the post-smoother its
  adjoint black-red, and P A_c^{-1} R = P A_c^{-1} P^T / 8).
* Prolongation: cell-centred trilinear interpolation (per dimension 3/4 of
  the parent, 1/4 of the nearer coarse neighbour).  Coarse ghosts outside the
  domain: mirror on the x/y sides (Neumann), negated mirror through the plates
  (homogeneous Dirichlet).
* Coarsest level: exact direct solve with a Cholesky factor of the dense
  coarse matrix (Sec. 3.2, "a sequential direct solver is applied to the
  coarsest mesh").
* Preconditioner application: one V-cycle from a zero initial guess with
  the right side v_j (Sec. 3.2, last paragraph).
* Full multigrid (Sec. 3.2: the first time step, solved from a zero guess,
  uses FMG; the later ones V-cycles): the paper gives no steps, so ``fmg``
  is the textbook cycle with this module's own transfers: right sides
  restricted to every level, the coarsest solved, then on each finer level
  one V-cycle from the interpolated coarser solution.  The right side is
  restricted algebraically (it is a Krylov vector, not a boundary-value
  problem), as in an algebraic FMG preconditioner.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.linalg as sla

from .operator import Faces, apply_faces, assemble_dense, diagonal, face_coefficients


def level_shapes(shape, coarse_max_cells=4096):
    """Shapes (nx, ny, nz) of all levels, finest first.

    Raises ValueError if the coarsest level holds more than
    ``coarse_max_cells`` cells."""
    shapes = [tuple(int(s) for s in shape)]
    while all(s % 2 == 0 and s >= 4 for s in shapes[-1]):
        shapes.append(tuple(s // 2 for s in shapes[-1]))
    nc = shapes[-1][0] * shapes[-1][1] * shapes[-1][2]
    if nc > coarse_max_cells:
        raise ValueError(f"grid {shape} coarsens to {shapes[-1]} "
                         f"({nc} cells > {coarse_max_cells})")
    return shapes


def coarsen_faces(F: Faces) -> Faces:
    """Coarse face coefficients: mean of the 4 finer faces on each coarse
    face (finer faces between children of one coarse cell drop out)."""
    nz, ny = F.wz.shape[0] + 1, F.bot.shape[0]
    nx = F.bot.shape[1]
    # finer x-faces between cells 2I+1 and 2I+2 lie on coarse x-faces
    wx = F.wx[:, :, 1::2].reshape(nz // 2, 2, ny // 2, 2, nx // 2 - 1).mean(axis=(1, 3))
    wy = F.wy[:, 1::2, :].reshape(nz // 2, 2, ny // 2 - 1, nx // 2, 2).mean(axis=(1, 4))
    wz = F.wz[1::2, :, :].reshape(nz // 2 - 1, ny // 2, 2, nx // 2, 2).mean(axis=(2, 4))
    bot = F.bot.reshape(ny // 2, 2, nx // 2, 2).mean(axis=(1, 3))
    top = F.top.reshape(ny // 2, 2, nx // 2, 2).mean(axis=(1, 3))
    return Faces(wx=wx, wy=wy, wz=wz, bot=bot, top=top)


@dataclass
class Level:
    shape: tuple  # (nx, ny, nz)
    h: tuple
    faces: Faces
    diag: np.ndarray


@dataclass
class Hierarchy:
    levels: list
    coarse_factor: tuple  # scipy cho_factor output of the dense coarsest A
    nu_pre: int
    nu_post: int
    dtype: type
    restriction: str = "mean"  # "mean" (of the 8 children) or "transpose" (P^T / 8)


def build_hierarchy(a, h, nu_pre=2, nu_post=2, coarse_max_cells=4096,
                    dtype=np.float64, restriction="mean"):
    """Level data for the V-cycle.  ``restriction``: "mean" (of the 8
    children) or "transpose" (P^T / 8).

    The finest level's faces are formed from the coefficient rounded to
    ``dtype`` (float32 for the mixed-precision preconditioner), in ``dtype``
    arithmetic; the coarser faces are averaged in float64 and then rounded to
    ``dtype``.  Diagonals and the coarse matrix are formed from the stored
    ``dtype`` faces in ``dtype`` arithmetic."""
    nz, ny, nx = a.shape
    shapes = level_shapes((nx, ny, nz), coarse_max_cells)
    levels = []
    F64 = face_coefficients(np.asarray(a, dtype=np.float64))
    h_l = tuple(float(x) for x in h)
    for li, shp in enumerate(shapes):
        if li == 0:
            F = face_coefficients(np.asarray(a).astype(dtype))
        else:
            F64 = coarsen_faces(F64)
            h_l = tuple(2.0 * x for x in h_l)
            F = F64.astype(dtype)
        levels.append(Level(shape=shp, h=h_l, faces=F, diag=diagonal(F, h_l)))
    A_c = assemble_dense(levels[-1].faces, levels[-1].h)
    factor = sla.cho_factor(A_c, lower=True)
    if restriction not in ("mean", "transpose"):
        raise ValueError("restriction must be 'mean' or 'transpose'")
    return Hierarchy(levels=levels, coarse_factor=factor, nu_pre=nu_pre,
                     nu_post=nu_post, dtype=dtype, restriction=restriction)


def colour_mask(shape_zyx, colour):
    """Cells whose (i + j + k) has the parity ``colour`` (0 = red)."""
    k, j, i = np.indices(shape_zyx)
    return (i + j + k) % 2 == colour


def rbgs_half_sweep(x, b, lev: Level, colour):
    """One Gauss-Seidel half-sweep over the cells of one colour, in place:
    x_c <- x_c + (b_c - (A x)_c) / D_c = (b_c + sum_f w_f x_nb / h_d^2) / D_c.

    Cells of one colour are never neighbours, so evaluating A x once before
    the update gives exactly the Gauss-Seidel values."""
    m = colour_mask(x.shape, colour)
    r = b - apply_faces(x, lev.faces, lev.h)
    x[m] += r[m] / lev.diag[m]
    return x


def restrict(r):
    """Coarse value = mean of the 8 children."""
    nz, ny, nx = r.shape
    return r.reshape(nz // 2, 2, ny // 2, 2, nx // 2, 2).mean(axis=(1, 3, 5))


def _interp_axis_transpose(f, axis, dirichlet):
    """Transpose of ``_interp_axis``: coarse[I] = 3/4 (f[2I] + f[2I+1]) +
    1/4 (f[2I-1] + f[2I+2]); the ghost terms of the first and last fine
    cells fold back onto coarse cells 0 and N-1 with the ghost's sign."""
    f = np.moveaxis(f, axis, 0)
    sign = -1.0 if dirichlet else 1.0
    even, odd = f[0::2], f[1::2]
    c = 0.75 * (even + odd)
    c[1:] += 0.25 * odd[:-1]  # f[2I-1] weights c[I] by 1/4
    c[:-1] += 0.25 * even[1:]  # f[2I+2] weights c[I] by 1/4
    c[0] += 0.25 * sign * even[0]  # ghost below cell 0 is sign * c[0]
    c[-1] += 0.25 * sign * odd[-1]  # ghost above cell N-1 is sign * c[N-1]
    return np.moveaxis(c, 0, axis)


def restrict_transpose(r):
    """R = P^T / 8: the transpose of ``prolong`` (one 1-D transpose per
    axis), scaled so that R keeps a constant interior field."""
    c = _interp_axis_transpose(r, 0, dirichlet=True)
    c = _interp_axis_transpose(c, 1, dirichlet=False)
    c = _interp_axis_transpose(c, 2, dirichlet=False)
    return c / 8.0


def restriction_of(hier):
    """The hierarchy's restriction operator."""
    return restrict_transpose if hier.restriction == "transpose" else restrict


def _interp_axis(c, axis, dirichlet):
    """Cell-centred linear interpolation doubling ``axis``:
    fine[2I] = 3/4 c[I] + 1/4 c[I-1], fine[2I+1] = 3/4 c[I] + 1/4 c[I+1],
    with ghost c[-1], c[N] = c[0], c[N-1] (mirror) or their negatives."""
    c = np.moveaxis(c, axis, 0)
    sign = -1.0 if dirichlet else 1.0
    lower = np.concatenate([sign * c[:1], c[:-1]], axis=0)  # c[I-1]
    upper = np.concatenate([c[1:], sign * c[-1:]], axis=0)  # c[I+1]
    fine = np.empty((2 * c.shape[0],) + c.shape[1:], dtype=c.dtype)
    fine[0::2] = 0.75 * c + 0.25 * lower
    fine[1::2] = 0.75 * c + 0.25 * upper
    return np.moveaxis(fine, 0, axis)


def prolong(e):
    """Trilinear cell-centred prolongation of a coarse correction
    (tensor product of the 1-D rule along z, y, x)."""
    e = _interp_axis(e, 0, dirichlet=True)  # z: plates, homogeneous Dirichlet
    e = _interp_axis(e, 1, dirichlet=False)  # y: Neumann sides
    e = _interp_axis(e, 2, dirichlet=False)  # x: Neumann sides
    return e


def coarse_solve(hier: Hierarchy, b):
    return sla.cho_solve(hier.coarse_factor, b.ravel()).reshape(b.shape).astype(hier.dtype)


def vcycle(hier: Hierarchy, b, level=0, x0=None):
    """One V-cycle for A_l x = b from x = 0, or from the guess x0 (Fig.
    multigriddiagram, applied recursively as described below eq. e31; the
    coarser levels always start from 0).  On the coarsest level the result is
    the direct solve whatever the guess."""
    lev = hier.levels[level]
    b = np.asarray(b, dtype=hier.dtype)
    if level == len(hier.levels) - 1:
        return coarse_solve(hier, b)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=hier.dtype)
    for _ in range(hier.nu_pre):
        rbgs_half_sweep(x, b, lev, 0)
        rbgs_half_sweep(x, b, lev, 1)
    r = b - apply_faces(x, lev.faces, lev.h)
    e = vcycle(hier, restriction_of(hier)(r), level + 1)
    x += prolong(e)
    for _ in range(hier.nu_post):
        rbgs_half_sweep(x, b, lev, 1)
        rbgs_half_sweep(x, b, lev, 0)
    return x


def fmg(hier: Hierarchy, b):
    """Full multigrid cycle for A x = b from no initial guess: the
    preconditioner of the first, cold-started solve (Sec. 3.2, FMG on the
    first time step).  The paper names the method without its steps; this is
    the textbook cycle:

    1. right sides of every level: b_0 = b, b_{l+1} = R b_l (the V-cycle's
       restriction);
    2. the coarsest level solved directly;
    3. level by level towards the finest, the coarser solution interpolated
       (the V-cycle's trilinear prolongation) is the initial guess of one
       V-cycle for A_l x_l = b_l."""
    nl = len(hier.levels)
    bs = [np.asarray(b, dtype=hier.dtype)]
    for _ in range(nl - 1):
        bs.append(restriction_of(hier)(bs[-1]))
    x = coarse_solve(hier, bs[-1])
    for level in range(nl - 2, -1, -1):
        x = vcycle(hier, bs[level], level, x0=prolong(x))
    return x
