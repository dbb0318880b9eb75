"""Pins of the oracle's operator (eq. e18, Sec. 2.2, boundary conditions of
Sec. 1) against values fixed independently of the oracle: hand-derived
stencils, closed-form solutions and the spectral decomposition."""
import os

import numpy as np
import pytest

from oracle.operator import (apply_faces, apply_operator, assemble_dense,
                             assemble_sparse, diagonal, face_coefficients,
                             lifting, rhs)
from oracle.exact import (manufactured, sparse_solve, spectral_eigenvalues,
                          spectral_solve)


def _read_golden(path):
    d = {"A": []}
    with open(path) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            key, *vals = line.split()
            vals = [float(v) for v in vals]
            if key == "A":
                d["A"].append(vals)
            else:
                d[key] = vals
    return d


@pytest.mark.parametrize("name", ["stencil_2x1x2.txt", "stencil_2x2x1.txt"])
def test_hand_derived_stencil(golden_dir, name):
    g = _read_golden(os.path.join(golden_dir, name))
    nx, ny, nz = (int(v) for v in g["shape"])
    h = tuple(g["h"])
    a = np.array(g["a"]).reshape(nz, ny, nx)
    A_expected = np.array(g["A"])
    A = assemble_dense(face_coefficients(a), h)
    np.testing.assert_allclose(A, A_expected, rtol=0, atol=1e-12)
    np.testing.assert_allclose(assemble_sparse(a, h).toarray(), A_expected, rtol=0, atol=1e-12)
    pb, pt = g["phi"]
    np.testing.assert_allclose(lifting(a, h, pb, pt).ravel(), g["lift"], rtol=0, atol=1e-12)
    # apply_operator with plate values = A x - lifting
    x = np.arange(1.0, nx * ny * nz + 1).reshape(a.shape)
    np.testing.assert_allclose(apply_operator(x, a, h, pb, pt).ravel(),
                               A_expected @ x.ravel() - np.array(g["lift"]), atol=1e-12)


def _rand_a(shape, rng, lo=0.5, hi=3.0):
    return rng.uniform(lo, hi, size=shape)


def test_sparse_and_dense_assemblies_agree():
    rng = np.random.default_rng(1)
    for shape in [(3, 4, 5), (2, 2, 2), (1, 3, 2), (4, 1, 1)]:
        a = _rand_a(shape, rng)
        h = (0.3, 0.7, 0.2)
        D = assemble_dense(face_coefficients(a), h)
        S = assemble_sparse(a, h).toarray()
        np.testing.assert_allclose(D, S, rtol=1e-14, atol=1e-12)
        np.testing.assert_allclose(np.diag(D), diagonal(face_coefficients(a), h).ravel(), rtol=1e-14)


def test_symmetric_positive_definite():
    """P4: <Au, v> = <u, Av> and every eigenvalue > 0."""
    rng = np.random.default_rng(2)
    a = _rand_a((5, 4, 6), rng, 0.01, 100.0)
    h = (1 / 6, 1 / 4, 1 / 5)
    A = assemble_dense(face_coefficients(a), h)
    assert np.max(np.abs(A - A.T)) <= 1e-14 * np.max(np.abs(A))
    u, v = rng.standard_normal((2, a.size))
    lhs = np.dot(A @ u, v)
    assert abs(lhs - np.dot(u, A @ v)) <= 1e-13 * abs(lhs) + 1e-12
    assert np.linalg.eigvalsh(A).min() > 0


def test_linear_in_z_is_exact():
    """P1: with a = a(x, y) and f = 0 the discrete solution is exactly
    phi_bot + (phi_top - phi_bot) z at the cell centres."""
    rng = np.random.default_rng(3)
    nx, ny, nz = 5, 4, 7
    axy = _rand_a((ny, nx), rng, 0.1, 10.0)
    a = np.broadcast_to(axy, (nz, ny, nx)).copy()
    h = (1 / nx, 1 / ny, 1 / nz)
    zc = (np.arange(nz) + 0.5) / nz
    pb, pt = -0.3, 2.5
    phi = np.broadcast_to((pb + (pt - pb) * zc)[:, None, None], a.shape).copy()
    assert np.max(np.abs(apply_operator(phi, a, h, pb, pt))) < 1e-11
    np.testing.assert_allclose(sparse_solve(a, np.zeros_like(a), h, pb, pt), phi, atol=1e-12)


def test_series_resistance_1d():
    """P5: a = a(z), f = 0: one flux J crosses every z-face, J = (phi_top -
    phi_bot) / R with R = hz/(2 a_0) + sum_faces hz / w + hz/(2 a_{N-1}),
    w the arithmetic face mean (Sec. 2.2)."""
    rng = np.random.default_rng(4)
    nx, ny, nz = 3, 2, 9
    az = rng.uniform(0.2, 50.0, nz)
    a = np.broadcast_to(az[:, None, None], (nz, ny, nx)).copy()
    hz = 1 / nz
    h = (0.5, 0.5, hz)
    pb, pt = 1.0, 4.0
    w = 0.5 * (az[1:] + az[:-1])
    R = hz / (2 * az[0]) + np.sum(hz / w) + hz / (2 * az[-1])
    J = (pt - pb) / R
    phi_z = np.empty(nz)
    phi_z[0] = pb + J * hz / (2 * az[0])
    for k in range(nz - 1):
        phi_z[k + 1] = phi_z[k] + J * hz / w[k]
    assert abs(phi_z[-1] + J * hz / (2 * az[-1]) - pt) < 1e-12
    phi = np.broadcast_to(phi_z[:, None, None], a.shape).copy()
    assert np.max(np.abs(apply_operator(phi, a, h, pb, pt))) < 1e-10
    np.testing.assert_allclose(sparse_solve(a, np.zeros_like(a), h, pb, pt), phi, rtol=1e-12)


def test_spectrum_matches_closed_form():
    """P2: constant a: eigenvalues sum_d 4 a sin^2(pi p_d / (2 N_d)) / h_d^2,
    p_z = 1..N_z (Dirichlet plates), p_x,y = 0..N-1 (Neumann sides)."""
    a0 = 2.5
    shape = (4, 3, 5)
    h = (0.2, 1 / 3, 0.25)
    a = np.full(shape, a0)
    ev = np.sort(np.linalg.eigvalsh(assemble_dense(face_coefficients(a), h)))
    ev_closed = np.sort(spectral_eigenvalues(shape, h, a0).ravel())
    np.testing.assert_allclose(ev, ev_closed, rtol=1e-12)


def test_spectral_solver_matches_sparse_direct():
    rng = np.random.default_rng(5)
    shape = (10, 8, 12)
    h = (1 / 12, 1 / 8, 1 / 10)
    f = rng.standard_normal(shape)
    a0 = 1.7
    a = np.full(shape, a0)
    b = rhs(f, a, h, 0.2, 1.0)
    ps = spectral_solve(b, h, a0)
    pd = sparse_solve(a, f, h, 0.2, 1.0)
    np.testing.assert_allclose(ps, pd, rtol=1e-11, atol=1e-12)
    # and it inverts the operator
    np.testing.assert_allclose(apply_faces(ps, face_coefficients(a), h), b, rtol=1e-10, atol=1e-10)


def test_manufactured_source_formula():
    """f = -div(a grad phi) of ``manufactured`` against central differences of
    the flux a grad phi of the same closed-form phi and a."""
    pi = np.pi
    phi_top = 1.0

    def phi(x, y, z):
        return phi_top * z + np.cos(pi * x) * np.cos(pi * y) * np.sin(pi * z)

    def a(x, y, z):
        return 1 + 0.5 * np.cos(pi * x) * np.cos(pi * y) * np.cos(pi * z)

    n = 8
    _, _, f = manufactured(n, phi_top)
    c = (np.arange(n) + 0.5) / n
    rng = np.random.default_rng(6)
    d = 1e-4
    for _ in range(10):
        k, j, i = rng.integers(0, n, 3)
        x, y, z = c[i], c[j], c[k]

        def flux(xx, yy, zz, axis):
            e = [0.0, 0.0, 0.0]
            e[axis] = d
            g = (phi(xx + e[0], yy + e[1], zz + e[2]) - phi(xx - e[0], yy - e[1], zz - e[2])) / (2 * d)
            return a(xx, yy, zz) * g

        div = 0.0
        for axis in range(3):
            e = [0.0, 0.0, 0.0]
            e[axis] = d
            div += (flux(x + e[0], y + e[1], z + e[2], axis)
                    - flux(x - e[0], y - e[1], z - e[2], axis)) / (2 * d)
        assert abs(-div - f[k, j, i]) < 1e-5 * (1 + abs(f[k, j, i]))


def test_manufactured_second_order():
    """P9: the discrete solution converges to the smooth one at second order
    (Sec. 2.2 expects second-order accuracy for smooth solutions)."""
    errs = []
    for n in (8, 16, 32):
        phi, a, f = manufactured(n)
        h = (1 / n,) * 3
        ph = sparse_solve(a, f, h, 0.0, 1.0)
        errs.append(np.sqrt(np.mean((ph - phi) ** 2)))
    ratios = [errs[i] / errs[i + 1] for i in range(len(errs) - 1)]
    for r in ratios:
        assert 3.6 < r < 4.4, ratios
