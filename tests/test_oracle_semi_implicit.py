"""Pins of the oracle's elliptic-side assembly and electric field (Sec.
2.1-2.2): closed forms from trigonometric identities and a discrete
conservation law, none of which re-types the oracle's stencils."""
import numpy as np

from oracle.semi_implicit import coefficient, electric_field, right_side, second_difference


def _centres(n):
    return (np.arange(n) + 0.5) / n


def test_second_difference_of_cosines_is_exact_with_neumann_ghosts():
    """cos(pi x) at cell centres is even about both ends of [0, 1], so the
    ghost equal to the boundary cell is its exact continuation and
    delta^2 cos(pi x_i) = -4 sin^2(pi h / 2) cos(pi x_i) holds in every cell,
    boundary cells included (a one-sided or zero ghost breaks it there)."""
    nz, ny, nx = 6, 5, 7
    z, y, x = np.meshgrid(_centres(nz), _centres(ny), _centres(nx), indexing="ij")
    u = np.cos(np.pi * x) * np.cos(2 * np.pi * y) * np.cos(np.pi * z)
    for axis, (n, k) in zip((2, 1, 0), ((nx, 1), (ny, 2), (nz, 1))):
        want = -4.0 * np.sin(np.pi * k / (2 * n)) ** 2 * u
        np.testing.assert_allclose(second_difference(u, axis), want, atol=1e-14)


def test_right_side_closed_form_and_conservation():
    nz, ny, nx = 8, 6, 10
    h = (1 / nx, 1 / ny, 1 / nz)
    z, y, x = np.meshgrid(_centres(nz), _centres(ny), _centres(nx), indexing="ij")
    n_e = 2.0 + np.cos(np.pi * x) * np.cos(np.pi * y) * np.cos(np.pi * z)
    n_p = 1.5 + 0.1 * x
    tau, De = 0.3, (0.7, 1.1, 0.2)
    lam = sum(D / hd ** 2 * 4.0 * np.sin(np.pi * hd / 2) ** 2 for D, hd in zip(De, h))
    want = n_p - n_e + tau * lam * (n_e - 2.0)
    np.testing.assert_allclose(right_side(n_e, n_p, h, tau, De), want, rtol=1e-13, atol=1e-13)
    # zero-flux ghosts conserve the total: the diffusion term sums to zero
    rng = np.random.default_rng(31)
    ne = rng.random((nz, ny, nx))
    f = right_side(ne, np.zeros_like(ne), h, tau, De)
    assert abs(f.sum() + ne.sum()) < 1e-11 * ne.sum()


def test_coefficient_reduces_to_its_terms():
    rng = np.random.default_rng(32)
    n_e, n_p = rng.random((2, 3, 4, 5))
    assert np.all(coefficient(n_e, n_p, 2.5, 0.0, 9.0, 9.0) == 2.5)  # tau = 0: vacuum permittivity only
    P = coefficient(n_e, n_p, 0.0, 1.0, 1.0, 0.0)
    assert np.array_equal(P, n_e)
    # the relaxation rate e/eps0 (mu_p n_p + mu_e n_e) scales with tau
    d = coefficient(n_e, n_p, 1.0, 0.4, 3.0, 0.5) - coefficient(n_e, n_p, 1.0, 0.2, 3.0, 0.5)
    np.testing.assert_allclose(d, 0.2 * (3.0 * n_e + 0.5 * n_p), rtol=1e-14)


def test_electric_field_closed_forms():
    """E of the exact solution for a = a(x, y), f = 0 (phi linear in z) is
    the uniform plate field in every cell, plates included; E of cosine
    profiles follows sin(pi k h)/h exactly, side cells included."""
    nz, ny, nx = 6, 4, 8
    h = (1 / nx, 1 / ny, 1 / nz)
    z, y, x = np.meshgrid(_centres(nz), _centres(ny), _centres(nx), indexing="ij")
    pb, pt = 0.3, 1.7
    ex, ey, ez, em = electric_field(pb + (pt - pb) * z, h, pb, pt)
    np.testing.assert_allclose(ez, -(pt - pb), rtol=1e-13)
    assert np.all(ex == 0) and np.all(ey == 0)
    np.testing.assert_allclose(em, abs(pt - pb), rtol=1e-13)
    phi = np.cos(np.pi * x) * np.cos(np.pi * y) + 0.0 * z
    ex, ey, ez, em = electric_field(phi, h, 0.0, 0.0)
    np.testing.assert_allclose(ex, np.sin(np.pi * x) * np.cos(np.pi * y) * np.sin(np.pi * h[0]) / h[0], atol=1e-13)
    np.testing.assert_allclose(ey, np.cos(np.pi * x) * np.sin(np.pi * y) * np.sin(np.pi * h[1]) / h[1], atol=1e-13)
    np.testing.assert_allclose(em, np.sqrt(ex ** 2 + ey ** 2 + ez ** 2), rtol=1e-15)
