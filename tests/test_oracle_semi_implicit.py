"""Pins of the oracle's elliptic-side assembly and electric field (Sec.
2.1-2.2): closed forms from trigonometric identities and a discrete
conservation law, none of which re-types the oracle's stencils."""
import numpy as np
import pytest

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


# ---------------------------------------------------------------- the time step
def _uniform_case(n=8, c=0.7):
    from oracle.semi_implicit import StepParams
    shape = (n, n, n)
    h = (1 / n,) * 3
    prm = StepParams(eps0_over_e=0.2, mu_e=3.0, mu_p=0.05, De=(0.01, 0.02, 0.03))
    return np.full(shape, c), np.full(shape, c), h, prm


def _ionisation(k):
    """Source term of the density equations with a constant ionisation
    coefficient: L_e = L_p = k |E| n_e (no drift or diffusion)."""
    def transport(n_e, n_p, E):
        s = k * E[3] * n_e
        return s, s
    return transport


def test_second_order_step_is_the_explicit_midpoint_rule_on_uniform_densities():
    """Uniform n_e = n_p: the right side of semi2 vanishes and P is uniform,
    so phi is exactly linear in z and |E| = |phi_top - phi_bot| in every
    cell; with the ionisation source the densities stay equal and uniform
    and each step multiplies them by 1 + x + x^2 / 2, x = k |E| tau (the
    explicit midpoint rule on n' = k |E| n), in every cell; the first-order
    scheme multiplies by 1 + x.  Two planted mistakes -- the corrector
    based on n^{n+1/2} instead of n^n, and a full-tau predictor -- give
    (1 + x/2)(1 + x) and 1 + x + x^2 instead."""
    from oracle.semi_implicit import time_step
    ne, npp, h, prm = _uniform_case()
    k, tau, pb, pt = 0.4, 0.3, 0.0, 2.0
    x = k * abs(pt - pb) * tau
    for scheme, g in (("second", 1 + x + x * x / 2), ("first", 1 + x)):
        e, p, phi = ne, npp, None
        for s in range(3):
            r = time_step(e, p, h, prm, tau, _ionisation(k), pb, pt, phi_prev=phi, scheme=scheme, tol=1e-13)
            np.testing.assert_allclose(r.E[3], abs(pt - pb), rtol=1e-10)
            np.testing.assert_allclose(r.n_e, ne * g ** (s + 1), rtol=1e-10)
            np.testing.assert_allclose(r.n_p, r.n_e, rtol=0, atol=0)
            e, p, phi = r.n_e, r.n_p, r.phi
    assert abs((1 + x / 2) * (1 + x) - (1 + x + x * x / 2)) > 1e-3
    assert abs((1 + x + x * x) - (1 + x + x * x / 2)) > 1e-3


def _series_resistance_phi(a_z, hz, pb, pt):
    """Exact discrete solution for a = a(z), f = 0 (1-D, eq. e18 with the
    mirrored plate ghosts): the flux F = w (phi_{k+1} - phi_k) / hz is the
    same through every z-face; the plate faces are half cells with
    coefficient a_c."""
    w = 0.5 * (a_z[1:] + a_z[:-1])
    R = hz / (2 * a_z[0]) + np.sum(hz / w) + hz / (2 * a_z[-1])
    F = (pt - pb) / R
    phi = np.empty_like(a_z)
    phi[0] = pb + F * hz / (2 * a_z[0])
    for k in range(len(a_z) - 1):
        phi[k + 1] = phi[k] + F * hz / w[k]
    return phi


@pytest.mark.parametrize("scheme, tau_eff_factor", [("second", 0.5), ("first", 1.0)])
def test_elliptic_problem_of_the_step_uses_half_tau_in_the_second_order_scheme(scheme, tau_eff_factor):
    """Densities n_e = n_p varying in z only (no diffusion): f = 0 and the
    coefficient P = eps0/e + tau_eff (mu_p + mu_e) n(z), so phi is the
    series-resistance solution with tau_eff = tau/2 in eq. semi2 and tau in
    eq. e15; the other factor gives a visibly different phi."""
    from oracle.semi_implicit import StepParams, time_step
    n = 16
    zc = (np.arange(n) + 0.5) / n
    prof = 1.0 + 40.0 * np.exp(-((zc - 0.4) / 0.1) ** 2)
    ne = np.broadcast_to(prof[:, None, None], (n, 4, 4)).copy()
    h = (1 / 4, 1 / 4, 1 / n)
    prm = StepParams(eps0_over_e=0.1, mu_e=2.0, mu_p=0.5, De=(0.0, 0.0, 0.0))
    tau, pb, pt = 0.6, 0.5, 1.5
    r = time_step(ne, ne.copy(), h, prm, tau, lambda e, p, E: (0 * e, 0 * p), pb, pt, scheme=scheme, tol=1e-13)
    want = _series_resistance_phi(0.1 + tau_eff_factor * tau * 2.5 * prof, h[2], pb, pt)
    wrong = _series_resistance_phi(0.1 + (1.5 - tau_eff_factor) * tau * 2.5 * prof, h[2], pb, pt)
    np.testing.assert_allclose(r.phi, np.broadcast_to(want[:, None, None], r.phi.shape), rtol=1e-10)
    assert np.abs(want - wrong).max() > 1e-3


def test_zero_transport_keeps_phi_and_warm_starts_take_no_steps():
    """With no transport the densities do not change, so every step solves
    the same elliptic problem: phi stays the same and each warm-started
    solve after the first converges in 0 steps (its guess already meets the
    tolerance)."""
    from oracle.semi_implicit import StepParams, time_step
    rng = np.random.default_rng(33)
    n = 16
    ne = 1.0 + rng.random((n, n, n))
    npp = 1.0 + rng.random((n, n, n))
    h = (1 / n,) * 3
    prm = StepParams(eps0_over_e=0.3, mu_e=1.0, mu_p=0.1, De=(0.01, 0.01, 0.01))
    zero = lambda e, p, E: (np.zeros_like(e), np.zeros_like(p))  # noqa: E731
    r0 = time_step(ne, npp, h, prm, 0.2, zero, 0.0, 1.0, tol=1e-10)
    assert r0.iterations > 0 and np.array_equal(r0.n_e, ne) and np.array_equal(r0.n_p, npp)
    r1 = time_step(r0.n_e, r0.n_p, h, prm, 0.2, zero, 0.0, 1.0, phi_prev=r0.phi, tol=1e-10)
    assert r1.iterations == 0 and np.array_equal(r1.phi, r0.phi)
