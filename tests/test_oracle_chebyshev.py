"""Pins of the oracle's Chebyshev(2)+SSOR smoother (Sec. 3.2, eq. qntn) and
of the counter-based generator that draws its Arnoldi start vectors."""
import numpy as np
import pytest

from oracle.chebyshev import (chebyshev_smooth, lambda_max_estimate, level_bounds, splitmix64, ssor,
                              start_vector, vcycle_chebyshev)
from oracle.fgmres import fgmres
from oracle.multigrid import build_hierarchy, vcycle
from oracle.operator import apply_operator, assemble_dense, face_coefficients, rhs
from workloads import make_config


def _level(n=4, seed=61):
    rng = np.random.default_rng(seed)
    a = np.exp(rng.uniform(-1.0, 1.0, (n, n, n)))
    h = (1 / n,) * 3
    hier = build_hierarchy(a, h)
    lev = hier.levels[0]
    A = assemble_dense(face_coefficients(a), h)
    N = a.size
    Minv = np.stack([ssor(lev, e.reshape(a.shape)).ravel() for e in np.eye(N)], axis=1)
    return lev, A, Minv, a.shape


def test_ssor_preconditioned_spectrum_lies_in_0_1():
    """Symmetric Gauss-Seidel is a convergent symmetric splitting: M^{-1} A
    has real eigenvalues in (0, 1]."""
    lev, A, Minv, _ = _level()
    ev = np.linalg.eigvals(Minv @ A)
    assert np.abs(ev.imag).max() < 1e-10
    assert ev.real.min() > 0 and ev.real.max() <= 1 + 1e-12


def test_smoother_error_propagator_is_the_chebyshev_polynomial_of_eq_qntn():
    """With b = 0 the smoother maps x to q_2(M^{-1} A) x,
    q_2(t) = T_2((lmax + l* - 2t)/(lmax - l*)) / T_2((lmax + l*)/(lmax - l*)),
    T_2(y) = 2 y^2 - 1; the matrix polynomial is formed densely here."""
    lev, A, Minv, shape = _level()
    lmax, lstar = 1.05, 0.12
    N = A.shape[0]
    E = np.stack([chebyshev_smooth(e.reshape(shape), np.zeros(shape), lev, lmax, lstar).ravel()
                  for e in np.eye(N)], axis=1)
    B = Minv @ A
    Y = ((lmax + lstar) * np.eye(N) - 2.0 * B) / (lmax - lstar)
    y0 = (lmax + lstar) / (lmax - lstar)
    Q = (2.0 * Y @ Y - np.eye(N)) / (2.0 * y0 * y0 - 1.0)
    np.testing.assert_allclose(E, Q, atol=1e-12)


def test_arnoldi_estimate_brackets_the_largest_eigenvalue():
    lev, A, Minv, shape = _level()
    true = np.linalg.eigvals(Minv @ A).real.max()
    est = lambda_max_estimate(lev, np.random.default_rng(62).uniform(-1, 1, shape))
    assert 0.9 * true <= est <= true + 1e-12


@pytest.mark.slow
def test_chebyshev_vcycle_against_red_black_gauss_seidel():
    """The evaluation behind the GPU path's smoother choice (filament
    workload, 32^3, max(a) = 1e4): both preconditioners converge; the
    Chebyshev(2)+SSOR V-cycle, about twice the smoothing work, takes at least
    as many FGMRES steps."""
    p = make_config(3, n=32)
    b = rhs(p.f, p.a, p.h, p.phi_bot, p.phi_top)
    hier = build_hierarchy(p.a, p.h)
    bounds = level_bounds(hier)

    def A(x):
        return apply_operator(x, p.a, p.h)
    r_cheb = fgmres(A, b, lambda v: vcycle_chebyshev(hier, bounds, v), tol=1e-8)
    r_gs = fgmres(A, b, lambda v: vcycle(hier, v), tol=1e-8)
    print(f"FGMRES steps: Chebyshev(2)+SSOR {r_cheb.iterations}, red-black SGS {r_gs.iterations}")
    assert r_cheb.converged and r_gs.converged
    assert r_cheb.iterations >= r_gs.iterations


def test_splitmix64_reference_outputs():
    """The first outputs of SplitMix64 seeded with 0, as published with the
    generator's reference implementation."""
    got = [int(v) for v in splitmix64(0, np.arange(1, 5, dtype=np.uint64))]
    assert got == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F, 0xF88BB8A8724C81EC]


def test_start_vector_is_uniform_on_minus_one_one():
    """2 (z >> 11) 2^-53 - 1 of a well-mixed stream: values in [-1, 1), mean
    0 and variance 1/3 within sampling error (2^18 cells), distinct levels
    draw different vectors, and the value of cell c is the formula applied
    to output c + 1."""
    v = start_vector((64, 64, 64), 0)
    n = v.size
    assert v.min() >= -1.0 and v.max() < 1.0
    assert abs(v.mean()) < 5 * np.sqrt(1 / 3 / n)
    assert abs(v.var() - 1 / 3) < 5 * np.sqrt(1 / 45 / n)
    w = start_vector((64, 64, 64), 1)
    assert abs(np.corrcoef(v.ravel(), w.ravel())[0, 1]) < 5 / np.sqrt(n)
    z = 0xE220A8397B1DCDAF  # output 1 of seed 0
    assert v.ravel()[0] == 2.0 * (z >> 11) * 2.0 ** -53 - 1.0


def test_vcycle_chebyshev_nu_repeats_the_smoother():
    """nu = 2 equals smoothing twice on each side, spelled out by hand on a
    two-level hierarchy."""
    from oracle.multigrid import coarse_solve, prolong, restrict
    from oracle.operator import apply_faces
    rng = np.random.default_rng(63)
    a = np.exp(rng.uniform(-1, 1, (6, 6, 6)))
    hier = build_hierarchy(a, (1 / 6,) * 3)
    assert len(hier.levels) == 2
    bounds = [(0.1, 1.1)]
    b = rng.standard_normal(a.shape)
    lev = hier.levels[0]
    x = chebyshev_smooth(chebyshev_smooth(np.zeros_like(b), b, lev, 1.1, 0.1), b, lev, 1.1, 0.1)
    x = x + prolong(coarse_solve(hier, restrict(b - apply_faces(x, lev.faces, lev.h))))
    x = chebyshev_smooth(chebyshev_smooth(x, b, lev, 1.1, 0.1), b, lev, 1.1, 0.1)
    np.testing.assert_allclose(vcycle_chebyshev(hier, bounds, b, nu=2), x, rtol=0, atol=0)
