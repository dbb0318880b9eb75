"""Pins of the oracle's other Krylov methods (Sec. 5.3, Table t1): the
optimality properties that define them, computed here by dense linear
algebra over explicit Krylov bases, and their relations to each other."""
import numpy as np
import pytest

from oracle.fgmres import fgmres
from oracle.krylov import bicgstab, cg, cgs, gmres
from oracle.multigrid import build_hierarchy, vcycle
from oracle.operator import apply_operator, assemble_dense, rhs


def _problem(n=8, seed=51):
    rng = np.random.default_rng(seed)
    a = np.exp(rng.uniform(-1.5, 1.5, (n, n, n)))
    f = rng.standard_normal((n, n, n))
    h = (1 / n,) * 3
    b = rhs(f, a, h, 0.2, 1.0).ravel()
    Ad = assemble_dense(__import__("oracle.operator", fromlist=["x"]).face_coefficients(a), h)
    hier = build_hierarchy(a, h)

    def A(x):
        return apply_operator(x.reshape(a.shape), a, h).ravel()

    def M(v):
        return vcycle(hier, v.reshape(a.shape)).ravel()
    return A, M, b, Ad


def _krylov_basis(op, v, k):
    """Orthonormal basis of span{v, op v, ..., op^{k-1} v}."""
    K = [v]
    for _ in range(k - 1):
        K.append(op(K[-1]))
    Q, _ = np.linalg.qr(np.stack(K, axis=1))
    return Q


def test_exact_preconditioner_converges_in_one_iteration():
    A, _, b, Ad = _problem()
    inv = np.linalg.inv(Ad)

    def M(v):
        return inv @ v
    for name, fn in (("cg", lambda: cg(A, b, M, tol=1e-10)), ("fcg", lambda: cg(A, b, M, tol=1e-10, flexible=True)),
                     ("gmres", lambda: gmres(A, b, M, tol=1e-10)), ("cgs", lambda: cgs(A, b, M, tol=1e-10)),
                     ("bicgstab", lambda: bicgstab(A, b, M, tol=1e-10))):
        res = fn()
        assert res.converged and res.iterations == 1, (name, res.iterations)
        np.testing.assert_allclose(res.x, inv @ b, rtol=1e-9, atol=1e-12)


def _jacobi(Ad):
    d = np.diag(Ad).copy()

    def M(v):
        return v / d
    return M


@pytest.mark.parametrize("k", [1, 3, 6])
def test_cg_minimises_the_energy_error_over_the_preconditioned_krylov_space(k):
    """CG with a symmetric positive definite preconditioner (Jacobi): x_k
    minimises ||x - x*||_A over span{M r0, (M A) M r0, ...} (x0 = 0), here
    computed by a dense Galerkin solve on an explicit basis.  (The V-cycle is
    not symmetric: its restriction, the mean of 8, is not the transpose of the
    trilinear prolongation, so CG has no such guarantee with it.)"""
    A, _, b, Ad = _problem()
    M = _jacobi(Ad)
    Q = _krylov_basis(lambda v: M(A(v)), M(b), k)
    c = np.linalg.solve(Q.T @ Ad @ Q, Q.T @ b)
    res = cg(A, b, M, tol=0.0, max_iter=k)
    np.testing.assert_allclose(res.x, Q @ c, rtol=1e-8, atol=1e-10 * np.abs(Q @ c).max())


def test_fcg_equals_cg_with_a_fixed_symmetric_preconditioner():
    A, _, b, Ad = _problem()
    M = _jacobi(Ad)
    r1 = cg(A, b, M, tol=0.0, max_iter=7)
    r2 = cg(A, b, M, tol=0.0, max_iter=7, flexible=True)
    np.testing.assert_allclose(r2.x, r1.x, rtol=1e-9, atol=1e-12 * np.abs(r1.x).max())


def test_vcycle_preconditioner_is_not_symmetric():
    """The reason the comparison favours the flexible and minimal-residual
    methods: with mean-of-8 restriction and trilinear prolongation the
    V-cycle's matrix is not symmetric (nor A-self-adjoint)."""
    A, M, b, Ad = _problem(n=4)
    n = Ad.shape[0]
    Mm = np.stack([M(e) for e in np.eye(n)], axis=1)
    assert np.linalg.norm(Mm - Mm.T) > 1e-3 * np.linalg.norm(Mm)


def _symmetric_vcycle(n=8, seed=51):
    """The _problem of size n with the V-cycle of R = P^T / 8, nu = 2 / 2."""
    rng = np.random.default_rng(seed)
    a = np.exp(rng.uniform(-1.5, 1.5, (n, n, n)))
    hier = build_hierarchy(a, (1 / n,) * 3, restriction="transpose")

    def M(v):
        return vcycle(hier, v.reshape(a.shape)).ravel()
    return M


@pytest.mark.parametrize("k", [1, 3, 6])
def test_cg_with_the_symmetric_vcycle_minimises_the_energy_error(k):
    """With the symmetric V-cycle (R = P^T / 8) CG is CG again: x_k
    minimises ||x - x*||_A over the Krylov space of M A from M r0 (dense
    Galerkin solve on an explicit basis), and FCG gives the same iterates."""
    A, _, b, Ad = _problem()
    M = _symmetric_vcycle()
    Q = _krylov_basis(lambda v: M(A(v)), M(b), k)
    c = np.linalg.solve(Q.T @ Ad @ Q, Q.T @ b)
    res = cg(A, b, M, tol=0.0, max_iter=k)
    np.testing.assert_allclose(res.x, Q @ c, rtol=1e-8, atol=1e-10 * np.abs(Q @ c).max())
    res_f = cg(A, b, M, tol=0.0, max_iter=k, flexible=True)
    np.testing.assert_allclose(res_f.x, res.x, rtol=1e-8, atol=1e-10 * np.abs(res.x).max())


def test_symmetric_vcycle_preconditioner_is_symmetric():
    """The counterpart of the test above: with R = P^T / 8 the V-cycle's
    matrix is symmetric (to rounding)."""
    A, _, b, Ad = _problem(n=4)
    M = _symmetric_vcycle(n=4)
    n = Ad.shape[0]
    Mm = np.stack([M(e) for e in np.eye(n)], axis=1)
    assert np.linalg.norm(Mm - Mm.T) <= 1e-13 * np.linalg.norm(Mm)


@pytest.mark.parametrize("k", [2, 5])
def test_gmres_minimises_the_residual_and_equals_fgmres(k):
    """Right-preconditioned GMRES: x_k = M u with u minimising ||b - A M u||
    over the Krylov space of A M (dense least squares); with a fixed M the
    iterates equal FGMRES's."""
    A, M, b, Ad = _problem()
    Q = _krylov_basis(lambda v: A(M(v)), b, k)
    AMQ = np.stack([A(M(Q[:, i])) for i in range(k)], axis=1)
    c, *_ = np.linalg.lstsq(AMQ, b, rcond=None)
    want = M(Q @ c)
    res = gmres(A, b, M, tol=0.0, max_iter=k)
    np.testing.assert_allclose(res.x, want, rtol=1e-8, atol=1e-10 * np.abs(want).max())
    ref = fgmres(A, b, M, tol=0.0, max_iter=k)
    np.testing.assert_allclose(res.x, ref.x, rtol=1e-9, atol=1e-12 * np.abs(ref.x).max())


@pytest.mark.parametrize("method", [cgs, bicgstab])
def test_nonsymmetric_methods_reach_the_exact_solution(method):
    """CGS and BiCGSTAB with the V-cycle converge to the dense solution, and
    the residual they update recursively matches the true one at exit."""
    A, M, b, Ad = _problem()
    res = method(A, b, M, tol=1e-10, max_iter=60)
    assert res.converged
    x_star = np.linalg.solve(Ad, b)
    assert np.linalg.norm(res.x - x_star) <= 1e-8 * np.linalg.norm(x_star)
    assert res.true_relres < 1e-10 and abs(res.res_hist[-1] - res.true_relres) < 1e-11


@pytest.mark.parametrize("constant_a", [True, False])
@pytest.mark.parametrize("method", ["fgmres", "gmres", "cg", "fcg", "cgs", "bicgstab"])
def test_methods_on_the_anisotropic_comparison_mesh(method, constant_a):
    """The streamer channel on a 16 x 16 x 20 mesh of the unit cube (the
    aspect of the 256 x 256 x 320 mesh of Table t1, h_z < h_x = h_y): each
    method with the oracle's V-cycle reaches the exact discrete solution,
    the spectral (cosine/sine transform) solution for a = 1 and a sparse
    direct solve for the variable coefficient."""
    from oracle.exact import sparse_solve, spectral_solve
    from workloads import config_streamer_mesh
    p = config_streamer_mesh(16, 16, 20, constant_a=constant_a)
    b = rhs(p.f, p.a, p.h, p.phi_bot, p.phi_top)
    hier = build_hierarchy(p.a, p.h)
    assert hier.levels[-1].shape == (4, 4, 5)

    def A(x):
        return apply_operator(x, p.a, p.h)

    def M(v):
        return vcycle(hier, v)
    fn = {"fgmres": fgmres, "gmres": gmres, "cg": cg, "fcg": lambda *a, **k: cg(*a, flexible=True, **k),
          "cgs": cgs, "bicgstab": bicgstab}[method]
    res = fn(A, b, M, tol=1e-11, max_iter=100)
    assert res.converged
    if constant_a:
        exact = spectral_solve(b, p.h)
    else:
        exact = sparse_solve(p.a, p.f, p.h, p.phi_bot, p.phi_top)
    assert np.linalg.norm(res.x - exact) <= 1e-9 * np.linalg.norm(exact)
