"""Pins of the oracle's FGMRES (Algorithm 1, Sec. 3.1; criterion, Sec. 5.2)."""
import numpy as np
import pytest

from oracle.fgmres import fgmres, solve_poisson
from oracle.operator import apply_operator, assemble_dense, face_coefficients, rhs
from oracle.exact import spectral_eigenvalues, spectral_solve
from workloads import make_config
from workloads.streamer import config_two_filaments


def _small_problem(shape=(3, 3, 3), seed=20):
    rng = np.random.default_rng(seed)
    a = rng.uniform(0.2, 5.0, shape)
    h = tuple(1.0 / s for s in shape[::-1])
    A = assemble_dense(face_coefficients(a), h)
    b = rng.standard_normal(a.size)
    return A, b


def test_arnoldi_relation_and_orthonormality():
    """P7: V_{k+1}^T V_{k+1} = I and A Z_k = V_{k+1} Hbar_k."""
    p = make_config(2, n=16)
    k = 6
    res = solve_poisson(p.a, p.f, p.h, p.phi_bot, p.phi_top, tol=0.0, max_iter=k)
    assert res.iterations == k and not res.converged
    V = np.stack([v.ravel() for v in res.V], axis=1)
    Z = np.stack([z.ravel() for z in res.Z], axis=1)
    assert V.shape[1] == k + 1
    # modified Gram-Schmidt loses orthogonality in proportion to the residual
    # reduction (about 1e-16 / r_k); a wrong step would give O(1) errors
    assert np.abs(V.T @ V - np.eye(k + 1)).max() <= 1e-14 / min(res.res_hist)
    AZ = np.stack([apply_operator(z, p.a, p.h).ravel() for z in res.Z], axis=1)
    VH = V @ res.Hbar[: k + 1, :k]
    assert np.linalg.norm(AZ - VH) <= 1e-12 * np.linalg.norm(AZ)


def test_estimate_equals_true_residual():
    p = make_config(1, n=16)
    for k in (3, 5):
        res = solve_poisson(p.a, p.f, p.h, p.phi_bot, p.phi_top, tol=0.0, max_iter=k)
        assert len(res.res_hist) == k + 1
        b = rhs(p.f, p.a, p.h, p.phi_bot, p.phi_top)
        true = np.linalg.norm(b - apply_operator(res.x, p.a, p.h)) / np.linalg.norm(b)
        assert abs(true - res.res_hist[-1]) <= 1e-9 * true + 1e-15
        assert abs(true - res.true_relres) <= 1e-12 * true + 1e-16


def test_identity_preconditioner_is_minimal_residual():
    """With M = I and m >= k, k steps minimise ||b - A x|| over the Krylov
    space span{b, Ab, ..., A^{k-1} b} (x_0 = 0)."""
    A, b = _small_problem()
    for k in (1, 3, 6):
        res = fgmres(lambda x: A @ x, b, lambda v: v, tol=0.0, restart=10, max_iter=k)
        K = np.empty((b.size, k))
        v = b.copy()
        for i in range(k):
            K[:, i] = v
            v = A @ v
        Q, _ = np.linalg.qr(K)
        y, *_ = np.linalg.lstsq(A @ Q, b, rcond=None)
        best = np.linalg.norm(b - A @ Q @ y)
        got = np.linalg.norm(b - A @ res.x)
        assert abs(got - best) <= 1e-9 * np.linalg.norm(b)


def test_exact_preconditioner_one_step():
    A, b = _small_problem(seed=21)
    Ainv = np.linalg.inv(A)
    res = fgmres(lambda x: A @ x, b, lambda v: Ainv @ v, tol=1e-12, restart=10)
    assert res.iterations == 1 and res.converged
    np.testing.assert_allclose(res.x, np.linalg.solve(A, b), rtol=1e-10)


def test_zero_rhs_returns_zero():
    A, b = _small_problem()
    res = fgmres(lambda x: A @ x, np.zeros_like(b), lambda v: v, x0=np.ones_like(b))
    assert res.iterations == 0 and res.converged and not res.x.any()


def test_fixed_step_count_across_restarts():
    p = make_config(1, n=8)
    res = solve_poisson(p.a, p.f, p.h, p.phi_bot, p.phi_top, tol=0.0, max_iter=13, restart=5)
    assert res.iterations == 13 and res.restarts == 2 and len(res.res_hist) == 14
    # estimates never increase within a cycle (minimal residual)
    h = res.res_hist
    for cyc in range(3):
        seg = h[1 + 5 * cyc: 1 + 5 * cyc + 5]
        assert all(seg[i + 1] <= seg[i] * (1 + 1e-12) for i in range(len(seg) - 1))


def test_max_iter_exhausted_reports_not_converged():
    p = make_config(3, n=16)
    res = solve_poisson(p.a, p.f, p.h, p.phi_bot, p.phi_top, tol=1e-14, max_iter=2)
    assert not res.converged and res.iterations == 2 and res.true_relres > 1e-14


def test_constant_coefficient_solution_within_residual_bound():
    """Against the exact spectral solution (P2): ||phi - phi*|| <=
    ||b - A phi|| / lambda_min."""
    p = make_config(1)  # 64^3, a = 1
    res = solve_poisson(p.a, p.f, p.h, p.phi_bot, p.phi_top, tol=1e-8)
    assert res.converged
    b = rhs(p.f, p.a, p.h, p.phi_bot, p.phi_top)
    exact = spectral_solve(b, p.h)
    lam_min = spectral_eigenvalues(p.a.shape, p.h).min()
    r = np.linalg.norm(b - apply_operator(res.x, p.a, p.h))
    assert np.linalg.norm(res.x - exact) <= r / lam_min * (1 + 1e-6)
    assert res.true_relres < 1e-8


def test_mixed_precision_preconditioner_reaches_fp64_tolerance():
    p = make_config(1, n=32)
    r64 = solve_poisson(p.a, p.f, p.h, p.phi_bot, p.phi_top, tol=1e-8)
    r32 = solve_poisson(p.a, p.f, p.h, p.phi_bot, p.phi_top, tol=1e-8, precision="mixed")
    assert r32.converged and r32.true_relres < 1e-8
    assert r32.iterations <= r64.iterations + 1
    b = rhs(p.f, p.a, p.h, p.phi_bot, p.phi_top)
    lam_min = spectral_eigenvalues(p.a.shape, p.h).min()
    bound = (r64.true_relres + r32.true_relres) * np.linalg.norm(b) / lam_min
    assert np.linalg.norm(r32.x - r64.x) <= bound


@pytest.mark.parametrize("cold", ["vcycle", "fmg"])
def test_iterations_do_not_grow_with_refinement(cold):
    """Sec. 5.3: the iteration count does not increase as the mesh is refined
    (with the full multigrid cycle: stays within one step)."""
    its = [solve_poisson(*(lambda p: (p.a, p.f, p.h, p.phi_bot, p.phi_top))(make_config(1, n=n)),
                         cold=cold).iterations
           for n in (16, 32, 64)]
    assert max(its) - min(its) <= 1, its
    if cold == "vcycle":
        assert its[-1] <= its[0], its


@pytest.mark.slow
def test_warm_started_steps_take_at_most_four_iterations():
    """P8: after the first step, warm-started solves need 2 to 4 iterations
    (Sec. 5.3, Fig. fstep) at the paper's mild coefficient contrast
    (max(a) <= about 2 for its physical P)."""
    prev = None
    its = []
    for step in range(4):
        p = config_two_filaments(64, a_max=2.0, step=step)
        res = solve_poisson(p.a, p.f, p.h, p.phi_bot, p.phi_top, tol=1e-8, x0=prev)
        assert res.converged
        its.append(res.iterations)
        prev = res.x
    assert all(2 <= k <= 4 for k in its[1:]), its


def test_cold_start_fmg_preconditioner():
    """Sec. 3.2: a solve without an initial guess uses the FMG cycle as its
    preconditioner; it reaches the same tolerance in fewer steps than the
    V-cycle on the filament workload, and a warm-started solve keeps the
    V-cycle whatever the option."""
    p = make_config(3, n=32)
    rv = solve_poisson(p.a, p.f, p.h, p.phi_bot, p.phi_top, tol=1e-8, cold="vcycle")
    rf = solve_poisson(p.a, p.f, p.h, p.phi_bot, p.phi_top, tol=1e-8, cold="fmg")
    assert rv.converged and rf.converged and rf.iterations < rv.iterations
    b = rhs(p.f, p.a, p.h, p.phi_bot, p.phi_top)
    assert np.linalg.norm(b - apply_operator(rf.x, p.a, p.h)) < 1e-8 * np.linalg.norm(b)
    x0 = 0.5 * rv.x
    w1 = solve_poisson(p.a, p.f, p.h, p.phi_bot, p.phi_top, tol=1e-8, x0=x0, cold="vcycle")
    w2 = solve_poisson(p.a, p.f, p.h, p.phi_bot, p.phi_top, tol=1e-8, x0=x0, cold="fmg")
    assert w1.iterations == w2.iterations and np.array_equal(w1.x, w2.x)


def test_warm_start_with_fmg_preconditioner_is_the_residual_equation_solve():
    """With warm = "fmg" a warm-started solve preconditions with the full
    multigrid cycle.  FGMRES from x0 builds its Krylov space from r0 = b -
    A x0, so it equals x0 plus FGMRES from zero on A e = r0 with the same
    preconditioner and the tolerance rescaled to ||b|| (same iterations, same
    iterate to rounding); on the two-filament time loop (max(a) = 1e4) it
    needs fewer steps than the V-cycle."""
    from oracle.fgmres import fgmres
    from oracle.multigrid import build_hierarchy, fmg
    p0 = config_two_filaments(32, step=0)
    x0 = solve_poisson(p0.a, p0.f, p0.h, p0.phi_bot, p0.phi_top, tol=1e-8).x
    p = config_two_filaments(32, step=1)
    wf = solve_poisson(p.a, p.f, p.h, p.phi_bot, p.phi_top, tol=1e-8, x0=x0, warm="fmg")
    wv = solve_poisson(p.a, p.f, p.h, p.phi_bot, p.phi_top, tol=1e-8, x0=x0)
    assert wf.converged and wv.converged and wf.iterations < wv.iterations
    b = rhs(p.f, p.a, p.h, p.phi_bot, p.phi_top)
    r0 = b - apply_operator(x0, p.a, p.h)
    hier = build_hierarchy(p.a, p.h)
    e = fgmres(lambda x: apply_operator(x, p.a, p.h), r0, lambda v: fmg(hier, v),
               tol=1e-8 * np.linalg.norm(b) / np.linalg.norm(r0))
    assert e.iterations == wf.iterations
    np.testing.assert_allclose(x0 + e.x, wf.x, rtol=0, atol=1e-10 * np.abs(wf.x).max())
