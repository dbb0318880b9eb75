"""Pins of the oracle's multigrid preconditioner (Sec. 3.2, Appendix A)."""
import numpy as np
import pytest

from oracle.operator import assemble_dense, face_coefficients, apply_faces
from oracle.multigrid import (build_hierarchy, coarsen_faces, level_shapes,
                              prolong, rbgs_half_sweep, restrict, restrict_transpose, vcycle)


def test_level_shapes():
    assert level_shapes((64, 64, 64))[-1] == (2, 2, 2)
    assert len(level_shapes((64, 64, 64))) == 6
    s768 = level_shapes((768, 768, 768))
    assert len(s768) == 9 and s768[-1] == (3, 3, 3)
    assert level_shapes((256, 256, 320))[-1] == (4, 4, 5)
    assert level_shapes((512, 512, 512))[-1] == (2, 2, 2)
    assert level_shapes((3, 5, 7)) == [(3, 5, 7)]
    with pytest.raises(ValueError):
        level_shapes((100, 100, 100))  # -> 25^3 = 15625 > 4096


def _pc_prolongation(shape_zyx):
    """Piecewise-constant prolongation matrix (fine x coarse)."""
    nz, ny, nx = shape_zyx
    nc = (nz // 2) * (ny // 2) * (nx // 2)
    P = np.zeros((nz * ny * nx, nc))
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                P[(k * ny + j) * nx + i, ((k // 2) * (ny // 2) + j // 2) * (nx // 2) + i // 2] = 1.0
    return P


@pytest.mark.parametrize("shape", [(4, 4, 4), (6, 4, 8), (2, 4, 2)])
def test_coarse_operator_is_half_galerkin(shape):
    """The face-averaged coarse operator equals (1/2) R A P with
    piecewise-constant P and R = P^T / 8 (mean of the 8 children)."""
    rng = np.random.default_rng(10)
    a = rng.uniform(0.01, 100.0, shape)
    h = (0.1, 0.2, 0.15)
    F = face_coefficients(a)
    A = assemble_dense(F, h)
    P = _pc_prolongation(shape)
    R = P.T / 8.0
    Ac = assemble_dense(coarsen_faces(F), tuple(2 * x for x in h))
    np.testing.assert_allclose(0.5 * R @ A @ P, Ac, rtol=1e-13, atol=1e-10)


def test_restriction_is_mean_of_children():
    rng = np.random.default_rng(11)
    r = rng.standard_normal((4, 6, 8))
    P = _pc_prolongation(r.shape)
    np.testing.assert_allclose(restrict(r).ravel(), P.T @ r.ravel() / 8.0, rtol=1e-14)


def _trilinear_bruteforce(c):
    """Fine values from explicit 8-point trilinear weights: per dimension 3/4
    on the parent and 1/4 on the nearer coarse neighbour; a neighbour outside
    the grid is replaced by the parent (x, y) or minus the parent (z)."""
    nz, ny, nx = c.shape
    out = np.zeros((2 * nz, 2 * ny, 2 * nx))
    for k in range(2 * nz):
        for j in range(2 * ny):
            for i in range(2 * nx):
                acc = 0.0
                for wz, kk in ((0.75, k // 2), (0.25, k // 2 + (1 if k % 2 else -1))):
                    for wy, jj in ((0.75, j // 2), (0.25, j // 2 + (1 if j % 2 else -1))):
                        for wx, ii in ((0.75, i // 2), (0.25, i // 2 + (1 if i % 2 else -1))):
                            s, k2, j2, i2 = 1.0, kk, jj, ii
                            if k2 < 0 or k2 >= nz:
                                k2, s = k // 2, -1.0
                            if j2 < 0 or j2 >= ny:
                                j2 = j // 2
                            if i2 < 0 or i2 >= nx:
                                i2 = i // 2
                            acc += wz * wy * wx * s * c[k2, j2, i2]
                out[k, j, i] = acc
    return out


def test_prolongation_weights():
    rng = np.random.default_rng(12)
    c = rng.standard_normal((3, 4, 2))
    np.testing.assert_allclose(prolong(c), _trilinear_bruteforce(c), rtol=1e-14, atol=1e-15)


def test_prolongation_reproduces_linear_fields():
    """Linear fields are interpolated exactly away from the boundary, and a
    field linear in z vanishing at the bottom plate exactly near that plate."""
    nc = 4
    cc = (np.arange(nc) + 0.5) / nc
    cf = (np.arange(2 * nc) + 0.5) / (2 * nc)
    Z, Y, X = np.meshgrid(cc, cc, cc, indexing="ij")
    Zf, Yf, Xf = np.meshgrid(cf, cf, cf, indexing="ij")
    e = prolong(2 * X - 3 * Y + 0.5 * Z)
    ref = 2 * Xf - 3 * Yf + 0.5 * Zf
    np.testing.assert_allclose(e[1:-1, 1:-1, 1:-1], ref[1:-1, 1:-1, 1:-1], atol=1e-14)
    ez = prolong(Z)
    np.testing.assert_allclose(ez[0], Zf[0], atol=1e-15)


def _gs_loop(x, b, faces, h, colour):
    """Sequential Gauss-Seidel over the cells of one colour, one cell at a
    time in lexicographic order, from the stencil written out per cell."""
    hx, hy, hz = h
    nz, ny, nx = x.shape
    x = x.copy()
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                if (i + j + k) % 2 != colour:
                    continue
                num, den = b[k, j, i], 0.0
                if i > 0:
                    w = faces.wx[k, j, i - 1] / hx ** 2
                    num += w * x[k, j, i - 1]
                    den += w
                if i < nx - 1:
                    w = faces.wx[k, j, i] / hx ** 2
                    num += w * x[k, j, i + 1]
                    den += w
                if j > 0:
                    w = faces.wy[k, j - 1, i] / hy ** 2
                    num += w * x[k, j - 1, i]
                    den += w
                if j < ny - 1:
                    w = faces.wy[k, j, i] / hy ** 2
                    num += w * x[k, j + 1, i]
                    den += w
                if k > 0:
                    w = faces.wz[k - 1, j, i] / hz ** 2
                    num += w * x[k - 1, j, i]
                    den += w
                else:
                    den += 2 * faces.bot[j, i] / hz ** 2
                if k < nz - 1:
                    w = faces.wz[k, j, i] / hz ** 2
                    num += w * x[k + 1, j, i]
                    den += w
                else:
                    den += 2 * faces.top[j, i] / hz ** 2
                x[k, j, i] = num / den
    return x


def test_gauss_seidel_half_sweep_matches_loop():
    rng = np.random.default_rng(13)
    shape = (5, 4, 3)
    a = rng.uniform(0.1, 10, shape)
    h = (0.3, 0.25, 0.2)
    hier = build_hierarchy(a, h, coarse_max_cells=10 ** 6)
    lev = hier.levels[0]
    x0 = rng.standard_normal(shape)
    b = rng.standard_normal(shape)
    for colour in (0, 1):
        got = rbgs_half_sweep(x0.copy(), b, lev, colour)
        np.testing.assert_allclose(got, _gs_loop(x0, b, lev.faces, h, colour), rtol=1e-13, atol=1e-13)


def test_symmetric_gauss_seidel_contracts_energy_norm():
    rng = np.random.default_rng(14)
    shape = (6, 6, 6)
    a = rng.uniform(0.01, 100, shape)
    h = (1 / 6,) * 3
    hier = build_hierarchy(a, h)
    lev = hier.levels[0]
    A = assemble_dense(lev.faces, h)
    b = np.zeros(shape)
    for _ in range(3):
        e = rng.standard_normal(shape)
        e1 = e.copy()
        for c in (0, 1, 1, 0):
            rbgs_half_sweep(e1, b, lev, c)
        assert e1.ravel() @ A @ e1.ravel() < e.ravel() @ A @ e.ravel()


def _matrix_of(fn, n, shape):
    M = np.zeros((n, n))
    u = np.zeros(shape)
    for c in range(n):
        u.flat[c] = 1.0
        M[:, c] = fn(u.copy()).ravel()
        u.flat[c] = 0.0
    return M


@pytest.mark.parametrize("restriction", ["mean", "transpose"])
def test_two_level_vcycle_matches_appendix_formula(restriction):
    """Appendix A: one two-level V-cycle from x = 0 is z = M_2 b with
    M_2 = Q P + P + Q P_{1,2} A_1^{-1} R_{2,1} (I - A_2 P), written with the
    separate pre- and post-smoothers: M = Q_post P_pre + P_post +
    Q_post P_{1,2} A_1^{-1} R_{2,1} (I - A_2 P_pre); R_{2,1} the mean of
    the 8 children or P_{1,2}^T / 8."""
    rng = np.random.default_rng(15)
    shape = (4, 4, 6)
    a = rng.uniform(0.05, 20.0, shape)
    h = (1 / 6, 1 / 4, 1 / 4)
    hier = build_hierarchy(a, h, nu_pre=2, nu_post=2, restriction=restriction)
    assert len(hier.levels) == 2
    lev, coarse = hier.levels
    n = a.size
    nc = n // 8
    A2 = assemble_dense(lev.faces, lev.h)
    A1 = assemble_dense(coarse.faces, coarse.h)
    zero = np.zeros(shape)

    def pre(b):
        x = np.zeros(shape)
        for _ in range(2):
            rbgs_half_sweep(x, b, lev, 0)
            rbgs_half_sweep(x, b, lev, 1)
        return x

    def post_map(x):  # smoother acting on x with b = 0: the Q_post factor
        for _ in range(2):
            rbgs_half_sweep(x, zero, lev, 1)
            rbgs_half_sweep(x, zero, lev, 0)
        return x

    def post_b(b):  # smoother from x = 0 with right side b: P_post
        x = np.zeros(shape)
        for _ in range(2):
            rbgs_half_sweep(x, b, lev, 1)
            rbgs_half_sweep(x, b, lev, 0)
        return x

    P_pre = _matrix_of(pre, n, shape)
    Q_post = _matrix_of(post_map, n, shape)
    P_post = _matrix_of(post_b, n, shape)
    # a consistent smoother: Q = I - P A
    np.testing.assert_allclose(Q_post, np.eye(n) - P_post @ A2, atol=1e-11)
    R = np.zeros((nc, n))
    P12 = np.zeros((n, nc))
    u = np.zeros(shape)
    for c in range(n):
        u.flat[c] = 1.0
        R[:, c] = restrict(u).ravel()
        u.flat[c] = 0.0
    uc = np.zeros((shape[0] // 2, shape[1] // 2, shape[2] // 2))
    for c in range(nc):
        uc.flat[c] = 1.0
        P12[:, c] = prolong(uc).ravel()
        uc.flat[c] = 0.0
    if restriction == "transpose":
        R = P12.T / 8.0
    I = np.eye(n)
    M_formula = (Q_post @ P_pre + P_post
                 + Q_post @ P12 @ np.linalg.solve(A1, R @ (I - A2 @ P_pre)))
    M_vcycle = _matrix_of(lambda b: vcycle(hier, b), n, shape)
    np.testing.assert_allclose(M_vcycle, M_formula, rtol=1e-10, atol=1e-12 * np.abs(M_formula).max())


def test_vcycle_is_linear_and_contracting():
    """P6: from x = 0 the V-cycle is a fixed linear map; as a stationary
    iteration x <- x + M (b - A x) it converges (spectral radius < 1)."""
    rng = np.random.default_rng(16)
    n = 8
    a = np.ones((n, n, n))
    h = (1 / n,) * 3
    hier = build_hierarchy(a, h)
    u, v = rng.standard_normal((2, n, n, n))
    np.testing.assert_allclose(vcycle(hier, 2 * u - 3 * v),
                               2 * vcycle(hier, u) - 3 * vcycle(hier, v), rtol=1e-12, atol=1e-14)
    A = assemble_dense(face_coefficients(a), h)
    M = _matrix_of(lambda b: vcycle(hier, b), n ** 3, (n, n, n))
    rho = np.max(np.abs(np.linalg.eigvals(np.eye(n ** 3) - M @ A)))
    assert rho < 0.15, rho


def test_single_level_vcycle_is_direct_solve():
    rng = np.random.default_rng(17)
    a = rng.uniform(0.5, 2, (3, 3, 3))
    h = (1 / 3,) * 3
    hier = build_hierarchy(a, h)
    assert len(hier.levels) == 1
    b = rng.standard_normal(a.shape)
    x = vcycle(hier, b)
    np.testing.assert_allclose(apply_faces(x, face_coefficients(a), h), b, rtol=1e-12, atol=1e-12)


# ---------------------------------------------------------------- full multigrid
def _interp_1d(n, dirichlet):
    """Dense 1-D cell-centred linear interpolation (2n x n): fine 2I is
    3/4 c_I + 1/4 c_{I-1}, fine 2I+1 is 3/4 c_I + 1/4 c_{I+1}; a ghost beyond
    an end is the end value (Neumann) or its negative (Dirichlet)."""
    P = np.zeros((2 * n, n))
    s = -1.0 if dirichlet else 1.0
    for I in range(n):
        P[2 * I, I] += 0.75
        P[2 * I + 1, I] += 0.75
        if I > 0:
            P[2 * I, I - 1] += 0.25
        else:
            P[2 * I, I] += 0.25 * s
        if I < n - 1:
            P[2 * I + 1, I + 1] += 0.25
        else:
            P[2 * I + 1, I] += 0.25 * s
    return P


def _mean_1d(n):
    """Dense 1-D pairing (n/2 x n): coarse I is the mean of fine 2I, 2I+1."""
    R = np.zeros((n // 2, n))
    for I in range(n // 2):
        R[I, 2 * I] = R[I, 2 * I + 1] = 0.5
    return R


def test_fmg_two_levels_closed_form():
    """Two levels: FMG gives x = x0 + M (b - A x0) with x0 = P A_1^{-1} R b
    (the coarse solution of the restricted right side, interpolated) and M
    the V-cycle from zero (eq. eRichard: a V-cycle from a guess is x0 plus M
    applied to the residual).  P, R and the coarse solve are formed here
    from their definitions (Kronecker products of 1-D matrices, a dense
    solve), not from the oracle's routines."""
    from oracle.multigrid import fmg
    rng = np.random.default_rng(21)
    shape = (6, 4, 10)  # (nz, ny, nx)
    a = rng.uniform(0.1, 10.0, shape)
    h = (1 / 10, 1 / 4, 1 / 6)
    hier = build_hierarchy(a, h)
    assert len(hier.levels) == 2
    nz, ny, nx = shape
    Pm = np.kron(_interp_1d(nz // 2, True), np.kron(_interp_1d(ny // 2, False), _interp_1d(nx // 2, False)))
    Rm = np.kron(_mean_1d(nz), np.kron(_mean_1d(ny), _mean_1d(nx)))
    A0 = assemble_dense(face_coefficients(a), h)
    coarse = hier.levels[1]
    A1 = assemble_dense(coarse.faces, coarse.h)
    b = rng.standard_normal(shape)
    x0 = Pm @ np.linalg.solve(A1, Rm @ b.ravel())
    want = x0 + vcycle(hier, (b.ravel() - A0 @ x0).reshape(shape)).ravel()
    np.testing.assert_allclose(fmg(hier, b).ravel(), want, rtol=1e-10, atol=1e-12 * np.abs(want).max())


def test_fmg_single_level_is_direct_solve_and_linear():
    from oracle.multigrid import fmg
    rng = np.random.default_rng(22)
    a = rng.uniform(0.5, 2, (3, 5, 7))
    h = (1 / 7, 1 / 5, 1 / 3)
    hier = build_hierarchy(a, h)
    assert len(hier.levels) == 1
    b = rng.standard_normal(a.shape)
    np.testing.assert_allclose(apply_faces(fmg(hier, b), face_coefficients(a), h), b, rtol=1e-12, atol=1e-12)
    a = rng.uniform(0.5, 2, (8, 8, 8))
    hier = build_hierarchy(a, (1 / 8,) * 3)
    u, v = rng.standard_normal((2, 8, 8, 8))
    np.testing.assert_allclose(fmg(hier, 2 * u - 3 * v), 2 * fmg(hier, u) - 3 * fmg(hier, v),
                               rtol=1e-12, atol=1e-13)


def test_fmg_error_shrinks_with_refinement():
    """The property FMG exists for: one cycle from no guess gives an
    algebraic error that stays at the size of the discretisation error as
    the grid is refined (relative error falling about like h^1.5 here),
    whereas one V-cycle from zero leaves a fixed fraction of the solution.
    Smooth manufactured solution with variable coefficient and homogeneous
    plates (b = f: a lifted plate term would be doubled by the mean-of-8
    restriction and spoil the coarse guess)."""
    from oracle.exact import manufactured, sparse_solve
    from oracle.multigrid import fmg
    from oracle.operator import rhs
    rel_fmg = []
    for n in (16, 32):
        phi, a, f = manufactured(n, 0.0)
        h = (1 / n,) * 3
        ph = sparse_solve(a, f, h, 0.0, 0.0)
        b = rhs(f, a, h, 0.0, 0.0)
        hier = build_hierarchy(a, h)
        disc = np.linalg.norm(ph - phi)
        alg_fmg = np.linalg.norm(fmg(hier, b) - ph)
        alg_v = np.linalg.norm(vcycle(hier, b) - ph)
        assert alg_fmg < 5 * disc, (n, alg_fmg, disc)
        assert alg_v > 10 * alg_fmg, (n, alg_v, alg_fmg)
        rel_fmg.append(alg_fmg / np.linalg.norm(ph))
    assert rel_fmg[0] < 0.015 and rel_fmg[1] < 0.5 * rel_fmg[0], rel_fmg


# ---------------------------------------------------------------- symmetric V-cycle
def test_transpose_restriction_is_the_kronecker_transpose():
    """restrict_transpose equals (P_z x P_y x P_x)^T / 8 with the 1-D
    interpolation matrices written out entry by entry (ghost rules:
    negated mirror through the plates in z, mirror on the sides)."""
    rng = np.random.default_rng(31)
    nz, ny, nx = 6, 4, 8
    r = rng.standard_normal((nz, ny, nx))
    P = np.kron(_interp_1d(nz // 2, True), np.kron(_interp_1d(ny // 2, False), _interp_1d(nx // 2, False)))
    want = (P.T @ r.ravel() / 8.0).reshape(nz // 2, ny // 2, nx // 2)
    np.testing.assert_allclose(restrict_transpose(r), want, rtol=1e-14, atol=1e-15)
    # and the prolongation is the same Kronecker product (the pair is consistent)
    c = rng.standard_normal((nz // 2, ny // 2, nx // 2))
    np.testing.assert_allclose(prolong(c).ravel(), P @ c.ravel(), rtol=1e-14, atol=1e-15)


def test_transpose_restriction_is_full_weighting_inside():
    """Away from the boundary R = P^T / 8 is the 4 x 4 x 4 full-weighting
    stencil (per dimension 1/8, 3/8, 3/8, 1/8), so a constant maps to the
    same constant and a linear field to its coarse-cell-centre value; at a
    plate the folded ghost (negated mirror) lowers the weight."""
    n = 8
    k, j, i = np.indices((n, n, n)).astype(float)
    lin = 0.3 * (i + 0.5) - 0.7 * (j + 0.5) + 1.1 * (k + 0.5)
    c = restrict_transpose(lin)
    K, J, I = np.indices((n // 2,) * 3).astype(float)
    want = 0.3 * (2 * I + 1) - 0.7 * (2 * J + 1) + 1.1 * (2 * K + 1)
    inner = (slice(1, -1),) * 3
    np.testing.assert_allclose(c[inner], want[inner], rtol=1e-13)
    one = restrict_transpose(np.ones((n, n, n)))
    np.testing.assert_allclose(one[1:-1], 1.0, rtol=1e-14)  # z-interior, sides folded with +
    # plate fold: the 1-D weights (3/4 - 1/4) + 3/4 + 1/4 = 3/2 instead of 2
    np.testing.assert_allclose(one[0], 0.75, rtol=1e-14)
    np.testing.assert_allclose(one[-1], 0.75, rtol=1e-14)


@pytest.mark.parametrize("shape", [(8, 8, 8), (4, 6, 8)])
def test_transpose_restriction_makes_the_vcycle_symmetric(shape):
    """With R = P^T / 8 and nu_pre = nu_post the V-cycle (pre red-black,
    post black-red) is a symmetric positive definite matrix (three levels at
    8^3, variable a); with the default mean-of-8 restriction it is not, and
    neither is it with nu_pre != nu_post (two planted asymmetries)."""
    rng = np.random.default_rng(32)
    a = np.exp(rng.uniform(-2.0, 2.0, shape))
    h = (1 / shape[2], 1 / shape[1], 1 / shape[0])
    n = a.size

    def mat(**kw):
        hier = build_hierarchy(a, h, **kw)
        return _matrix_of(lambda b: vcycle(hier, b), n, shape), len(hier.levels)

    M, nl = mat(nu_pre=2, nu_post=2, restriction="transpose")
    assert nl >= 2
    assert np.linalg.norm(M - M.T) <= 1e-13 * np.linalg.norm(M)
    assert np.linalg.eigvalsh(0.5 * (M + M.T)).min() > 0
    M1, _ = mat(nu_pre=1, nu_post=1, restriction="transpose")
    assert np.linalg.norm(M1 - M1.T) <= 1e-13 * np.linalg.norm(M1)
    Mm, _ = mat(nu_pre=2, nu_post=2, restriction="mean")
    assert np.linalg.norm(Mm - Mm.T) > 1e-3 * np.linalg.norm(Mm)
    Mu, _ = mat(nu_pre=2, nu_post=1, restriction="transpose")
    assert np.linalg.norm(Mu - Mu.T) > 1e-3 * np.linalg.norm(Mu)


def test_symmetric_vcycle_contracts():
    """The symmetric V-cycle is a convergent stationary iteration too
    (x <- x + M (b - A x)): spectral radius 0.20 at a = 1 and 0.32 at
    contrast e^4 on 8^3 (the mean-of-8 V-cycle: 0.14 and 0.25)."""
    n = 8
    h = (1 / n,) * 3
    rng = np.random.default_rng(33)
    for a, bound in ((np.ones((n, n, n)), 0.25), (np.exp(rng.uniform(-2.0, 2.0, (n, n, n))), 0.35)):
        hier = build_hierarchy(a, h, restriction="transpose")
        A = assemble_dense(face_coefficients(a), h)
        M = _matrix_of(lambda b: vcycle(hier, b), n ** 3, (n, n, n))
        rho = np.max(np.abs(np.linalg.eigvals(np.eye(n ** 3) - M @ A)))
        assert rho < bound, rho
