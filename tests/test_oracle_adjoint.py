"""Pins of the oracle's adjoint gradient (derived from eq. e18) against a
dense autograd solve and against finite differences (P10)."""
import numpy as np
import torch

from oracle.adjoint import coefficient_gradient, solve_and_gradient
from oracle.exact import sparse_solve
from oracle.operator import rhs
from workloads import make_config


def _overlap_box_mask(n, box=((0.4, 0.6), (0.4, 0.6), (0.45, 0.55))):
    """Cells overlapping the probe box (at 8^3 no cell centre lies inside its
    z-range, so the small copy uses the overlap rule)."""
    e = np.arange(n + 1) / n
    masks = []
    for lo, hi in box:
        masks.append((e[1:] > lo) & (e[:-1] < hi))
    mx, my, mz = masks
    return mz[:, None, None] & my[None, :, None] & mx[None, None, :]


def _grad_loss_torch(phi, mask, h):
    """L = sum over the mask of |grad phi|^2 h^3, central differences."""
    L = phi.new_zeros(())
    idx = torch.nonzero(torch.as_tensor(mask))
    k, j, i = idx[:, 0], idx[:, 1], idx[:, 2]
    gx = (phi[k, j, i + 1] - phi[k, j, i - 1]) / (2 * h)
    gy = (phi[k, j + 1, i] - phi[k, j - 1, i]) / (2 * h)
    gz = (phi[k + 1, j, i] - phi[k - 1, j, i]) / (2 * h)
    return ((gx ** 2 + gy ** 2 + gz ** 2) * h ** 3).sum()


def _dense_torch_solve(a, f, h, pb, pt):
    """phi = A(a)^{-1} (f + lifting(a)) assembled densely in torch (autograd
    through a and f)."""
    nz, ny, nx = a.shape
    n = nz * ny * nx
    af = a.reshape(-1)
    idx = torch.arange(n).reshape(nz, ny, nx)
    A = torch.zeros(n, n, dtype=a.dtype)
    for axis, hd in ((2, h[0]), (1, h[1]), (0, h[2])):
        m = a.shape[axis]
        lo = idx.narrow(axis, 0, m - 1).reshape(-1)
        hi = idx.narrow(axis, 1, m - 1).reshape(-1)
        c = 0.5 * (af[lo] + af[hi]) / hd ** 2
        A = A.index_put((lo, lo), c, accumulate=True)
        A = A.index_put((hi, hi), c, accumulate=True)
        A = A.index_put((lo, hi), -c, accumulate=True)
        A = A.index_put((hi, lo), -c, accumulate=True)
    bot = idx[0].reshape(-1)
    top = idx[-1].reshape(-1)
    A = A.index_put((bot, bot), 2 * af[bot] / h[2] ** 2, accumulate=True)
    A = A.index_put((top, top), 2 * af[top] / h[2] ** 2, accumulate=True)
    b = f.reshape(-1).clone()
    b = b.index_put((bot,), 2 * af[bot] * pb / h[2] ** 2, accumulate=True)
    b = b.index_put((top,), 2 * af[top] * pt / h[2] ** 2, accumulate=True)
    return torch.linalg.solve(A, b).reshape(nz, ny, nx)


def test_adjoint_gradient_matches_dense_autograd():
    n = 8
    p = make_config(4, n=n)  # the gradient workload's generators at 8^3
    mask = _overlap_box_mask(n)
    h = p.h[0]
    a_t = torch.tensor(p.a, requires_grad=True)
    f_t = torch.tensor(p.f, requires_grad=True)
    phi_t = _dense_torch_solve(a_t, f_t, p.h, p.phi_bot, p.phi_top)
    L = _grad_loss_torch(phi_t, mask, h)
    L.backward()
    # dL/dphi from the loss alone, at the oracle's phi
    phi_o = sparse_solve(p.a, p.f, p.h, p.phi_bot, p.phi_top)
    phi_leaf = torch.tensor(phi_o, requires_grad=True)
    _grad_loss_torch(phi_leaf, mask, h).backward()
    gphi = phi_leaf.grad.numpy()
    phi, lam, dLda, fwd, adj = solve_and_gradient(p.a, p.f, p.h, p.phi_bot, p.phi_top, gphi, tol=1e-13)
    assert fwd.converged and adj.converged
    scale_f = np.abs(f_t.grad.numpy()).max()
    scale_a = np.abs(a_t.grad.numpy()).max()
    np.testing.assert_allclose(lam, f_t.grad.numpy(), atol=1e-9 * scale_f)
    np.testing.assert_allclose(dLda, a_t.grad.numpy(), atol=1e-8 * scale_a)


def test_adjoint_gradient_matches_finite_differences():
    """Central differences of a linear functional L = <g, phi> with exact
    (sparse direct) re-solves; relative step 1e-6."""
    rng = np.random.default_rng(30)
    shape = (5, 4, 6)
    a = rng.uniform(0.5, 50.0, shape)
    f = rng.standard_normal(shape)
    h = (1 / 6, 1 / 4, 1 / 5)
    pb, pt = 0.3, 1.7
    g = rng.standard_normal(shape)
    phi = sparse_solve(a, f, h, pb, pt)
    lam = sparse_solve(a, g, h, 0.0, 0.0)
    grad = coefficient_gradient(phi, lam, h, pb, pt)
    for c in rng.choice(a.size, 12, replace=False):
        d = 1e-6 * a.flat[c]
        ap, am = a.copy(), a.copy()
        ap.flat[c] += d
        am.flat[c] -= d
        fd = (np.vdot(g, sparse_solve(ap, f, h, pb, pt)) - np.vdot(g, sparse_solve(am, f, h, pb, pt))) / (2 * d)
        assert abs(fd - grad.flat[c]) <= 1e-6 * np.abs(grad).max(), (c, fd, grad.flat[c])
    # dL/df = lambda
    for c in rng.choice(a.size, 4, replace=False):
        d = 1e-3
        fp, fm = f.copy(), f.copy()
        fp.flat[c] += d
        fm.flat[c] -= d
        fd = (np.vdot(g, sparse_solve(a, fp, h, pb, pt)) - np.vdot(g, sparse_solve(a, fm, h, pb, pt))) / (2 * d)
        assert abs(fd - lam.flat[c]) <= 1e-9 * np.abs(lam).max()
    # lifting enters through b: rhs() consistent with the solve
    assert np.allclose(rhs(f, a, h, pb, pt) - f, rhs(np.zeros_like(f), a, h, pb, pt))
