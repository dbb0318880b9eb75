"""fgmres_solve_static: the solve on the library's per-GPU device array,
for callers that cannot allocate device memory.  Called through the C ABI
(ctypes) and checked against fgmres_solve on a caller-allocated workspace:
the same kernels on the same data, so the results agree to the last bit;
two calls in a row, the second on a smaller grid (the array keeps the first
call's contents), and a grid too large for the array is refused before
anything runs."""
import ctypes

import numpy as np
import pytest
import torch

from oracle.fgmres import solve_poisson
from workloads import make_config

pytestmark = pytest.mark.gpu

import paper_1812_08606_amd as gm  # noqa: E402  (fails loudly if the library is missing)
from paper_1812_08606_amd import _lib  # noqa: E402

DEV = torch.device("cuda:0")


def T(x):
    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device=DEV)


def _static_solve(lib, p, a, f, phi, precision, tol, max_iter=200):
    nz, ny, nx = p.a.shape
    opt = _lib.Options()
    lib.gmg_default_options(ctypes.byref(opt))
    opt.precision = gm.MIXED if precision == "mixed" else gm.FP64
    opt.max_iter = max_iter
    cap = max_iter + 2
    hist = (ctypes.c_double * cap)()
    its, nh = ctypes.c_int(0), ctypes.c_int(0)
    rel = ctypes.c_double(float("nan"))
    stream = torch.cuda.current_stream(DEV).cuda_stream
    st = lib.fgmres_solve_static(nx, ny, nz, *p.h, ctypes.c_void_p(a.data_ptr()), ctypes.byref(opt),
                                 ctypes.c_void_p(stream), ctypes.c_void_p(f.data_ptr()), p.phi_bot, p.phi_top, tol,
                                 ctypes.c_void_p(phi.data_ptr()), 0, ctypes.byref(its), hist, cap, ctypes.byref(nh),
                                 ctypes.byref(rel))
    return st, its.value, list(hist[:nh.value]), rel.value


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_static_solve_equals_workspace_solve_twice_second_smaller(precision):
    lib = _lib.load()
    for cfg, n in ((3, 48), (2, 32)):
        print(f"static solve {precision} workload {cfg} n={n}", flush=True)
        p = make_config(cfg, n=n)
        a, f = T(p.a), T(p.f)
        ref = gm.GMGPoisson(a, precision=precision).solve(f, p.phi_bot, p.phi_top, tol=1e-8)
        phi = torch.full_like(a, float("nan"))
        st, its, hist, rel = _static_solve(lib, p, a, f, phi, precision, 1e-8)
        assert st == gm.solver.OK and its == ref.iterations
        assert torch.equal(phi, ref.phi)
        assert hist == ref.res_hist and rel == ref.final_relres
    # float64 at a fixed step count against the oracle (the parity bar)
    p = make_config(2, n=32)
    k = 4
    phi = torch.empty(p.a.shape, dtype=torch.float64, device=DEV)
    st, its, _, _ = _static_solve(lib, p, T(p.a), T(p.f), phi, "fp64", 0.0, max_iter=k)
    ora = solve_poisson(p.a, p.f, p.h, p.phi_bot, p.phi_top, tol=0.0, max_iter=k)
    assert st == gm.solver.NOT_CONVERGED and its == k
    assert np.linalg.norm(phi.cpu().numpy() - ora.x) / np.linalg.norm(ora.x) < 1e-10


def test_static_solve_rejects_a_grid_beyond_the_array():
    """128^3 in mixed precision needs about 295 MiB of workspace, more than
    the 64 MiB array: GMG_ERR_WORKSPACE before anything runs (phi untouched)."""
    lib = _lib.load()
    n = 128
    opt = _lib.Options()
    lib.gmg_default_options(ctypes.byref(opt))
    assert lib.gmg_workspace_bytes(n, n, n, ctypes.byref(opt)) > gm.solver.STATIC_SCRATCH_BYTES
    a = torch.ones((n, n, n), dtype=torch.float64, device=DEV)
    f = torch.ones_like(a)
    phi = torch.full_like(a, 7.0)
    p = type("P", (), {"a": np.empty((n, n, n)), "h": (1 / n,) * 3, "phi_bot": 0.0, "phi_top": 1.0})
    st, _, _, _ = _static_solve(lib, p, a, f, phi, "mixed", 1e-8)
    assert st == -4
    assert bool((phi == 7.0).all())
    with pytest.raises(gm.GMGError) as e:
        gm.fgmres_solve_static(a, f, 0.0, 1.0, 1e-8, out=phi)
    assert e.value.status == -4


def test_static_solve_python_binding_and_graphs_refused():
    p = make_config(1, n=32)
    a, f = T(p.a), T(p.f)
    out = torch.empty_like(a)
    res = gm.fgmres_solve_static(a, f, p.phi_bot, p.phi_top, 1e-8, out=out, precision="fp64")
    ref = gm.GMGPoisson(a, precision="fp64").solve(f, p.phi_bot, p.phi_top, tol=1e-8)
    assert res.converged and torch.equal(res.phi, ref.phi)
    with pytest.raises(gm.GMGError) as e:
        gm.fgmres_solve_static(a, f, p.phi_bot, p.phi_top, 1e-8, out=out, graphs=1)
    assert e.value.status == -1
