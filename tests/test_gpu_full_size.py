"""GPU solves at the workloads' own sizes, checked by the CPU oracle.

* The 256^3 filament workload (max(a) = 1e3) in float64 after a fixed number
  of steps equals the oracle's solve to 1e-10 in phi (the parity rule at the
  workload's real size, not a scaled-down copy).
* The 512^3 headline workload (max(a) = 1e4): the converged mixed and float64
  solutions are checked with the oracle's operator (true relative residual
  below 1e-8, reported within 0.1%), and their difference from the exact
  discrete solution is bounded by ||r|| / lambda_min (lambda_min of the a = 1
  operator bounds that of a >= 1 from below).
* Opt-in (GMG_FULL_ORACLE=1, about 30 GB of host memory and several minutes):
  the oracle's own float64 solve at 512^3 with the benchmark's solver
  settings; the GPU float64 solve after the same number of steps matches it to
  1e-10, and the converged mixed and float64 solutions are compared with it.
"""
import os
import sys
import time

import numpy as np
import pytest
import torch

from oracle.exact import spectral_eigenvalues
from oracle.fgmres import fgmres, solve_poisson
from oracle.multigrid import build_hierarchy, fmg
from oracle.operator import apply_operator, rhs
from workloads import make_config

pytestmark = pytest.mark.gpu

import paper_1812_08606_amd as gm  # noqa: E402  (fails loudly if the library is missing)

DEV = torch.device("cuda:0")


def T(x):
    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device=DEV)


def npy(t):
    return t.detach().cpu().numpy()


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def say(msg):
    print(msg, file=sys.stderr, flush=True)


def lambda_min_unit(shape_zyx, h):
    """Smallest eigenvalue of the a = 1 operator (DST-II in z, constant mode
    in x and y): a lower bound of that of any a >= 1."""
    return spectral_eigenvalues((shape_zyx[0], 1, 1), (h[0], h[1], h[2])).min()


@pytest.mark.slow
def test_config2_full_size_fp64_fixed_steps_match_oracle():
    """Filament workload at its own 256^3, float64, 3 FGMRES steps with full
    multigrid cycles (the cold-start default) from tol = 0: phi within 1e-10
    of the oracle's, residual histories within 1e-6."""
    p = make_config(2)
    assert p.a.shape == (256, 256, 256)
    k = 3
    say("config 2 at 256^3: GPU fp64, 3 steps")
    s = gm.GMGPoisson(T(p.a), precision="fp64", max_iter=k)
    res = s.solve(T(p.f), p.phi_bot, p.phi_top, tol=0.0)
    say("config 2 at 256^3: oracle fp64, 3 steps")
    t0 = time.perf_counter()
    ref = solve_poisson(p.a, p.f, p.h, p.phi_bot, p.phi_top, tol=0.0, max_iter=k)
    err = rel(npy(res.phi), ref.x)
    say(f"config 2 at 256^3: oracle {time.perf_counter() - t0:.0f} s; |phi_gpu - phi_oracle| / |phi_oracle| = "
        f"{err:.2e}; histories {res.res_hist} / {ref.res_hist}")
    assert res.iterations == ref.iterations == k
    assert err < 1e-10
    np.testing.assert_allclose(res.res_hist, ref.res_hist, rtol=1e-6, atol=1e-15)


@pytest.mark.slow
def test_config3_full_size_converged_solutions_checked_by_oracle_operator():
    """Headline workload at 512^3 (max(a) = 1e4), solved from zero to 1e-8
    with the benchmark's solver (full multigrid cycles, 2 pre- and 3
    post-smoothing sweeps), mixed and float64: the oracle's operator gives a
    true relative residual below 1e-8 that matches the reported one within
    0.1%; the two solutions differ by no more than the residual bound, and
    each lies within ||r|| / lambda_min of the exact discrete solution."""
    p = make_config(3, n=512)
    b = rhs(p.f, p.a, p.h, p.phi_bot, p.phi_top)
    bn = np.linalg.norm(b)
    lam = lambda_min_unit(p.a.shape, p.h)
    a_d, f_d = T(p.a), T(p.f)
    phis, rn = {}, {}
    for precision in ("mixed", "fp64"):
        s = gm.GMGPoisson(a_d, precision=precision, nu_pre=2, nu_post=3)
        res = s.solve(f_d, p.phi_bot, p.phi_top, tol=1e-8)
        phi, reported = npy(res.phi), res.final_relres
        del s, res
        torch.cuda.empty_cache()
        r = np.linalg.norm(b - apply_operator(phi, p.a, p.h))
        phis[precision], rn[precision] = phi, r
        say(f"512^3 {precision}: true relres {r / bn:.3e} (reported {reported:.3e}); bound on |phi - phi*| / |phi| "
            f"{r / lam / np.linalg.norm(phi):.2e}")
        assert r < 1e-8 * bn
        assert abs(r / bn - reported) <= 1e-3 * r / bn
    d = np.linalg.norm(phis["mixed"] - phis["fp64"])
    say(f"512^3: |phi_mixed - phi_fp64| / |phi_fp64| = {d / np.linalg.norm(phis['fp64']):.2e} "
        f"(bound {(rn['mixed'] + rn['fp64']) / lam / np.linalg.norm(phis['fp64']):.2e})")
    assert d <= (rn["mixed"] + rn["fp64"]) / lam


@pytest.mark.slow
@pytest.mark.skipif(os.environ.get("GMG_FULL_ORACLE") != "1",
                    reason="opt-in: the oracle's own 512^3 solve needs about 30 GB of host memory and several "
                           "minutes (set GMG_FULL_ORACLE=1)")
def test_config3_full_size_against_oracle_solve():
    """The oracle's float64 solve of the 512^3 headline workload with the
    benchmark's solver (full multigrid cycles, V(2,3)), stopped after the
    steps the GPU takes to reach 1e-8: the GPU float64 solve after the same
    steps equals it to 1e-10; the converged mixed and float64 GPU solutions
    are compared with it."""
    p = make_config(3, n=512)
    a_d, f_d = T(p.a), T(p.f)
    out = {}
    for precision in ("mixed", "fp64"):
        s = gm.GMGPoisson(a_d, precision=precision, nu_pre=2, nu_post=3)
        res = s.solve(f_d, p.phi_bot, p.phi_top, tol=1e-8)
        out[precision] = (npy(res.phi), res.iterations)
        del s, res
        torch.cuda.empty_cache()
    k = out["fp64"][1]
    s = gm.GMGPoisson(a_d, precision="fp64", nu_pre=2, nu_post=3, max_iter=k)
    fixed = s.solve(f_d, p.phi_bot, p.phi_top, tol=0.0)
    phi_fixed, hist_fixed = npy(fixed.phi), fixed.res_hist
    del s, fixed, a_d, f_d
    torch.cuda.empty_cache()
    say(f"512^3 oracle fp64 solve, {k} steps (FMG, V(2,3)) ...")
    t0 = time.perf_counter()
    hier = build_hierarchy(p.a, p.h, nu_pre=2, nu_post=3)
    b = rhs(p.f, p.a, p.h, p.phi_bot, p.phi_top)
    step = [0]

    def A(x):
        return apply_operator(x, p.a, p.h)

    def M(v):
        step[0] += 1
        say(f"  oracle step {step[0]} at {time.perf_counter() - t0:.0f} s")
        return fmg(hier, v)

    ref = fgmres(A, b, M, tol=0.0, max_iter=k)
    say(f"oracle: {time.perf_counter() - t0:.0f} s, true relres {ref.true_relres:.3e}")
    e_fixed = rel(phi_fixed, ref.x)
    e_mixed = rel(out["mixed"][0], ref.x)
    e_fp64 = rel(out["fp64"][0], ref.x)
    say(f"512^3: fp64 after {k} steps vs oracle {e_fixed:.2e}; converged mixed ({out['mixed'][1]} steps) vs "
        f"oracle {e_mixed:.2e}; converged fp64 ({k} steps) vs oracle {e_fp64:.2e}")
    assert e_fixed < 1e-10
    np.testing.assert_allclose(hist_fixed, ref.res_hist, rtol=1e-6, atol=1e-15)
    assert ref.true_relres < 1e-8
    # both converged GPU solutions lie within the residual bound of the oracle's
    lam = lambda_min_unit(p.a.shape, p.h)
    bn = np.linalg.norm(b)
    for precision in ("mixed", "fp64"):
        r = np.linalg.norm(b - A(out[precision][0]))
        assert np.linalg.norm(out[precision][0] - ref.x) <= (r + ref.true_relres * bn) / lam
