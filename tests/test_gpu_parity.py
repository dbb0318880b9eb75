"""GPU path (HIP library through the C ABI) against the CPU oracle.

FP64: element-wise relative agreement 1e-10 in phi at a fixed step count
(tol = 0, max_iter = k), 1e-12..1e-13 for the single operations.  Mixed
precision: the float32 V-cycle against the oracle's float32 V-cycle, and the
converged phi against the FP64 oracle within the residual bound."""
import numpy as np
import pytest
import torch

from oracle.adjoint import coefficient_gradient
from oracle.exact import spectral_eigenvalues
from oracle.fgmres import solve_poisson
from oracle.multigrid import build_hierarchy, fmg, vcycle
from oracle.operator import apply_operator, rhs
from workloads import config_streamer_mesh, make_config

pytestmark = pytest.mark.gpu

import paper_1812_08606_amd as gm  # noqa: E402  (fails loudly if the library is missing)
DEV = torch.device("cuda:0")


def T(x):
    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device=DEV)


def npy(t):
    return t.detach().cpu().numpy()


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _rand_problem(shape_xyz, seed, contrast=1e2):
    nx, ny, nz = shape_xyz
    rng = np.random.default_rng(seed)
    a = np.exp(rng.uniform(-0.5, 0.5, (nz, ny, nx)) * np.log(contrast))
    f = rng.standard_normal((nz, ny, nx))
    h = (1.0 / nx, 1.3 / ny, 0.9 / nz)
    return a, f, h


# shapes (nx, ny, nz): ragged x tail, odd sizes, single-level grids, several
# coarsening levels
OP_SHAPES = [(70, 12, 8), (5, 3, 2), (1, 1, 1), (33, 17, 7), (128, 4, 6), (64, 64, 64)]
VC_SHAPES = [(48, 40, 36), (70, 12, 8), (64, 64, 64), (6, 4, 10), (3, 5, 7), (130, 8, 4)]


@pytest.mark.parametrize("shape", OP_SHAPES)
def test_operator_matches_oracle(shape):
    print(f"operator {shape}", flush=True)
    a, f, h = _rand_problem(shape, 1)
    rng = np.random.default_rng(2)
    x = rng.standard_normal(a.shape)
    s = gm.GMGPoisson(T(a), h=h, precision="fp64")
    y = npy(s.apply(T(x), 0.3, -1.2))
    ref = apply_operator(x, a, h, 0.3, -1.2)
    np.testing.assert_allclose(y, ref, rtol=1e-12, atol=1e-13 * np.abs(ref).max())


@pytest.mark.parametrize("shape", VC_SHAPES)
def test_vcycle_fp64_matches_oracle(shape):
    print(f"vcycle fp64 {shape}", flush=True)
    a, f, h = _rand_problem(shape, 3)
    s = gm.GMGPoisson(T(a), h=h, precision="fp64")
    hier = build_hierarchy(a, h, nu_pre=2, nu_post=2)
    assert [tuple(l.shape) for l in hier.levels] == s.levels
    z = npy(s.vcycle(T(f)))
    ref = vcycle(hier, f)
    assert rel(z, ref) < 1e-12
    np.testing.assert_allclose(z, ref, rtol=1e-9, atol=1e-12 * np.abs(ref).max())


@pytest.mark.parametrize("shape", VC_SHAPES)
def test_vcycle_mixed_matches_float32_oracle(shape):
    print(f"vcycle mixed {shape}", flush=True)
    a, f, h = _rand_problem(shape, 4)
    s = gm.GMGPoisson(T(a), h=h, precision="mixed")
    hier = build_hierarchy(a, h, nu_pre=2, nu_post=2, dtype=np.float32)
    z = npy(s.vcycle(T(f)))
    ref = vcycle(hier, f.astype(np.float32)).astype(np.float64)
    assert rel(z, ref) < 2e-5


@pytest.mark.parametrize("shape", [(64, 32, 48), (130, 8, 4), (66, 10, 12), (256, 12, 8), (200, 40, 48)])
@pytest.mark.parametrize("sweep", ["half", "fused"])
def test_vcycle_colour_split_finest_level(shape, sweep):
    """The finest level's colour-split kernels (several wave rows and block
    tiles, ragged last wave and tile, thin grids), with one kernel per
    half-sweep or one per symmetric sweep (the last pre-smoothing one also
    restricting the residual), give the oracle's V-cycle."""
    print(f"vcycle colour-split {shape} {sweep}", flush=True)
    a, f, h = _rand_problem(shape, 6)
    s64 = gm.GMGPoisson(T(a), h=h, precision="fp64", fine_sweep=sweep)
    assert rel(npy(s64.vcycle(T(f))), vcycle(build_hierarchy(a, h), f)) < 1e-12
    s32 = gm.GMGPoisson(T(a), h=h, precision="mixed", fine_sweep=sweep)
    s32.profile(True)
    z = npy(s32.vcycle(T(f)))
    names = set(s32.profile_read())
    s32.profile(False)
    assert ("sym_fine_f32" in names) == (sweep == "fused") and ("gs_fine_f32" in names) == (sweep == "half")
    assert ("sym_resid_fine_f32" in names) == (sweep == "fused") != ("resid_restrict_fine_f32" in names)
    ref32 = vcycle(build_hierarchy(a, h, dtype=np.float32), f.astype(np.float32)).astype(np.float64)
    assert rel(z, ref32) < 2e-5


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
@pytest.mark.parametrize("n, fused_by_default", [(256, False), (512, True)])
def test_fused_and_half_sweeps_agree_full_size(n, fused_by_default, precision):
    """Filament workload at 256^3 and 512^3 (max(a) = 1e3, 1e4): the V-cycle
    with fused symmetric sweeps equals the one with half-sweep kernels to
    rounding (float32 or float64), and the default picks the fused kernel of
    the finest level only on the long-chunk grid (it fuses the sweeps of the
    coarse levels from 128^3 up, so it matches neither mode to the bit)."""
    print(f"fused vs half sweeps {n}^3 {precision}", flush=True)
    p = make_config(2 if n == 256 else 3, n=n)
    a, f = T(p.a), T(p.f)
    v = f / f.norm()
    z = {}
    fused_name = "sym_fine_f32" if precision == "mixed" else "sym_fine_f64"
    for sweep in ("half", "fused", "auto"):
        s = gm.GMGPoisson(a, precision=precision, fine_sweep=sweep)
        s.profile(True)
        z[sweep] = s.vcycle(v)
        names = set(s.profile_read())
        s.profile(False)
        assert (fused_name in names) == (sweep == "fused" or (sweep == "auto" and fused_by_default))
        del s
    d = ((z["fused"] - z["half"]).norm() / z["half"].norm()).item()
    print(f"  |z_fused - z_half| / |z_half| = {d:.2e}", flush=True)
    assert d < (1e-5 if precision == "mixed" else 1e-13)
    d_auto = ((z["auto"] - z["half"]).norm() / z["half"].norm()).item()
    assert d_auto < (1e-5 if precision == "mixed" else 1e-13)


# (nx, ny, nz) with coarse face levels above the bottom kernel: 512 x 32 x
# 48 (level 1 256 x 16 x 24: two-wave rows, three row tiles, the last
# ragged, three z-chunks; level 2 128 x 8 x 12: one-wave rows), 128 x 96 x
# 80 (levels 64 x 48 x 40 and 32 x 24 x 20), 768 x 32 x 24 and 1024 x 32 x
# 16 (level 1 with rows of 192 and 256 pairs: three- and four-wave rows in
# float32, half-sweeps in float64)
FACE_SHAPES = [(512, 32, 48), (128, 96, 80), (768, 32, 24), (1024, 32, 16)]


@pytest.mark.parametrize("shape", FACE_SHAPES)
@pytest.mark.parametrize("nu", [(2, 2), (2, 3), (1, 1), (3, 1)])
def test_fused_coarse_sweeps_match_half_sweeps(shape, nu):
    """The fused symmetric sweep of the coarse levels (k_sym_face, chosen
    on every eligible level in "fused" mode) computes what two half-sweep
    kernels compute: V-cycles and full multigrid cycles (odd sweep counts take
    the out-of-place prolongation) with fused sweeps equal those with
    half-sweeps to rounding (the compiler contracts the kernels' products
    into fused multiply-adds differently), in both precisions, and match the
    oracle."""
    print(f"fused coarse sweeps {shape} nu={nu}", flush=True)
    a, f, h = _rand_problem(shape, 31)
    hier64 = build_hierarchy(a, h, nu_pre=nu[0], nu_post=nu[1])
    for precision in ("fp64", "mixed"):
        out = {}
        for sweep in ("half", "fused"):
            s = gm.GMGPoisson(T(a), h=h, precision=precision, fine_sweep=sweep, nu_pre=nu[0], nu_post=nu[1])
            s.profile(True)
            out[sweep] = (s.vcycle(T(f)), s.fmg(T(f)))
            names = set(s.profile_read())
            s.profile(False)
            fused_l1 = shape[0] // 4 <= (256 if precision == "mixed" else 128)  # pairs per level-1 row
            assert ("sym_L1_" + ("f32" if precision == "mixed" else "f64") in names) == (sweep == "fused" and fused_l1)
            assert any(n.startswith("gs_L2") for n in names) == (sweep == "half")
        tol = 1e-5 if precision == "mixed" else 1e-13
        for i in range(2):
            d = ((out["fused"][i] - out["half"][i]).norm() / out["half"][i].norm()).item()
            assert d < tol, (precision, i, d)
        if precision == "fp64":
            assert rel(npy(out["fused"][0]), vcycle(hier64, f)) < 1e-12
            assert rel(npy(out["fused"][1]), fmg(hier64, f)) < 1e-12


# shapes (nx, ny, nz): the bottom kernel's full multigrid (64^3: levels 16^3
# down to 2^3 in one workgroup), per-level kernels down to a direct coarsest
# solve (48 x 40 x 36: coarsest 12 x 10 x 9), two levels, one level, ragged
# x tail, several block tiles
FMG_SHAPES = [(64, 64, 64), (48, 40, 36), (6, 4, 10), (3, 5, 7), (130, 8, 4), (200, 40, 48)]


@pytest.mark.parametrize("shape", FMG_SHAPES)
def test_fmg_matches_oracle(shape):
    """Full multigrid cycle (gmg_fmg) against the oracle's, float64 and the
    float32 cycle of mixed precision with either finest-level sweep."""
    print(f"fmg {shape}", flush=True)
    a, f, h = _rand_problem(shape, 23)
    s64 = gm.GMGPoisson(T(a), h=h, precision="fp64")
    assert rel(npy(s64.fmg(T(f))), fmg(build_hierarchy(a, h), f)) < 1e-12
    ref32 = fmg(build_hierarchy(a, h, dtype=np.float32), f.astype(np.float32)).astype(np.float64)
    for sweep in ("half", "fused"):
        s32 = gm.GMGPoisson(T(a), h=h, precision="mixed", fine_sweep=sweep)
        assert rel(npy(s32.fmg(T(f))), ref32) < 2e-5, sweep


@pytest.mark.parametrize("nu", [(0, 1), (1, 0), (1, 1), (3, 2)])
def test_fmg_sweep_counts(nu):
    a, f, h = _rand_problem((16, 16, 16), 24)
    s = gm.GMGPoisson(T(a), h=h, precision="fp64", nu_pre=nu[0], nu_post=nu[1])
    hier = build_hierarchy(a, h, nu_pre=nu[0], nu_post=nu[1])
    assert rel(npy(s.fmg(T(f))), fmg(hier, f)) < 1e-12


@pytest.mark.parametrize("nu", [(0, 1), (1, 0), (1, 1), (3, 2)])
def test_vcycle_sweep_counts(nu):
    a, f, h = _rand_problem((16, 16, 16), 5)
    s = gm.GMGPoisson(T(a), h=h, precision="fp64", nu_pre=nu[0], nu_post=nu[1])
    hier = build_hierarchy(a, h, nu_pre=nu[0], nu_post=nu[1])
    assert rel(npy(s.vcycle(T(f))), vcycle(hier, f)) < 1e-12


CASES = [  # (workload, n, k steps, restart)
    (1, 32, 5, 10),
    (2, 32, 8, 5),   # crosses two restarts
    (3, 64, 10, 10),
    (5, 32, 6, 10),
]


@pytest.mark.parametrize("cold", ["vcycle", "fmg"])
@pytest.mark.parametrize("case", CASES)
def test_fgmres_fp64_fixed_steps_matches_oracle(case, cold):
    """Cold-started solves at a fixed step count, preconditioned by V-cycles
    or by full multigrid cycles."""
    cfg, n, k, m = case
    print(f"fgmres fp64 workload {cfg} n={n} k={k} {cold}", flush=True)
    p = make_config(cfg, n=n)
    s = gm.GMGPoisson(T(p.a), precision="fp64", restart=m, max_iter=k, cold_cycle=cold)
    res = s.solve(T(p.f), p.phi_bot, p.phi_top, tol=0.0)
    ref = solve_poisson(p.a, p.f, p.h, p.phi_bot, p.phi_top, tol=0.0, max_iter=k, restart=m, cold=cold)
    assert res.status == gm.solver.NOT_CONVERGED and res.iterations == k == ref.iterations
    assert rel(npy(res.phi), ref.x) < 1e-10
    gh, oh = np.array(res.res_hist), np.array(ref.res_hist)
    assert len(gh) == len(oh) == k + 1
    # estimates near 1e-14 carry absolute rounding errors of ~1e-16 (Givens
    # rotations here, a library least-squares solve in the oracle)
    np.testing.assert_allclose(gh, oh, rtol=1e-6, atol=1e-15)


def test_restart_after_a_converged_estimate():
    """Below the attainable accuracy (float64, tol 1e-14 at 16^3) a cycle's
    estimate drops under tol while the true residual stays near 2e-14: the
    residual pass that follows each cycle, run without its store because the
    solve looked finished, runs again with the store and the solve restarts
    from it.  Restart after restart, the solve ends where the oracle's does
    (max_iter reached, or converged if its rounding lands below tol), and it
    reports the true residual."""
    p = make_config(2, n=16)
    s = gm.GMGPoisson(T(p.a), precision="fp64", restart=4, max_iter=30)
    res = s.solve(T(p.f), p.phi_bot, p.phi_top, tol=1e-14)
    ref = solve_poisson(p.a, p.f, p.h, p.phi_bot, p.phi_top, tol=1e-14, max_iter=30, restart=4)
    print(f"  GPU {res.iterations} steps, true relres {res.final_relres:.2e}; oracle {ref.iterations}, "
          f"{ref.true_relres:.2e}", flush=True)
    b = rhs(p.f, p.a, p.h, p.phi_bot, p.phi_top)
    true = np.linalg.norm(b - apply_operator(npy(res.phi), p.a, p.h)) / np.linalg.norm(b)
    if res.status == 0:
        assert res.final_relres < 1e-14 and res.iterations <= 30
    else:
        assert res.status == gm.solver.NOT_CONVERGED and res.iterations == ref.iterations == 30
    assert res.final_relres < 1e-13 and true < 1e-13
    assert rel(npy(res.phi), ref.x) < 1e-10


def _converged_pair(p, precision, tol=1e-8, **kw):
    s = gm.GMGPoisson(T(p.a), precision=precision, **kw)
    return s, s.solve(T(p.f), p.phi_bot, p.phi_top, tol=tol)


def test_config1_fp64_converged_matches_oracle():
    p = make_config(1)  # 64^3, a = 1
    s, res = _converged_pair(p, "fp64")
    ref = solve_poisson(p.a, p.f, p.h, p.phi_bot, p.phi_top, tol=1e-8)
    print(f"config1 fp64: gpu {res.iterations} steps, oracle {ref.iterations}", flush=True)
    assert res.converged and ref.converged
    assert abs(res.iterations - ref.iterations) <= 1
    if res.iterations != ref.iterations:
        ref = solve_poisson(p.a, p.f, p.h, p.phi_bot, p.phi_top, tol=0.0, max_iter=res.iterations)
        res = gm.GMGPoisson(T(p.a), precision="fp64", max_iter=res.iterations).solve(
            T(p.f), p.phi_bot, p.phi_top, tol=0.0)
    assert rel(npy(res.phi), ref.x) < 1e-10


def test_config1_mixed_within_residual_bound():
    p = make_config(1)
    s, res = _converged_pair(p, "mixed")
    ref = solve_poisson(p.a, p.f, p.h, p.phi_bot, p.phi_top, tol=1e-8)
    assert res.converged and res.final_relres < 1e-8
    b = rhs(p.f, p.a, p.h, p.phi_bot, p.phi_top)
    phi = npy(res.phi)
    r_gpu = np.linalg.norm(b - apply_operator(phi, p.a, p.h)) / np.linalg.norm(b)
    assert r_gpu < 1e-8
    lam_min = spectral_eigenvalues(p.a.shape, p.h).min()
    bound = (r_gpu + ref.true_relres) * np.linalg.norm(b) / lam_min
    err = np.linalg.norm(phi - ref.x)
    print(f"config1 mixed: {res.iterations} steps (fp64 oracle {ref.iterations}), "
          f"|phi - phi_fp64| / |phi_fp64| = {err / np.linalg.norm(ref.x):.2e}", flush=True)
    assert err <= bound
    assert res.iterations <= ref.iterations + 1


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_filament_full_size_residual(precision):
    """256^3, max(a) = 1e3: converged phi checked by the oracle's operator."""
    p = make_config(2)
    s, res = _converged_pair(p, precision)
    b = rhs(p.f, p.a, p.h, p.phi_bot, p.phi_top)
    r = np.linalg.norm(b - apply_operator(npy(res.phi), p.a, p.h)) / np.linalg.norm(b)
    print(f"filament 256^3 {precision}: {res.iterations} steps, true relres {r:.2e} "
          f"(reported {res.final_relres:.2e})", flush=True)
    assert res.converged and r < 1e-8
    assert abs(r - res.final_relres) <= 1e-3 * r + 1e-15


def test_operator_full_size_sampled():
    """512^3 (the headline grid): A x at 2000 sampled cells, stencil written
    out per cell from e18."""
    n = 512
    p = make_config(3, n=n)
    rng = np.random.default_rng(7)
    x = rng.standard_normal(p.a.shape)
    s = gm.GMGPoisson(T(p.a), precision="mixed")
    y = npy(s.apply(T(x), p.phi_bot, p.phi_top))
    h2 = (1.0 / n) ** 2
    a = p.a
    for _ in range(2000):
        k, j, i = (int(v) for v in rng.integers(0, n, 3))
        acc = 0.0
        for dk, dj, di in ((0, 0, 1), (0, 0, -1), (0, 1, 0), (0, -1, 0), (1, 0, 0), (-1, 0, 0)):
            kk, jj, ii = k + dk, j + dj, i + di
            if not (0 <= jj < n and 0 <= ii < n):
                continue
            if kk < 0 or kk >= n:
                pb = p.phi_bot if kk < 0 else p.phi_top
                acc += a[k, j, i] * (x[k, j, i] - (2 * pb - x[k, j, i])) / h2
            else:
                acc += 0.5 * (a[k, j, i] + a[kk, jj, ii]) * (x[k, j, i] - x[kk, jj, ii]) / h2
        assert abs(y[k, j, i] - acc) <= 1e-12 * (abs(acc) + a[k, j, i] / h2)


@pytest.mark.parametrize("warm", ["vcycle", "fmg"])
def test_warm_start_time_loop_matches_oracle(warm):
    """Per-step coefficient renewal and warm start (Sec. 2.1; Sec. 3.2): the
    two-filament workload advected one cell per step, 64^3, FP64; the
    warm-started solves preconditioned by V-cycles (the paper's choice) or by
    full multigrid cycles (option warm_cycle)."""
    n = 64
    prev_g = prev_o = None
    s = None
    for step in range(3):
        p = make_config(5, n=n, step=step)
        a = T(p.a)
        if s is None:
            s = gm.GMGPoisson(a, precision="fp64", warm_cycle=warm)
        else:
            s.update_coefficient(a)
        res = s.solve(T(p.f), p.phi_bot, p.phi_top, tol=1e-8, x0=prev_g)
        ref = solve_poisson(p.a, p.f, p.h, p.phi_bot, p.phi_top, tol=1e-8, x0=prev_o, warm=warm)
        print(f"time step {step} ({warm}): gpu {res.iterations}, oracle {ref.iterations}", flush=True)
        assert res.converged and res.iterations == ref.iterations
        assert rel(npy(res.phi), ref.x) < 1e-10
        prev_g, prev_o = res.phi.clone(), ref.x


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_warm_started_steps_take_two_to_four_iterations(precision):
    """The paper's iteration claim (Sec. 5.3, Fig. fstep): after the first
    time step, warm-started solves with V-cycles need 2 to 4 FGMRES
    iterations to 1e-8 at its mild coefficient contrast.  Two-filament
    workload advected one cell per step at 64^3 with max(a) = 2, one cold
    and four warm-started solves, each taking as many iterations as the
    float64 oracle's."""
    from workloads import config_two_filaments
    prev_g = prev_o = None
    s = None
    its = []
    for step in range(5):
        p = config_two_filaments(64, a_max=2.0, step=step)
        a = T(p.a)
        if s is None:
            s = gm.GMGPoisson(a, precision=precision)
        else:
            s.update_coefficient(a)
        res = s.solve(T(p.f), p.phi_bot, p.phi_top, tol=1e-8, x0=prev_g)
        ref = solve_poisson(p.a, p.f, p.h, p.phi_bot, p.phi_top, tol=1e-8, x0=prev_o)
        print(f"max(a) = 2, step {step} ({precision}): gpu {res.iterations}, oracle {ref.iterations}", flush=True)
        assert res.converged and res.iterations == ref.iterations
        its.append(res.iterations)
        prev_g, prev_o = res.phi.clone(), ref.x
    assert all(2 <= k <= 4 for k in its[1:]), its


@pytest.mark.parametrize("warm", ["vcycle", "fmg"])
def test_mixed_time_loop_two_filaments_within_residual_bound(warm):
    """The two-filament time loop in mixed precision on a 96^3 copy (the
    768^3 hierarchy's shape: 96 -> 3, coarsest 27 cells): every warm-started
    step converges, and its phi differs from the float64 oracle's by no more
    than the residual bound ||r_gpu + r_oracle|| / lambda_min (lambda_min of
    the a = 1 operator bounds that of a >= 1 from below)."""
    n = 96
    lam_min = spectral_eigenvalues((n, n, n), (1 / n,) * 3).min()
    s = None
    prev_g = prev_o = None
    for step in range(3):
        p = make_config(5, n=n, step=step)
        a = T(p.a)
        if s is None:
            s = gm.GMGPoisson(a, precision="mixed", warm_cycle=warm)
        else:
            s.update_coefficient(a)
        res = s.solve(T(p.f), p.phi_bot, p.phi_top, tol=1e-8, x0=prev_g)
        ref = solve_poisson(p.a, p.f, p.h, p.phi_bot, p.phi_top, tol=1e-8, x0=prev_o, warm=warm)
        b = rhs(p.f, p.a, p.h, p.phi_bot, p.phi_top)
        phi = npy(res.phi)
        r_gpu = np.linalg.norm(b - apply_operator(phi, p.a, p.h))
        r_ref = np.linalg.norm(b - apply_operator(ref.x, p.a, p.h))
        err = np.linalg.norm(phi - ref.x)
        print(f"mixed time step {step} ({warm}): gpu {res.iterations} steps, oracle {ref.iterations}, "
              f"|dphi|/|phi| = {err / np.linalg.norm(ref.x):.2e}", flush=True)
        assert res.converged and r_gpu < 1e-8 * np.linalg.norm(b)
        assert err <= (r_gpu + r_ref) / lam_min
        prev_g, prev_o = res.phi.clone(), ref.x


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_solve_from_zero_ignores_the_output_buffer(precision):
    """A solve without an initial guess never reads phi before its first
    update (which writes phi = Z y): the result does not depend on what the
    output buffer held, NaN included, is the same to the bit as into a
    zeroed buffer, and phi is exactly zero when the solve stops before any
    step (tolerance above 1: the zero guess already passes, Algorithm 1's
    test on the initial residual), or on max_iter = 0.  The same for GMRES
    and for a V-cycle's output."""
    p = make_config(2, n=32)
    f = T(p.f)
    for restart, max_iter in ((10, 200), (2, 200)):  # one cycle; restarts after two steps
        s = gm.GMGPoisson(T(p.a), precision=precision, restart=restart, max_iter=max_iter)
        zero = torch.zeros_like(f)
        nan = torch.full_like(f, float("nan"))
        r0 = s.solve(f, p.phi_bot, p.phi_top, out=zero)
        r1 = s.solve(f, p.phi_bot, p.phi_top, out=nan)
        assert r0.converged and r1.converged and r0.iterations == r1.iterations
        assert torch.equal(r0.phi, r1.phi) and torch.isfinite(r1.phi).all()
        assert r0.final_relres == r1.final_relres
        for method in ("fgmres", "gmres"):
            g0, _ = s.krylov_solve(f, p.phi_bot, p.phi_top, method=method, out=torch.zeros_like(f))
            g1, _ = s.krylov_solve(f, p.phi_bot, p.phi_top, method=method, out=torch.full_like(f, float("nan")))
            assert torch.equal(g0.phi, g1.phi) and torch.isfinite(g1.phi).all()
    early = s.solve(f, p.phi_bot, p.phi_top, tol=2.0, out=torch.full_like(f, float("nan")))
    assert early.converged and early.iterations == 0 and not early.phi.abs().max().item()
    s0 = gm.GMGPoisson(T(p.a), precision=precision, max_iter=0)
    none = s0.solve(f, p.phi_bot, p.phi_top, out=torch.full_like(f, float("nan")), raise_on_error=False)
    assert none.iterations == 0 and not none.phi.abs().max().item()
    z0 = npy(s.vcycle(f))
    assert np.isfinite(z0).all() and np.array_equal(z0, npy(s.vcycle(f)))


def test_determinism():
    p = make_config(2, n=32)
    s = gm.GMGPoisson(T(p.a), precision="mixed")
    r1 = npy(s.solve(T(p.f), p.phi_bot, p.phi_top).phi)
    r2 = npy(s.solve(T(p.f), p.phi_bot, p.phi_top).phi)
    assert np.array_equal(r1, r2)


# ---------------------------------------------------------------- edge cases
def test_zero_right_side_gives_zero():
    p = make_config(1, n=16)
    s = gm.GMGPoisson(T(p.a), precision="fp64")
    x0 = torch.ones(p.a.shape, dtype=torch.float64, device=DEV)
    res = s.solve(torch.zeros_like(x0), 0.0, 0.0, x0=x0)
    assert res.status == 0 and res.iterations == 0 and not res.phi.abs().max().item()


@pytest.mark.parametrize("method", ["fgmres", "gmres", "cg", "fcg", "cgs", "bicgstab"])
def test_zero_right_side_gives_zero_every_krylov_method(method):
    """b = 0 with a nonzero initial guess: every method of the comparison
    returns phi = 0 and relative residual 0, as fgmres_solve does."""
    p = make_config(1, n=16)
    s = gm.GMGPoisson(T(p.a), precision="fp64")
    x0 = torch.ones(p.a.shape, dtype=torch.float64, device=DEV)
    res, napp = s.krylov_solve(torch.zeros_like(x0), 0.0, 0.0, method=method, x0=x0)
    assert res.status == 0 and res.iterations == 0 and napp == 0
    assert res.final_relres == 0.0 and not res.phi.abs().max().item()


def test_max_iter_exhausted():
    p = make_config(3, n=16)
    s = gm.GMGPoisson(T(p.a), precision="fp64", max_iter=2)
    res = s.solve(T(p.f), p.phi_bot, p.phi_top, tol=1e-14)
    assert res.status == gm.solver.NOT_CONVERGED and res.iterations == 2 and len(res.res_hist) == 3


def test_exact_initial_guess_takes_no_steps():
    p = make_config(1, n=16)
    s = gm.GMGPoisson(T(p.a), precision="fp64")
    phi = s.solve(T(p.f), p.phi_bot, p.phi_top, tol=1e-12).phi
    res = s.solve(T(p.f), p.phi_bot, p.phi_top, tol=1e-8, x0=phi.clone())
    assert res.status == 0 and res.iterations == 0


def test_single_level_grid_breaks_down_happily():
    """No coarsening (odd sizes): the V-cycle is the exact inverse, so A z_1 =
    v_1 and the first step ends the solve exactly."""
    a, f, h = _rand_problem((3, 5, 7), 8)
    s = gm.GMGPoisson(T(a), h=h, precision="fp64")
    res = s.solve(T(f), 0.2, 0.7, tol=1e-12)
    assert res.status == 0 and res.iterations == 1
    b = rhs(f, a, h, 0.2, 0.7)
    assert np.linalg.norm(b - apply_operator(npy(res.phi), a, h)) <= 1e-12 * np.linalg.norm(b)


@pytest.mark.parametrize("shape", [(15, 16, 17), (30, 32, 34)])
def test_large_coarsest_level_inverted_on_gpu(shape):
    """Coarsest levels of more than 1024 cells are inverted on the GPU
    (Gauss-Jordan): a single-level grid of 4080 cells is solved in one
    FGMRES step to 1e-12 (checked with the oracle's operator), a two-level
    grid over that coarsest level gives the oracle's V-cycle (whose coarse
    solve is a Cholesky solve), and the mixed solve converges."""
    import time
    print(f"large coarsest level {shape}", flush=True)
    a, f, h = _rand_problem(shape, 41)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s = gm.GMGPoisson(T(a), h=h, precision="fp64")
    torch.cuda.synchronize()
    nx, ny, nz = s.levels[-1]
    print(f"  set-up {time.perf_counter() - t0:.2f} s, coarsest {nx} x {ny} x {nz}", flush=True)
    assert nx * ny * nz == 4080
    b = rhs(f, a, h, 0.2, 0.7)
    if len(s.levels) == 1:
        res = s.solve(T(f), 0.2, 0.7, tol=1e-12)
        assert res.status == 0 and res.iterations == 1
        assert np.linalg.norm(b - apply_operator(npy(res.phi), a, h)) <= 1e-12 * np.linalg.norm(b)
    else:
        hier = build_hierarchy(a, h)
        assert rel(npy(s.vcycle(T(f))), vcycle(hier, f)) < 1e-10
    sm = gm.GMGPoisson(T(a), h=h, precision="mixed")
    res = sm.solve(T(f), 0.2, 0.7, tol=1e-10)
    assert res.status == 0
    assert np.linalg.norm(b - apply_operator(npy(res.phi), a, h)) <= 1e-10 * np.linalg.norm(b)


def _offset(t):
    """A contiguous copy of t whose storage starts 8 bytes past a 16-byte
    boundary (the pair-lane kernels load 16-byte vectors; such buffers take
    the one-cell kernels)."""
    buf = torch.empty(t.numel() + 1, dtype=t.dtype, device=t.device)
    v = buf[1:].view(t.shape)
    v.copy_(t)
    assert v.data_ptr() % 16 == 8
    return v


def test_unaligned_buffers_take_the_one_cell_kernels():
    """Caller buffers that are not 16-byte aligned (8 bytes past a
    boundary): the solve (initial and true residuals), dL/da, the assembly of
    a time step and E give what aligned buffers give, to rounding (the one-
    cell kernels may contract products into FMAs differently, and the sums of
    the residual norms run in another order)."""

    def close(x, y):
        assert x.data_ptr() != y.data_ptr()
        assert (x - y).abs().max().item() <= 1e-14 * y.abs().max().item()

    p = make_config(2, n=32)
    a, f = T(p.a), T(p.f)
    s = gm.GMGPoisson(a, precision="fp64")
    r0 = s.solve(f, p.phi_bot, p.phi_top, tol=1e-10)
    out = _offset(torch.zeros_like(f))
    r1 = s.solve(_offset(f), p.phi_bot, p.phi_top, tol=1e-10, out=out)
    assert r1.iterations == r0.iterations
    assert rel(npy(r1.phi), npy(r0.phi)) < 1e-13
    lam = s.solve(f * 0.5 + 1.0, 0.0, 0.0, tol=1e-10).phi
    g0 = s.face_flux_grad(r0.phi, lam, p.phi_bot, p.phi_top)
    g1 = s.face_flux_grad_into(_offset(r0.phi), _offset(lam), p.phi_bot, p.phi_top, _offset(torch.zeros_like(f)))
    close(g1, g0)
    ne, np_ = T(p.a) * 0.1, T(p.a) * 0.2
    a0, f0 = s.assemble_elliptic(ne, np_, 1.0, 1e-3, 2.0, 0.5, De=(0.1, 0.2, 0.3))
    a1, f1 = s.assemble_elliptic(_offset(ne), _offset(np_), 1.0, 1e-3, 2.0, 0.5, De=(0.1, 0.2, 0.3),
                                 out=(_offset(a0), _offset(f0)))
    close(a1, a0)
    close(f1, f0)
    e0 = s.electric_field(r0.phi, p.phi_bot, p.phi_top)
    e1 = s.electric_field(_offset(r0.phi), p.phi_bot, p.phi_top, out=tuple(_offset(x) for x in e0))
    for x, y in zip(e1, e0):
        close(x, y)


def test_error_statuses():
    p = make_config(1, n=16)
    a = T(p.a)
    f = T(p.f)
    s = gm.GMGPoisson(a, precision="mixed")
    bad = f.clone()
    bad[3, 4, 5] = float("nan")
    assert s.solve(bad, 0.0, 1.0, raise_on_error=False).status == -3
    with pytest.raises(gm.GMGError) as e:
        gm.GMGPoisson(-a)
    assert e.value.status == -1
    an = a.clone()
    an[0, 0, 0] = float("inf")
    with pytest.raises(gm.GMGError) as e:
        gm.GMGPoisson(an)
    assert e.value.status == -3
    with pytest.raises(gm.GMGError) as e:
        gm.GMGPoisson(torch.ones((50, 50, 50), dtype=torch.float64, device=DEV))  # 25^3 coarsest
    assert e.value.status == -2
    assert s.solve(f, 0.0, 1.0, tol=-1.0, raise_on_error=False).status == -1


def test_workspace_too_small_rejected():
    import ctypes
    from paper_1812_08606_amd import _lib
    lib = _lib.load()
    opt = _lib.Options()
    lib.gmg_default_options(ctypes.byref(opt))
    a = torch.ones((16, 16, 16), dtype=torch.float64, device=DEV)
    need = lib.gmg_workspace_bytes(16, 16, 16, ctypes.byref(opt))
    ws = torch.empty(need, dtype=torch.uint8, device=DEV)
    ctx = ctypes.c_void_p()
    st = lib.gmg_setup(16, 16, 16, 1 / 16, 1 / 16, 1 / 16, ctypes.c_void_p(a.data_ptr()), ctypes.byref(opt),
                       ctypes.c_void_p(ws.data_ptr()), need - 256, None, ctypes.byref(ctx))
    assert st == -4 and not ctx.value


# ---------------------------------------------------------------- gradients
def test_face_flux_grad_matches_oracle():
    a, f, h = _rand_problem((70, 12, 8), 9)
    rng = np.random.default_rng(10)
    phi, lam = rng.standard_normal((2,) + a.shape)
    s = gm.GMGPoisson(T(a), h=h, precision="fp64")
    g = npy(s.face_flux_grad(T(phi), T(lam), 0.4, 1.5))
    ref = coefficient_gradient(phi, lam, h, 0.4, 1.5)
    np.testing.assert_allclose(g, ref, rtol=1e-12, atol=1e-13 * np.abs(ref).max())


def _probe_loss(phi, mask, h):
    idx = torch.nonzero(mask)
    k, j, i = idx[:, 0], idx[:, 1], idx[:, 2]
    gx = (phi[k, j, i + 1] - phi[k, j, i - 1]) / (2 * h)
    gy = (phi[k, j + 1, i] - phi[k, j - 1, i]) / (2 * h)
    gz = (phi[k + 1, j, i] - phi[k - 1, j, i]) / (2 * h)
    return ((gx ** 2 + gy ** 2 + gz ** 2) * h ** 3).sum()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_autograd_matches_oracle_adjoint(precision):
    """Backward of poisson_solve against the oracle's adjoint gradient
    (pinned itself by a dense autograd solve and by finite differences)."""
    from oracle.adjoint import solve_and_gradient
    p = make_config(4, n=16)
    n = 16
    from workloads import probe_box_mask
    mask = torch.tensor(probe_box_mask(n, box=((0.3, 0.7), (0.3, 0.7), (0.3, 0.7))), device=DEV)
    a = T(p.a).requires_grad_(True)
    f = T(p.f).requires_grad_(True)
    phi = gm.poisson_solve(f, a, p.phi_bot, p.phi_top, tol=1e-13, precision=precision)
    L = _probe_loss(phi, mask, 1.0 / n)
    L.backward()
    phi_leaf = phi.detach().clone().requires_grad_(True)
    _probe_loss(phi_leaf, mask, 1.0 / n).backward()
    gphi = npy(phi_leaf.grad)
    _, lam, dLda, fwd, adj = solve_and_gradient(p.a, p.f, p.h, p.phi_bot, p.phi_top, gphi, tol=1e-13)
    np.testing.assert_allclose(npy(f.grad), lam, rtol=0, atol=1e-8 * np.abs(lam).max())
    np.testing.assert_allclose(npy(a.grad), dLda, rtol=0, atol=1e-8 * np.abs(dLda).max())


def _grads(phi, mask, h):
    idx = torch.nonzero(mask)
    k, j, i = idx[:, 0], idx[:, 1], idx[:, 2]
    return ((phi[k, j, i + 1] - phi[k, j, i - 1]) / (2 * h),
            (phi[k, j + 1, i] - phi[k, j - 1, i]) / (2 * h),
            (phi[k + 1, j, i] - phi[k - 1, j, i]) / (2 * h))


def test_gradient_finite_differences_config4():
    """Config 4 (256^3, max(a) = 1e3): adjoint dL/da and dL/df against the
    central difference (L(a + d e_c) - L(a - d e_c)) / 2d with relative step
    d = 1e-6 on 20 seeded cells near the probe box.

    L changes by only ~1e-10 of itself at this step, below the noise of
    independent re-solves, so each perturbed solution is formed as
    phi_0 + e with A_+- e = b_+- - A_+- phi_0 solved in FP64 to 1e-12 of that
    residual, and L_+ - L_- is summed from the gradients of e_+ and e_-
    (2 grad phi_0 . (grad e_+ - grad e_-) + |grad e_+|^2 - |grad e_-|^2)."""
    p = make_config(4)
    n = p.shape[0]
    h = 1.0 / n
    from workloads import probe_box_mask
    mask = torch.tensor(probe_box_mask(n), device=DEV)
    a = T(p.a).requires_grad_(True)
    f = T(p.f).requires_grad_(True)
    phi = gm.poisson_solve(f, a, p.phi_bot, p.phi_top, tol=1e-8, precision="mixed")
    L = _probe_loss(phi, mask, h)
    L.backward()
    ga, gf = npy(a.grad), npy(f.grad)
    a0, f0 = T(p.a), T(p.f)
    solver = gm.GMGPoisson(a0, precision="fp64")
    phi0 = solver.solve(f0, p.phi_bot, p.phi_top, tol=1e-13).phi
    G0 = _grads(phi0, mask, h)

    def correction(a_t, f_t):
        solver.update_coefficient(a_t)
        r = f_t - solver.apply(phi0, p.phi_bot, p.phi_top)
        res = solver.solve(r, 0.0, 0.0, tol=1e-12)
        assert res.converged
        return _grads(res.phi, mask, h)

    def delta_L(ap, fp, am, fm):
        Ep, Em = correction(ap, fp), correction(am, fm)
        tot = 0.0
        for g0, ep, em in zip(G0, Ep, Em):
            tot += (2 * g0 * (ep - em) + ep * ep - em * em).sum().item()
        return tot * h ** 3

    rng = np.random.default_rng(40)
    lo, hi = int(0.35 * n), int(0.65 * n)
    cells = [tuple(int(v) for v in rng.integers(lo, hi, 3)) for _ in range(20)]
    gmax = np.abs(ga).max()
    print(f"L = {L.item():.6e}, max|dL/da| = {gmax:.3e}", flush=True)
    worst = 0.0
    for (k, j, i) in cells:
        d = 1e-6 * max(abs(p.a[k, j, i]), 1e-6 * np.abs(p.a).max())
        ap, am = a0.clone(), a0.clone()
        ap[k, j, i] += d
        am[k, j, i] -= d
        fd = delta_L(ap, f0, am, f0) / (2 * d)
        g = ga[k, j, i]
        print(f"  a-cell {(k, j, i)}: a={p.a[k, j, i]:.3e} adjoint {g:.6e} fd {fd:.6e}", flush=True)
        if abs(g) > 1e-3 * gmax:
            worst = max(worst, abs(fd - g) / abs(g))
            assert abs(fd - g) <= 1e-4 * abs(g), ((k, j, i), fd, g)
        else:
            assert abs(fd - g) <= 1e-7 * gmax, ((k, j, i), fd, g)
    fmax = np.abs(gf).max()
    for (k, j, i) in cells[:5]:
        d = 1e-6 * max(abs(p.f[k, j, i]), 1e-6 * np.abs(p.f).max())
        fp, fm = f0.clone(), f0.clone()
        fp[k, j, i] += d
        fm[k, j, i] -= d
        fd = delta_L(a0, fp, a0, fm) / (2 * d)
        g = gf[k, j, i]
        print(f"  f-cell {(k, j, i)}: adjoint {g:.6e} fd {fd:.6e}", flush=True)
        if abs(g) > 1e-3 * fmax:
            worst = max(worst, abs(fd - g) / abs(g))
        assert abs(fd - g) <= 1e-4 * abs(g) + 1e-7 * fmax, ((k, j, i), fd, g)
    print(f"worst relative FD mismatch {worst:.2e}", flush=True)


# ---------------------------------------------------------------- semi-implicit step
STEP_SHAPES = [(70, 12, 8), (5, 3, 2), (1, 1, 1), (33, 17, 7), (64, 64, 64)]
STEP_PRM = dict(eps0_over_e=0.02, tau_eff=0.35, mu_e=1.7, mu_p=0.017, De=(0.3, 0.5, 0.7))


def _densities(shape_xyz, seed):
    nx, ny, nz = shape_xyz
    rng = np.random.default_rng(seed)
    return rng.random((nz, ny, nx)), rng.random((nz, ny, nx))


@pytest.mark.parametrize("shape", STEP_SHAPES)
def test_assemble_elliptic_matches_oracle(shape):
    """Coefficient P and right side of e18 from the densities (Sec. 2.2)."""
    from oracle.semi_implicit import coefficient, right_side
    n_e, n_p = _densities(shape, 41)
    a0 = np.ones_like(n_e)
    h = (1.0 / shape[0], 1.3 / shape[1], 0.9 / shape[2])
    s = gm.GMGPoisson(T(a0), h=h, precision="fp64")
    a, f = s.assemble_elliptic(T(n_e), T(n_p), **STEP_PRM)
    p = STEP_PRM
    np.testing.assert_allclose(npy(a), coefficient(n_e, n_p, p["eps0_over_e"], p["tau_eff"], p["mu_e"], p["mu_p"]),
                               rtol=1e-15)
    ref = right_side(n_e, n_p, h, p["tau_eff"], p["De"])
    np.testing.assert_allclose(npy(f), ref, rtol=1e-13, atol=1e-13 * np.abs(ref).max())


@pytest.mark.parametrize("shape", STEP_SHAPES)
def test_electric_field_matches_oracle(shape):
    from oracle.semi_implicit import electric_field
    rng = np.random.default_rng(42)
    nx, ny, nz = shape
    phi = rng.standard_normal((nz, ny, nx))
    h = (1.0 / nx, 1.3 / ny, 0.9 / nz)
    s = gm.GMGPoisson(T(np.ones_like(phi)), h=h, precision="fp64")
    got = s.electric_field(T(phi), 0.4, -1.2)
    for g_, r_ in zip(got, electric_field(phi, h, 0.4, -1.2)):
        np.testing.assert_allclose(npy(g_), r_, rtol=1e-14, atol=1e-14 * np.abs(r_).max())


def test_semi_implicit_step_full_size():
    """512^3: the densities of the filament workload assembled into a and f,
    the solve, and E of the solution, each against the oracle's formula on
    the whole grid (the solve by its residual)."""
    from oracle.semi_implicit import coefficient, electric_field, right_side
    from workloads.streamer import config_filament
    p = config_filament(512, a_max=1e4, seed_number=3)
    kappa = p.meta["kappa"]
    n_e = (p.a - 1.0) / kappa
    n_p = p.f / 50.0 + n_e
    prm = dict(eps0_over_e=0.02, tau_eff=1.0, mu_e=kappa / 50.0, mu_p=kappa / 5000.0, De=(1e-6, 1e-6, 1e-6))
    print("semi-implicit step 512^3", flush=True)
    s = gm.GMGPoisson(T(np.ones_like(n_e)), precision="mixed")
    a, f = s.assemble_elliptic(T(n_e), T(n_p), **prm)
    h = (1 / 512,) * 3
    a_ref = coefficient(n_e, n_p, prm["eps0_over_e"], prm["tau_eff"], prm["mu_e"], prm["mu_p"])
    assert rel(npy(a), a_ref) < 1e-15
    f_ref = right_side(n_e, n_p, h, prm["tau_eff"], prm["De"])
    assert rel(npy(f), f_ref) < 1e-14
    s.update_coefficient(a)
    res = s.solve(f, 0.0, 1.0, tol=1e-8)
    assert res.converged
    E = s.electric_field(res.phi, 0.0, 1.0)
    E_ref = electric_field(npy(res.phi), h, 0.0, 1.0)
    for g_, r_ in zip(E, E_ref):
        assert rel(npy(g_), r_) < 1e-14


def _step_case(n):
    """Densities behind the two-filament workload (n_e = (a - 1) / kappa,
    n_p = f / 50 + n_e) and step parameters for which P = a / 50 plus an ion
    term at tau_eff = 1."""
    from oracle.semi_implicit import StepParams
    from workloads import config_two_filaments
    p = config_two_filaments(n, step=0)
    kappa = p.meta["kappa"]
    ne = (p.a - 1.0) / kappa
    npp = p.f / 50.0 + ne
    prm = StepParams(eps0_over_e=1.0 / 50.0, mu_e=kappa / 50.0, mu_p=kappa / 5000.0, De=(1e-4, 1e-4, 1e-4))
    return p, ne, npp, prm


def _ionisation_and_recombination(n_e, n_p, E):
    """The caller's transport of these tests: an ionisation source 0.1 |E|
    n_e and a recombination loss 0.01 n_e n_p for both species (cell-local;
    the same code runs on NumPy arrays and torch tensors)."""
    s = 0.1 * E[3] * n_e - 0.01 * n_e * n_p
    return s, s


@pytest.mark.parametrize("scheme", ["second", "first"])
def test_semi_implicit_time_steps_match_oracle(scheme):
    """Three time steps of the second-order scheme (eqs. e1, e2, semi2) or
    of the first-order one (eqs. semi-implicit, e15) on the two-filament
    densities at 64^3, float64: gmg_elliptic_step (assembly, renewal,
    warm-started solve, field) and gmg_density_update around the caller's
    transport give the oracle's phi, E and densities within 1e-10, with the
    same iteration counts."""
    from oracle.semi_implicit import time_step
    p, ne, npp, prm = _step_case(64)
    tau = 1.0
    st = gm.SemiImplicitStepper(T(ne), p.phi_bot, p.phi_top, prm.eps0_over_e, prm.mu_e, prm.mu_p, prm.De,
                                scheme=scheme, precision="fp64")
    ge, gp = T(ne), T(npp)
    oe, op, ophi = ne, npp, None
    for k in range(3):
        info = st.step(ge, gp, tau, _ionisation_and_recombination)
        r = time_step(oe, op, p.h, prm, tau, _ionisation_and_recombination, p.phi_bot, p.phi_top, phi_prev=ophi,
                      scheme=scheme)
        print(f"{scheme}-order step {k}: gpu {info.iterations} it, oracle {r.iterations} it, "
              f"|dn_e| {rel(npy(info.n_e), r.n_e):.1e}", flush=True)
        assert info.status == 0 and info.iterations == r.iterations
        assert rel(npy(info.phi), r.phi) < 1e-10
        for g_, r_ in zip(info.E, r.E):
            assert rel(npy(g_), r_) < 1e-10
        assert rel(npy(info.n_e), r.n_e) < 1e-10 and rel(npy(info.n_p), r.n_p) < 1e-10
        ge, gp = info.n_e, info.n_p
        oe, op, ophi = r.n_e, r.n_p, r.phi


def test_semi_implicit_time_steps_mixed_in_place():
    """Mixed precision, densities updated in place (out = the inputs), 128^3:
    every warm-started step converges, its phi checked with the oracle's
    operator on the coefficient and right side of eq. semi2, and the density
    update equals n + tau L recomputed from the returned field."""
    from oracle.semi_implicit import coefficient, right_side
    p, ne, npp, prm = _step_case(128)
    tau = 1.0
    st = gm.SemiImplicitStepper(T(ne), p.phi_bot, p.phi_top, prm.eps0_over_e, prm.mu_e, prm.mu_p, prm.De)
    ge, gp = T(ne), T(npp)
    for k in range(3):
        e0, p0 = npy(ge), npy(gp)
        info = st.step(ge, gp, tau, _ionisation_and_recombination, out=(ge, gp))
        a = coefficient(e0, p0, prm.eps0_over_e, tau / 2, prm.mu_e, prm.mu_p)
        b = rhs(right_side(e0, p0, p.h, tau / 2, prm.De), a, p.h, p.phi_bot, p.phi_top)
        r = np.linalg.norm(b - apply_operator(npy(info.phi), a, p.h)) / np.linalg.norm(b)
        print(f"mixed step {k}: {info.iterations} it, true relres {r:.2e}", flush=True)
        assert info.status == 0 and r < 1e-8
        E = tuple(npy(x) for x in info.E)
        le, lp = _ionisation_and_recombination(e0, p0, E)
        he, hp = e0 + tau / 2 * le, p0 + tau / 2 * lp
        le, lp = _ionisation_and_recombination(he, hp, E)
        np.testing.assert_allclose(npy(info.n_e), e0 + tau * le, rtol=1e-12, atol=1e-14)
        np.testing.assert_allclose(npy(info.n_p), p0 + tau * lp, rtol=1e-12, atol=1e-14)


def test_two_filament_time_loop_full_size():
    """The largest workload at its real shape (768^3, two filaments, max(a) =
    1e4, mixed): the cold solve of step 0 (full multigrid cycles) and the
    warm-started solve of step 1 after the coefficient renewal (V-cycles);
    each converges, and the oracle's operator on the whole grid gives a true
    relative residual below 1e-8 that matches the reported one within 0.1%."""
    s = prev = None
    for step in (0, 1):
        print(f"two filaments 768^3 step {step}", flush=True)
        p = make_config(5, step=step)
        a, f = T(p.a), T(p.f)
        if s is None:
            s = gm.GMGPoisson(a, precision="mixed")
        else:
            s.update_coefficient(a)
        res = s.solve(f, p.phi_bot, p.phi_top, tol=1e-8, x0=prev)
        b = rhs(p.f, p.a, p.h, p.phi_bot, p.phi_top)
        r = np.linalg.norm(b - apply_operator(npy(res.phi), p.a, p.h)) / np.linalg.norm(b)
        print(f"  {res.iterations} steps, true relres {r:.2e} (reported {res.final_relres:.2e})", flush=True)
        assert res.converged and r < 1e-8 and abs(r - res.final_relres) <= 1e-3 * r
        prev = res.phi.clone()
        del p, b, f


# ---------------------------------------------------------------- other Krylov methods
KRYLOV = ["gmres", "cg", "fcg", "cgs", "bicgstab"]


def _krylov_case(case):
    """("cfg", number, n) a numbered cubic workload; ("mesh", nx, ny, nz, const)
    the streamer channel on an anisotropic mesh of the unit cube (h_z < h_x)."""
    if case[0] == "cfg":
        return make_config(case[1], n=case[2])
    return config_streamer_mesh(case[1], case[2], case[3], constant_a=case[4])


@pytest.mark.parametrize("method", KRYLOV)
@pytest.mark.parametrize("case", [("cfg", 3, 32, 4), ("cfg", 5, 32, 3), ("mesh", 32, 32, 40, False, 4),
                                  ("mesh", 24, 16, 40, True, 3)])
def test_krylov_methods_fixed_steps_match_oracle(method, case):
    """Each method of the comparison (Sec. 5.3) after a fixed number of
    iterations, float64, against the oracle's implementation with the
    oracle's V-cycle: cubic workloads and the anisotropic meshes of the
    comparison (the 256 x 256 x 320 mesh's aspect, variable and constant a)."""
    from oracle.krylov import bicgstab, cg, cgs, gmres
    k = case[-1]
    print(f"krylov {method} case {case}", flush=True)
    p = _krylov_case(case[:-1])
    s = gm.GMGPoisson(T(p.a), precision="fp64", max_iter=k)
    res, napp = s.krylov_solve(T(p.f), p.phi_bot, p.phi_top, method=method, tol=0.0)
    hier = build_hierarchy(p.a, p.h)
    b = rhs(p.f, p.a, p.h, p.phi_bot, p.phi_top)

    def A(x):
        return apply_operator(x, p.a, p.h)

    def M(v):
        return vcycle(hier, v)
    fn = {"gmres": gmres, "cg": cg, "fcg": lambda *a, **kw: cg(*a, flexible=True, **kw), "cgs": cgs,
          "bicgstab": bicgstab}[method]
    ref = fn(A, b, M, tol=0.0, max_iter=k)
    assert res.status == gm.solver.NOT_CONVERGED and res.iterations == ref.iterations == k
    assert napp == ref.precond
    assert rel(npy(res.phi), ref.x) < 1e-9
    assert abs(res.final_relres - ref.true_relres) <= 1e-6 * ref.true_relres


@pytest.mark.parametrize("method", ["fgmres"] + KRYLOV)
def test_krylov_methods_converge_mixed(method):
    """Mixed precision, filament workload 64^3 (max(a) = 1e4): every method
    reaches the 1e-8 relative residual, checked with the oracle's operator."""
    p = make_config(3, n=64)
    s = gm.GMGPoisson(T(p.a), precision="mixed")
    res, napp = s.krylov_solve(T(p.f), p.phi_bot, p.phi_top, method=method, tol=1e-8)
    b = rhs(p.f, p.a, p.h, p.phi_bot, p.phi_top)
    r = np.linalg.norm(b - apply_operator(npy(res.phi), p.a, p.h)) / np.linalg.norm(b)
    print(f"krylov {method}: {res.iterations} iterations, {napp} preconditioner applications, "
          f"true relres {r:.2e}", flush=True)
    assert res.converged and r < 1e-8 and abs(r - res.final_relres) <= 1e-3 * r


def _table_mesh_solve(method):
    global _MESH_PROBLEM
    if _MESH_PROBLEM is None:
        _MESH_PROBLEM = config_streamer_mesh(256, 256, 320)
    p = _MESH_PROBLEM
    print(f"krylov {method} on {p.name}", flush=True)
    s = gm.GMGPoisson(T(p.a), precision="mixed")
    res, napp = s.krylov_solve(T(p.f), p.phi_bot, p.phi_top, method=method, tol=1e-8)
    b = rhs(p.f, p.a, p.h, p.phi_bot, p.phi_top)
    r = np.linalg.norm(b - apply_operator(npy(res.phi), p.a, p.h)) / np.linalg.norm(b)
    print(f"  {res.iterations} iterations, {napp} preconditioner applications, true relres {r:.2e}",
          flush=True)
    return res, r


@pytest.mark.parametrize("method", ["fgmres", "gmres", "fcg", "cgs", "bicgstab"])
def test_krylov_methods_converge_on_table_mesh(method):
    """Mixed precision on the full 256 x 256 x 320 mesh of the comparison
    (Sec. 5.3, Table t1; h_z = 1/320 < h_x = h_y = 1/256), max(a) = 1e4: the
    method reaches the 1e-8 relative residual, checked with the oracle's
    operator, and reports it within 0.1%."""
    res, r = _table_mesh_solve(method)
    assert res.converged and r < 1e-8 and abs(r - res.final_relres) <= 1e-3 * r


def test_cg_stagnates_on_table_mesh_and_says_so():
    """Plain preconditioned CG needs a symmetric preconditioner; the V-cycle
    here is not symmetric (mean-of-8 restriction against trilinear
    prolongation) and in mixed precision not even a fixed linear map.  On the
    256 x 256 x 320 mesh with max(a) = 1e4 CG stalls above the tolerance
    (flexible CG, which allows a varying preconditioner, converges): it must
    then stop at max_iter with status NOT_CONVERGED and report the true
    residual of the iterate it returns."""
    res, r = _table_mesh_solve("cg")
    assert res.status == gm.solver.NOT_CONVERGED and res.iterations == 200
    assert r > 1e-8 and abs(r - res.final_relres) <= 1e-3 * r


_MESH_PROBLEM = None


# ---------------------------------------------------------------- symmetric V-cycle
SYM_SHAPES = [(48, 40, 36), (70, 12, 8), (64, 64, 64), (6, 4, 10), (130, 8, 4), (64, 32, 48)]


@pytest.mark.parametrize("shape", SYM_SHAPES)
def test_transpose_restriction_vcycle_matches_oracle(shape):
    """The V-cycle with R = P^T / 8 (restriction "transpose": residual pass,
    full-weighting pass, every level through per-level kernels) against the
    oracle's, float64 and float32, with half-sweep and fused finest-level
    sweeps."""
    print(f"vcycle transpose restriction {shape}", flush=True)
    a, f, h = _rand_problem(shape, 41)
    hier = build_hierarchy(a, h, restriction="transpose")
    s64 = gm.GMGPoisson(T(a), h=h, precision="fp64", restriction="transpose")
    assert s64.levels == [tuple(l.shape) for l in hier.levels]
    z = npy(s64.vcycle(T(f)))
    ref = vcycle(hier, f)
    assert rel(z, ref) < 1e-12
    np.testing.assert_allclose(z, ref, rtol=1e-9, atol=1e-12 * np.abs(ref).max())
    ref32 = vcycle(build_hierarchy(a, h, dtype=np.float32, restriction="transpose"),
                   f.astype(np.float32)).astype(np.float64)
    for sweep in ("half", "fused"):
        s32 = gm.GMGPoisson(T(a), h=h, precision="mixed", restriction="transpose", fine_sweep=sweep)
        assert rel(npy(s32.vcycle(T(f))), ref32) < 2e-5


@pytest.mark.parametrize("n", [32, 128])
def test_transpose_restriction_vcycle_is_symmetric(n):
    """(u, M v) = (M u, v) for the float64 V-cycle with R = P^T / 8 and
    nu_pre = nu_post, on the filament workload (max(a) = 1e4); with the mean
    restriction the two differ."""
    p = make_config(3, n=n)
    rng = np.random.default_rng(42)
    u, v = T(rng.standard_normal(p.a.shape)), T(rng.standard_normal(p.a.shape))
    for restriction, symmetric in (("transpose", True), ("mean", False)):
        s = gm.GMGPoisson(T(p.a), precision="fp64", restriction=restriction, cold_cycle="vcycle")
        uMv = float((u * s.vcycle(v)).sum())
        Muv = float((s.vcycle(u) * v).sum())
        d = abs(uMv - Muv) / abs(uMv)
        print(f"{restriction} {n}^3: |(u,Mv) - (Mu,v)| / |(u,Mv)| = {d:.2e}", flush=True)
        assert (d < 1e-12) if symmetric else (d > 1e-6)


@pytest.mark.parametrize("method", ["cg", "fcg"])
@pytest.mark.parametrize("case", [("cfg", 3, 32, 6), ("mesh", 32, 32, 40, False, 6)])
def test_cg_with_symmetric_vcycle_fixed_steps_match_oracle(method, case):
    """CG and FCG preconditioned by the symmetric V-cycle, float64, after a
    fixed number of iterations, against the oracle."""
    from oracle.krylov import cg
    k = case[-1]
    p = _krylov_case(case[:-1])
    s = gm.GMGPoisson(T(p.a), precision="fp64", max_iter=k, restriction="transpose")
    res, napp = s.krylov_solve(T(p.f), p.phi_bot, p.phi_top, method=method, tol=0.0)
    hier = build_hierarchy(p.a, p.h, restriction="transpose")
    b = rhs(p.f, p.a, p.h, p.phi_bot, p.phi_top)
    ref = cg(lambda x: apply_operator(x, p.a, p.h), b, lambda v: vcycle(hier, v), tol=0.0, max_iter=k,
             flexible=method == "fcg")
    assert res.iterations == ref.iterations == k and napp == ref.precond
    assert rel(npy(res.phi), ref.x) < 1e-9


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_cg_converges_on_table_mesh_with_symmetric_vcycle(precision):
    """The 256 x 256 x 320 comparison mesh with max(a) = 1e4 (Sec. 5.3, Table
    t1): preconditioned by the symmetric V-cycle, CG reaches the 1e-8
    relative residual (checked with the oracle's operator), in at most 1.5
    times the iterations FGMRES takes with the same V-cycle."""
    global _MESH_PROBLEM
    if _MESH_PROBLEM is None:
        _MESH_PROBLEM = config_streamer_mesh(256, 256, 320)
    p = _MESH_PROBLEM
    s = gm.GMGPoisson(T(p.a), precision=precision, restriction="transpose")
    b = rhs(p.f, p.a, p.h, p.phi_bot, p.phi_top)
    its = {}
    for method in ("fgmres", "cg"):
        res, napp = s.krylov_solve(T(p.f), p.phi_bot, p.phi_top, method=method, tol=1e-8)
        r = np.linalg.norm(b - apply_operator(npy(res.phi), p.a, p.h)) / np.linalg.norm(b)
        print(f"symmetric V-cycle, {precision}, {method}: {res.iterations} iterations, true relres {r:.2e}",
              flush=True)
        assert res.converged and r < 1e-8 and abs(r - res.final_relres) <= 1e-3 * r
        its[method] = res.iterations
    assert its["cg"] <= 1.5 * its["fgmres"]


# ---------------------------------------------------------------- HIP graphs
@pytest.mark.parametrize("precision, warm", [("mixed", "vcycle"), ("fp64", "vcycle"), ("mixed", "fmg")])
def test_graph_replays_equal_eager_launches(precision, warm):
    """Preconditioner applications replayed from captured HIP graphs give
    bit-identical solves to eager launches, over repeated replays with the
    program's own eager work and synchronisations in between: cold solves
    (full multigrid), warm solves (V-cycles, or full multigrid cycles with
    the warm_cycle option), BiCGSTAB, and after a change of the coefficient
    buffer."""
    p = make_config(2, n=64)
    a = T(p.a)
    f = T(p.f)
    sg = gm.GMGPoisson(a, precision=precision, graphs=True, warm_cycle=warm)
    se = gm.GMGPoisson(a, precision=precision, graphs=False, warm_cycle=warm)
    for rep in range(3):
        rg = sg.solve(f, p.phi_bot, p.phi_top, tol=1e-8)
        re_ = se.solve(f, p.phi_bot, p.phi_top, tol=1e-8)
        assert rg.iterations == re_.iterations and torch.equal(rg.phi, re_.phi), rep
        torch.cuda.synchronize()
        x0 = 0.5 * re_.phi
        wg = sg.solve(f, p.phi_bot, p.phi_top, tol=1e-8, x0=x0.clone())
        we = se.solve(f, p.phi_bot, p.phi_top, tol=1e-8, x0=x0.clone())
        assert torch.equal(wg.phi, we.phi), rep
        kg, _ = sg.krylov_solve(f, p.phi_bot, p.phi_top, method="bicgstab")
        ke, _ = se.krylov_solve(f, p.phi_bot, p.phi_top, method="bicgstab")
        assert torch.equal(kg.phi, ke.phi), rep
    a2 = a * 1.5
    sg.update_coefficient(a2)
    se.update_coefficient(a2)
    rg = sg.solve(f, p.phi_bot, p.phi_top, tol=1e-8)
    re_ = se.solve(f, p.phi_bot, p.phi_top, tol=1e-8)
    assert torch.equal(rg.phi, re_.phi)


# ---------------------------------------------------------------- Chebyshev smoother
CHEB_SHAPES = [(48, 40, 36), (70, 12, 8), (64, 64, 64), (6, 4, 10), (130, 8, 4), (32, 32, 40)]


def _oracle_cheb(a, h):
    from oracle.chebyshev import lambda_max_estimate, start_vector
    hier = build_hierarchy(a, h)
    lams = []
    for li, lev in enumerate(hier.levels[:-1]):
        nx, ny, nz = lev.shape
        lams.append(lambda_max_estimate(lev, start_vector((nz, ny, nx), li)))
    return hier, lams


@pytest.mark.parametrize("shape", CHEB_SHAPES)
def test_chebyshev_estimates_and_vcycle_match_oracle(shape):
    """Chebyshev(2)+SSOR smoother (Sec. 3.2, eq. qntn), float64: the Arnoldi
    estimate of every smoothed level (SplitMix64 start vectors drawn on each
    side) and one V-cycle from zero against the oracle's."""
    from oracle.chebyshev import vcycle_chebyshev
    print(f"chebyshev fp64 {shape}", flush=True)
    a, f, h = _rand_problem(shape, 8)
    s = gm.GMGPoisson(T(a), h=h, precision="fp64", smoother="chebyshev")
    hier, lams = _oracle_cheb(a, h)
    assert [tuple(l.shape) for l in hier.levels] == s.levels
    got = s.chebyshev_estimates()
    assert len(got) == len(lams)
    np.testing.assert_allclose(got, lams, rtol=1e-11)
    bounds = [(0.1 * lam, 1.1 * lam) for lam in lams]
    z = npy(s.vcycle(T(f)))
    ref = vcycle_chebyshev(hier, bounds, f)
    assert rel(z, ref) < 1e-11
    np.testing.assert_allclose(z, ref, rtol=1e-8, atol=1e-11 * np.abs(ref).max())


@pytest.mark.parametrize("nu", [(2, 1), (1, 2), (0, 1)])
def test_chebyshev_vcycle_applications(nu):
    """nu_pre / nu_post applications of the smoother (0: none before the
    coarse correction) against the oracle's V-cycle with the same counts."""
    from oracle.chebyshev import chebyshev_smooth
    from oracle.multigrid import coarse_solve, prolong, restrict
    from oracle.operator import apply_faces
    a, f, h = _rand_problem((32, 24, 16), 9)
    s = gm.GMGPoisson(T(a), h=h, precision="fp64", smoother="chebyshev", nu_pre=nu[0], nu_post=nu[1])
    hier, lams = _oracle_cheb(a, h)

    def cyc(b, level):
        lev = hier.levels[level]
        if level == len(hier.levels) - 1:
            return coarse_solve(hier, b)
        lmax, lstar = 1.1 * lams[level], 0.1 * lams[level]
        x = np.zeros_like(b)
        for _ in range(nu[0]):
            x = chebyshev_smooth(x, b, lev, lmax, lstar)
        x = x + prolong(cyc(restrict(b - apply_faces(x, lev.faces, lev.h)), level + 1))
        for _ in range(nu[1]):
            x = chebyshev_smooth(x, b, lev, lmax, lstar)
        return x
    assert rel(npy(s.vcycle(T(f))), cyc(f, 0)) < 1e-11


@pytest.mark.parametrize("case", [(3, 32, 6, 10), (2, 32, 8, 5)])
def test_chebyshev_fgmres_fixed_steps_match_oracle(case):
    """FGMRES(m) with the Chebyshev V-cycle, fixed step count, float64."""
    from oracle.chebyshev import vcycle_chebyshev
    from oracle.fgmres import fgmres
    cfg, n, k, m = case
    print(f"chebyshev fgmres workload {cfg} n={n} k={k} m={m}", flush=True)
    p = make_config(cfg, n=n)
    s = gm.GMGPoisson(T(p.a), precision="fp64", smoother="chebyshev", restart=m, max_iter=k)
    res = s.solve(T(p.f), p.phi_bot, p.phi_top, tol=0.0)
    hier, lams = _oracle_cheb(p.a, p.h)
    bounds = [(0.1 * lam, 1.1 * lam) for lam in lams]
    b = rhs(p.f, p.a, p.h, p.phi_bot, p.phi_top)
    ref = fgmres(lambda x: apply_operator(x, p.a, p.h), b, lambda v: vcycle_chebyshev(hier, bounds, v),
                 tol=0.0, restart=m, max_iter=k)
    assert res.iterations == ref.iterations == k
    assert rel(npy(res.phi), ref.x) < 1e-10


def test_chebyshev_mixed_converges_and_renews_bounds():
    """Mixed precision (float32 smoother and estimate's SSOR), filament 64^3,
    max(a) = 1e4: the estimates agree with float64's to float32 rounding; the
    solve converges (checked with the oracle's operator) in at most one step
    more than the float64 oracle's Chebyshev solve; a new coefficient
    re-estimates the bounds exactly as a fresh context does; the full
    multigrid entry point is refused (V-cycles only)."""
    from oracle.chebyshev import vcycle_chebyshev
    from oracle.fgmres import fgmres
    p = make_config(3, n=64)
    s = gm.GMGPoisson(T(p.a), precision="mixed", smoother="chebyshev")
    s64 = gm.GMGPoisson(T(p.a), precision="fp64", smoother="chebyshev")
    np.testing.assert_allclose(s.chebyshev_estimates(), s64.chebyshev_estimates(), rtol=1e-4)
    res = s.solve(T(p.f), p.phi_bot, p.phi_top, tol=1e-8)
    b = rhs(p.f, p.a, p.h, p.phi_bot, p.phi_top)
    r = np.linalg.norm(b - apply_operator(npy(res.phi), p.a, p.h)) / np.linalg.norm(b)
    hier, lams = _oracle_cheb(p.a, p.h)
    bounds = [(0.1 * lam, 1.1 * lam) for lam in lams]
    ref = fgmres(lambda x: apply_operator(x, p.a, p.h), b, lambda v: vcycle_chebyshev(hier, bounds, v), tol=1e-8)
    print(f"chebyshev mixed 64^3: {res.iterations} steps (fp64 oracle {ref.iterations}), relres {r:.2e}",
          flush=True)
    assert res.converged and r < 1e-8 and res.iterations <= ref.iterations + 1
    a2 = T(p.a) * 1.5 + 0.25
    s.update_coefficient(a2)
    fresh = gm.GMGPoisson(a2, precision="mixed", smoother="chebyshev")
    assert s.chebyshev_estimates() == fresh.chebyshev_estimates()
    r2 = s.solve(T(p.f), p.phi_bot, p.phi_top, tol=1e-8)
    r3 = fresh.solve(T(p.f), p.phi_bot, p.phi_top, tol=1e-8)
    assert r2.converged and torch.equal(r2.phi, r3.phi)
    with pytest.raises(gm.solver.GMGError):
        s.fmg(T(p.f))


def test_chebyshev_graphs_and_krylov_methods():
    """The Chebyshev V-cycle replayed from captured HIP graphs equals its
    eager launches over repeated solves and after a renewal (the recurrence
    coefficients are launch arguments, so a renewal must drop the graphs);
    and it preconditions the other Krylov methods (BiCGSTAB, flexible CG) to
    convergence, checked with the oracle's operator."""
    p = make_config(2, n=64)
    a, f = T(p.a), T(p.f)
    sg = gm.GMGPoisson(a, precision="mixed", smoother="chebyshev", graphs=True)
    se = gm.GMGPoisson(a, precision="mixed", smoother="chebyshev", graphs=False)
    for rep in range(3):
        rg = sg.solve(f, p.phi_bot, p.phi_top, tol=1e-8)
        re_ = se.solve(f, p.phi_bot, p.phi_top, tol=1e-8)
        assert rg.converged and torch.equal(rg.phi, re_.phi), rep
        torch.cuda.synchronize()
    a2 = a * 3.0 + 1.0
    sg.update_coefficient(a2)
    se.update_coefficient(a2)
    assert sg.chebyshev_estimates() == se.chebyshev_estimates()
    rg = sg.solve(f, p.phi_bot, p.phi_top, tol=1e-8)
    re_ = se.solve(f, p.phi_bot, p.phi_top, tol=1e-8)
    assert torch.equal(rg.phi, re_.phi)
    b = rhs(p.f, npy(a2), p.h, p.phi_bot, p.phi_top)
    for method in ("bicgstab", "fcg"):
        res, napp = se.krylov_solve(f, p.phi_bot, p.phi_top, method=method, tol=1e-8)
        r = np.linalg.norm(b - apply_operator(npy(res.phi), npy(a2), p.h)) / np.linalg.norm(b)
        print(f"chebyshev-preconditioned {method}: {res.iterations} iterations, relres {r:.2e}", flush=True)
        assert res.converged and r < 1e-8
