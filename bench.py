#!/usr/bin/env python3
"""Benchmark of the GMG-preconditioned FGMRES solve on one MI355X.

Default workload (c3): the 512^3 single-filament problem (max(a) = 1e4,
f = 50 (n_p - n_e)), unit cube, phi = 0 / 1 on the plates, tolerance 1e-8,
FGMRES(10) with one multigrid cycle per step: full multigrid cycles in a
solve from no initial guess, V-cycles in a warm-started one (the library's
default), with 2 pre- and 3 post-smoothing sweeps (the library's default is
2 and 2; one more post-sweep saves a FGMRES step of the cold solves here).  One benchmark step is one pass of
the whole hot path: coefficient renewal (hierarchy rebuild), the forward
solve from a zero guess, the adjoint solve for a fixed dL/dphi and the dL/da
face-flux kernel.  Each step therefore holds two converged 1e-8 solves;
``value`` counts cells x solves per second over the timed steps (inputs
resident in HBM).

Workloads c1, c2, c4 (64^3 constant coefficient, 256^3 filament with
max(a) = 1e3, 256^3 gradient workload) run the same step on their fields.
Workload c5: the 768^3 two-filament time loop.  Step t advects both
filaments t cells in +z (the step-0 fields rolled along z on the device),
renews the coefficient and solves warm-started from the previous phi; one
solve per step, with the library's V(2,2) smoothing and full multigrid
cycles for the warm-started solves (option warm_cycle; the library default
is the paper's V-cycle, which takes 7 steps here against 4-5).

Besides the step, the other Krylov methods of Sec. 5.3 (Table t1) are timed
on the workload's forward problem, and again on the streamer channel meshed
256 x 256 x 320 and 512 x 512 x 640 on the unit cube (the comparison's
meshes, h_z < h_x = h_y), with its variable coefficient and with a = 1
(Table t2's constant-coefficient problem).  The red-black Gauss-Seidel
smoother is also compared with the paper's Chebyshev(2)+SSOR smoother on the
workload's forward problem (solve time, iterations, renewal time).

Prints one JSON line on stdout; progress goes to stderr.

  python bench.py [--steps K] [--warmup W] [--gpus 1] [--workload c1..c5] [--n N]
"""
import argparse
import hashlib
import json
import os
import re
import statistics
import sys
import time

os.environ.setdefault("OPENBLAS_NUM_THREADS", "1")  # the CPU oracle leg runs on one core

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "converged cells/s per 1e-8 Poisson solve + HBM GB/s, FP64 vs mixed, 512^3"
PEAK_HBM_GBS = 8000.0  # MI355X HBM3E
# what the counted kernels (the fused finest-level sweeps) are built from:
# their device code (the fused sweep's header and the shared helpers it
# includes) and the host functions that set their launch shapes
KERNEL_SOURCES = {
    "sym_fine_f32": ["gmg_common.hpp", "gmg_sym.hpp"],
    "sym_fine_f64": ["gmg_common.hpp", "gmg_sym.hpp"],
}
LAUNCH_SOURCES = {
    "sym_fine_f32": ("gmg.hip", r"Launch sym_launch\(.*?\n}\n"),
    "sym_fine_f64": ("gmg.hip", r"Launch sym_launch\(.*?\n}\n"),
}
TRAFFIC_FILES = {
    "sym_fine_f32": os.path.join(ROOT, "profiles", "traffic_sym_fine_f32_filament512.md"),
    "sym_fine_f64": os.path.join(ROOT, "profiles", "traffic_sym_fine_f64_filament512.md"),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed steps (c3: 3, c5: 19)")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=["c1", "c2", "c3", "c4", "c5"], default="c3")
    ap.add_argument("--n", type=int, default=None, help="grid edge (default: the workload's)")
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 side-by-side run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-n", type=int, default=160, help="edge of the CPU-oracle sample grid")
    ap.add_argument("--no-profile", action="store_true", help="skip the per-kernel event pass")
    ap.add_argument("--no-krylov", action="store_true",
                    help="skip the comparison runs (Krylov methods, meshes, smoothers)")
    ap.add_argument("--nu-pre", type=int, default=None,
                    help="pre-smoothing sweeps of the step (default 2)")
    ap.add_argument("--nu-post", type=int, default=None,
                    help="post-smoothing sweeps of the step (default 3 for c1-c4, 2 for c5)")
    ap.add_argument("--warm-cycle", choices=["vcycle", "fmg"], default="fmg",
                    help="cycle of the warm-started solves of c5 (default fmg: 4-5 instead of 7 steps)")
    ap.add_argument("--no-smoothers", action="store_true",
                    help="skip the comparison of the Gauss-Seidel and Chebyshev smoothers")
    ap.add_argument("--krylov-meshes", default="256x256x320,512x512x640",
                    help="comma-separated nx x ny x nz meshes of the unit cube for the Krylov comparison "
                         "('' skips it)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a 1 GiB device copy (scale of the hardware traffic counters)")
    args = ap.parse_args()
    if args.steps is None:
        args.steps = 19 if args.workload == "c5" else 3
    if args.n is None:
        args.n = {"c1": 64, "c2": 256, "c3": 512, "c4": 256, "c5": 768}[args.workload]
    # smoothing of the benchmark step: V(2,3) for the cold-start workloads
    # (fewest FGMRES steps per unit time with full multigrid cycles at 256^3
    # and 512^3), the library's V(2,2) for the warm-started time loop
    if args.nu_pre is None and args.nu_post is None:
        args.nu_pre, args.nu_post = (2, 2) if args.workload == "c5" else (2, 3)
    return args


# ---------------------------------------------------------------------------
# Algorithmic bytes per cell of the level a kernel runs on: every kernel reads
# each input once and writes each output once, at element granularity.
# s = bytes of the V-cycle precision.  On the finest level the iterate x and
# its right side B are stored by colour, so a half-sweep touches half of each.
# ---------------------------------------------------------------------------
def split_name(name):
    """'gs_fine_f32' -> ('gs', 0); 'gs_L2_f32' -> ('gs', 2); other -> (name, None)."""
    m = re.match(r"^(.*)_(fine|L(\d+)|coarsest)_(f32|f64)$", name)
    if not m:
        return name, None
    level = 0 if m.group(2) == "fine" else (int(m.group(3)) if m.group(3) else -1)
    return m.group(1), level


def bytes_per_cell(base, level, s, nu_post=2):
    if level == 0:
        if base == "sym":  # fused symmetric sweep: old X of the second colour, a, B read; X written
            return 0.5 * s + s + s + s
        if base == "sym_first":  # from x = 0: u (float64) and a read; B and X (both colours) written
            return 8 + s + s + s
        if base == "sym_resid":  # fused symmetric sweep and its residual restricted: + coarse right side (1/8)
            return 0.5 * s + s + s + s + s / 8
        if base == "gs":  # X of the other colour, a, B of the own colour read; X own colour written
            return 0.5 * s + s + 0.5 * s + 0.5 * s
        if base == "gs_first":  # u (float64) and a read; B (both colours) and X (own colour) written
            return 8 + s + s + 0.5 * s
        if base == "resid_restrict":  # X, B, a read; coarse right side (1/8) written
            return 3 * s + s / 8
        if base == "prolong_add":  # the red half of X read and written (both halves without post-sweeps)
            return (1 if nu_post > 0 else 2) * s + s / 8
        if base == "restrict_rhs":  # u (float64) read; B and the coarse right side (1/8) written
            return 8 + s + s / 8
        if base == "prolong_set":  # coarse x read, the black half of X written (the guess the red sweep reads)
            return 0.5 * s + s / 8
        return None
    if level is not None and level > 0:  # face coefficients wx, wy, wz (plates neglected)
        if base == "sym":  # fused symmetric sweep: old x of the second colour, faces, b read; x written
            return 0.5 * s + 3 * s + s + s
        if base == "sym_first":  # from x = 0: faces, b read; x written
            return 3 * s + s + s
        if base == "gs":  # x, faces read; b, x of the own colour read / written
            return s + 3 * s + 0.5 * s + 0.5 * s
        if base == "gs_first":  # faces, b of the own colour read; x written
            return 3 * s + 0.5 * s + s
        if base == "resid_restrict":  # x, b, faces read; coarse right side written
            return s + s + 3 * s + s / 8
        if base == "prolong_add":  # x read and written, coarse x read
            return 2 * s + s / 8
        if base == "restrict":  # b read, coarse right side written
            return s + s / 8
        if base == "prolong_set":  # coarse x read, x written
            return s + s / 8
    return None


def cheb_bytes_per_cell(base, level, s):
    """Kernels of a V-cycle with the Chebyshev(2)+SSOR smoother (the SSOR
    half-sweeps are the Gauss-Seidel kernels and keep their models)."""
    if base == "cheb_update":  # d, x written; e, d, x read, except d in the first step of an
        # application and x in the first from zero: mean of 3s, 5s, 4s, 5s over a V-cycle's 4 steps
        return 4.25 * s
    if level == 0:
        if base == "cheb_resid":  # X (both colours), u (float64), a read; r (float64, natural) written
            return 2 * s + 16
        if base == "restrict_rhs":  # r (float64) read; B scratch and the coarse right side written
            return 8 + s + s / 8
        if base == "prolong_add":  # both colours of X read and written, coarse x read
            return 2 * s + s / 8
    elif level is not None and level > 0:
        if base == "cheb_resid":  # x, b, faces read; r written
            return 6 * s
        if base == "ssor_first":
            return bytes_per_cell("gs_first", level, s)
        if base == "ssor":
            return bytes_per_cell("gs", level, s)
    return bytes_per_cell(base, level, s)


def outer_bytes(name, nv, s_z):
    if name.startswith("op_multidot"):  # z, a read, w written, nv vectors read
        return s_z + 8 + 8 + 8 * nv
    if name == "axpy_norm":  # w read+written, nv vectors read
        return 16 + 8 * nv
    if name == "init_residual":  # f, a, x read; r written
        return 32
    if name.startswith("update"):  # phi read+written, nv preconditioned vectors read
        return 16 + s_z * nv
    if name == "face_grad":  # phi, lam read; dL/da written
        return 24
    if name == "assemble_step":  # n_e, n_p read; a, f written
        return 32
    if name == "electric_field":  # phi read; E_x, E_y, E_z, |E| written
        return 40
    return None


def nv_sequence(iterations, restart):
    """Vectors per Arnoldi step j (j+1 within each restart cycle)."""
    return [it % restart + 1 for it in range(iterations)]


def kernel_source_hash(kernel="sym_fine_f32"):
    """Hash of the device sources and of the kernel's launch function."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1812_08606_amd", "csrc")
    for f in KERNEL_SOURCES[kernel]:
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    fname, pattern = LAUNCH_SOURCES[kernel]
    text = open(os.path.join(csrc, fname)).read()
    m = re.search(pattern, text, flags=re.S)
    h.update((m.group(0) if m else text).encode())
    return h.hexdigest()[:16]


def measured_traffic(kernel="sym_fine_f32"):
    """HBM bytes per launch of a finest-level sweep kernel at 512^3 from the
    committed counter summary, if it was taken on the current kernel sources."""
    path = TRAFFIC_FILES.get(kernel)
    if path is None or not os.path.exists(path):
        return None
    txt = open(path).read()
    m_b = re.search(r"traffic_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    m_h = re.search(r"kernel_source_sha256_16:\s*([0-9a-f]+)", txt)
    if not (m_b and m_h) or m_h.group(1) != kernel_source_hash(kernel):
        return None
    return float(m_b.group(1))


def kernel_table(prof, prof_steps, its_prof, s, N, restart=10):
    """Per-kernel rows (name, ms per step, launches per step, average ms per
    launch, algorithmic GB/s, algorithmic bytes per launch) from an event
    pass, sorted by time, and the algorithmic bytes of the whole pass.  s:
    bytes of the V-cycle precision (also of the stored z_j)."""
    nvs = [nv for its in its_prof for nv in nv_sequence(its, restart)]
    table = []
    total_bytes = 0.0
    for name, (tot_ms, cnt) in sorted(prof.items(), key=lambda kv: -kv[1][0]):
        base, level = split_name(name)
        tb = None
        bpl = None
        if level is not None and level >= 0:
            bpc = bytes_per_cell(base, level, s)
            if bpc is not None:
                bpl = bpc * N / 8 ** level
                tb = bpl * cnt
        elif name.startswith("op_multidot") or name == "axpy_norm":
            tb = sum(outer_bytes(name, nv, s) for nv in nvs) * N
        elif name.startswith("update"):
            b_upd = 0.0
            for its in its_prof:
                left = its
                while left > 0:
                    k = min(left, restart)
                    b_upd += outer_bytes(name, k, s)
                    left -= k
            tb = b_upd * N
        elif outer_bytes(name, 0, s) is not None:
            tb = outer_bytes(name, 0, s) * N * cnt
        gbs = tb / (tot_ms * 1e-3) / 1e9 if tb else None
        if tb:
            total_bytes += tb
        table.append((name, tot_ms / prof_steps, cnt / prof_steps, tot_ms / cnt, gbs, bpl))
    return table, total_bytes


def roofline_of(table, ms_per_step, traffic_ok):
    """Roofline entry of the dominant kernel with a per-launch byte model
    (the first such row of the time-sorted table): algorithmic bytes per
    launch over the event-timed average launch; measured traffic from the
    committed counter summary when traffic_ok and the sources match."""
    dom = next((t for t in table if t[5] is not None), None)
    if dom is None:
        return None
    name, ms_s, cnt, avg_ms, gbs, bpl = dom
    achieved = bpl / (avg_ms * 1e-3) / 1e9
    return {
        "bound": "hbm",
        "kernel": name,
        "achieved": round(achieved, 1),
        "peak": PEAK_HBM_GBS,
        "unit": "GB/s",
        "frac": round(achieved / PEAK_HBM_GBS, 4),
        "traffic": measured_traffic(name) if traffic_ok else None,
        "avg_launch_ms": round(avg_ms, 5),
        "bytes_per_launch": bpl,
        "share_of_step": round(ms_s / ms_per_step, 3),
    }


def kernel_rows(table, limit=12):
    """The table's first rows for the JSON line."""
    return [{"kernel": name, "ms_per_step": round(ms_s, 4), "launches_per_step": round(cnt, 2),
             "avg_ms": round(avg, 5), "GBps": round(gbs) if gbs else None}
            for name, ms_s, cnt, avg, gbs, _ in table[:limit]]


KRYLOV_METHODS = ("fgmres", "gmres", "cg", "fcg", "cgs", "bicgstab")


def time_krylov_methods(torch, make_solver, f, pb, pt, tol):
    """Each Krylov method of the comparison from no initial guess, one
    V-cycle per preconditioner application: one untimed solve, then the
    median of 3 event-timed solves; then FGMRES and CG preconditioned by the
    symmetric V-cycle (restriction R = P^T / 8; "_symmetric").
    make_solver(restriction) builds the solver (one at a time on the GPU)."""
    phi = torch.empty_like(f)
    out = {}
    for restriction, methods, suffix in (("mean", KRYLOV_METHODS, ""),
                                         ("transpose", ("fgmres", "cg"), "_symmetric")):
        slv = make_solver(restriction)
        for method in methods:
            out[method + suffix] = _time_method(torch, slv, method, f, pb, pt, tol, phi)
        del slv
        torch.cuda.empty_cache()
    for method, d in out.items():
        d["ratio_to_fgmres"] = d["solve_ms"] / out["fgmres"]["solve_ms"]
        log(f"  {method:18s} {d['solve_ms']:8.2f} ms  {d['iterations']:3d} it  "
            f"{d['preconditioner_applications']:3d} M  ratio {d['ratio_to_fgmres']:.3f}")
    return out


def _time_method(torch, slv, method, f, pb, pt, tol, phi):
    """One untimed solve, then the median of 3 event-timed solves."""
    res, napp = slv.krylov_solve(f, pb, pt, method=method, tol=tol, out=phi)
    times = []
    for _ in range(3):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        res, napp = slv.krylov_solve(f, pb, pt, method=method, tol=tol, out=phi)
        e1.record()
        e1.synchronize()
        times.append(e0.elapsed_time(e1))
    return dict(solve_ms=statistics.median(times), iterations=res.iterations, preconditioner_applications=napp,
                converged=res.converged, final_relres=res.final_relres)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "sharding of this solver is a design, not part of this build.", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_1812_08606_amd as gm  # raises if the HIP library is missing
    from workloads import make_config, probe_box_mask

    dev = torch.device("cuda:0")
    # smoothing sweeps of the benchmark step (None: the library default)
    nu_kw = {"nu_pre": args.nu_pre, "nu_post": args.nu_post}
    step_kw = dict(nu_kw, warm_cycle=args.warm_cycle)
    n = args.n
    N = n ** 3
    h = 1.0 / n
    c5 = args.workload == "c5"
    cfg = int(args.workload[1])
    t_gen = time.perf_counter()
    p = make_config(cfg, n=n)
    a0 = torch.tensor(p.a, device=dev)
    f0 = torch.tensor(p.f, device=dev)
    del p.a, p.f
    log(f"inputs: workload {args.workload} ({p.name}), generated in {time.perf_counter() - t_gen:.1f}s")
    mask = None if c5 else torch.tensor(probe_box_mask(n), device=dev)

    def probe_loss(phi):
        idx = torch.nonzero(mask)
        k, j, i = idx[:, 0], idx[:, 1], idx[:, 2]
        gx = (phi[k, j, i + 1] - phi[k, j, i - 1]) / (2 * h)
        gy = (phi[k, j + 1, i] - phi[k, j - 1, i]) / (2 * h)
        gz = (phi[k + 1, j, i] - phi[k - 1, j, i]) / (2 * h)
        return ((gx ** 2 + gy ** 2 + gz ** 2) * h ** 3).sum()

    def run_c3(precision):
        solver = gm.GMGPoisson(a0, precision=precision, **step_kw)
        phi = torch.empty_like(a0)
        lam = torch.empty_like(a0)
        grad = torch.empty_like(a0)
        # dL/dphi of the probe-box loss at the solution (fixed input of the backward)
        solver.solve(f0, p.phi_bot, p.phi_top, args.tol, out=phi)
        leaf = phi.detach().clone().requires_grad_(True)
        probe_loss(leaf).backward()
        gphi = leaf.grad.detach().contiguous()
        del leaf
        info = {"solves": []}

        def step():
            solver.update_coefficient(a0)
            r1 = solver.solve(f0, p.phi_bot, p.phi_top, args.tol, out=phi)
            r2 = solver.solve(gphi, 0.0, 0.0, args.tol, out=lam)
            solver.face_flux_grad_into(phi, lam, p.phi_bot, p.phi_top, grad)
            info["solves"] = [r1, r2]

        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / args.steps
        solves = info["solves"]
        # forward solve alone, timed with events on the solver's stream
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        solve_ms = []
        for _ in range(3):
            e0.record()
            solver.solve(f0, p.phi_bot, p.phi_top, args.tol, out=phi)
            e1.record()
            e1.synchronize()
            solve_ms.append(e0.elapsed_time(e1))
        # coefficient renewal alone (hierarchy rebuild and coarsest inverse)
        setup_ms = []
        for _ in range(3):
            e0.record()
            solver.update_coefficient(a0)
            e1.record()
            e1.synchronize()
            setup_ms.append(e0.elapsed_time(e1))
        prof = {}
        if not args.no_profile:
            solver.profile(True)
            solver.profile_reset()
            for _ in range(args.steps):
                step()
            prof = solver.profile_read()
            solver.profile(False)
        out = dict(ms_per_step=ms, solve_ms=statistics.median(solve_ms), setup_ms=statistics.median(setup_ms),
                   solves=solves, prof=prof,
                   prof_steps=args.steps, levels=solver.levels, solves_per_step=2, phi=phi.cpu())
        del solver, phi, lam, grad, gphi
        torch.cuda.empty_cache()
        return out

    def run_c5(precision):
        # the densities behind the generator's a = 1 + kappa n_e, f = 50 (n_p - n_e)
        kappa = p.meta["kappa"]
        ne0 = (a0 - 1.0) / kappa
        np0 = f0 / 50.0 + ne0
        # elliptic side (Sec. 2.2): P = eps0/e + tau_eff (mu_p n_p + mu_e n_e)
        # is the generator's coefficient divided by 50 plus an ion term (ions
        # 100 times slower than electrons); the right side of e18 is the
        # generator's divided by 50 plus the diffusion term (tau_eff D / h^2 =
        # 0.59 at 768^3)
        step_prm = dict(eps0_over_e=1.0 / 50.0, tau_eff=1.0, mu_e=kappa / 50.0, mu_p=kappa / 5000.0,
                        De=(1e-6, 1e-6, 1e-6))
        solver = gm.GMGPoisson(a0, precision=precision, **step_kw)
        phi = torch.zeros_like(a0)
        a_t = torch.empty_like(a0)
        f_t = torch.empty_like(f0)
        E = tuple(torch.empty_like(a0) for _ in range(4))
        state = {"t": 0, "first": True, "solves": []}

        def step():
            t = state["t"]
            ne_t = torch.roll(ne0, t, dims=0)
            np_t = torch.roll(np0, t, dims=0)
            solver.assemble_elliptic(ne_t, np_t, out=(a_t, f_t), **step_prm)
            del ne_t, np_t
            solver.update_coefficient(a_t)
            r = solver.solve(f_t, p.phi_bot, p.phi_top, args.tol, out=phi,
                             x0=None if state["first"] else phi)
            solver.electric_field(phi, p.phi_bot, p.phi_top, out=E)
            state["first"] = False
            state["t"] = t + 1
            state["solves"].append(r)

        for _ in range(args.warmup):
            step()
        state["solves"] = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / args.steps
        solves = list(state["solves"])
        prof = {}
        if not args.no_profile:
            solver.profile(True)
            solver.profile_reset()
            for _ in range(2):
                step()
            prof = solver.profile_read()
            solver.profile(False)
        out = dict(ms_per_step=ms, solve_ms=None, solves=solves, prof=prof, prof_steps=2,
                   prof_solves=list(state["solves"][-2:]), levels=solver.levels, solves_per_step=1)
        del solver, phi, a_t, f_t, E, ne0, np0
        torch.cuda.empty_cache()
        return out

    run = run_c5 if c5 else run_c3
    log("mixed precision run ...")
    mixed = run("mixed")
    its_mixed = [r.iterations for r in mixed["solves"]]
    log(f"mixed: {mixed['ms_per_step']:.2f} ms/step, iterations {its_mixed}, "
        f"relres {[float(f'{r.final_relres:.2e}') for r in mixed['solves']]}")
    fp64 = None
    if not args.no_fp64:
        log("fp64 run ...")
        fp64 = run("fp64")
        log(f"fp64: {fp64['ms_per_step']:.2f} ms/step, iterations {[r.iterations for r in fp64['solves']]}")

    # -- the Krylov methods of the comparison in Sec. 5.3 (Table t1): the
    # forward solve from zero with each method, one V-cycle per
    # preconditioner application, event-timed (median of 3) ----------------
    krylov = None
    if not c5 and not args.no_krylov:
        log("Krylov method comparison (mixed, V-cycle preconditioner) ...")
        krylov = time_krylov_methods(torch, lambda r: gm.GMGPoisson(a0, precision="mixed", restriction=r), f0,
                                     p.phi_bot, p.phi_top, args.tol)
        torch.cuda.empty_cache()

    # -- the same comparison on the meshes of Table t1 / t2 (unit cube,
    # h_z < h_x = h_y), variable a (the semi-implicit scheme's problem) and
    # a = 1 (the explicit scheme's constant-coefficient problem) ------------
    krylov_meshes = None
    if not c5 and not args.no_krylov and args.krylov_meshes:
        from workloads import config_streamer_mesh
        krylov_meshes = {}
        for spec in args.krylov_meshes.split(","):
            mx, my, mz = (int(v) for v in spec.split("x"))
            t_gen = time.perf_counter()
            q = config_streamer_mesh(mx, my, mz)
            aq = torch.tensor(q.a, device=dev)
            fq = torch.tensor(q.f, device=dev)
            del q.a, q.f
            log(f"Krylov comparison on the {spec} mesh (inputs in {time.perf_counter() - t_gen:.1f}s) ...")
            entry = {"cells": mx * my * mz, "h": list(q.h)}
            for label, coef in (("variable_a", aq), ("constant_a", torch.ones_like(aq))):
                log(f"  {label} (max a = {float(coef.max()):g})")
                entry[label] = time_krylov_methods(
                    torch, lambda r, coef=coef: gm.GMGPoisson(coef, precision="mixed", restriction=r), fq,
                    q.phi_bot, q.phi_top, args.tol)
                torch.cuda.empty_cache()
                # the solver as the benchmark step runs it: full multigrid
                # cycles from zero with the step's smoothing
                solver = gm.GMGPoisson(coef, precision="mixed", **step_kw)
                phi_m = torch.empty_like(fq)
                res = solver.solve(fq, q.phi_bot, q.phi_top, args.tol, out=phi_m)
                times = []
                for _ in range(3):
                    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    e0.record()
                    res = solver.solve(fq, q.phi_bot, q.phi_top, args.tol, out=phi_m)
                    e1.record()
                    e1.synchronize()
                    times.append(e0.elapsed_time(e1))
                entry[label]["fgmres_fmg_step_smoothing"] = dict(
                    solve_ms=statistics.median(times), iterations=res.iterations, converged=res.converged,
                    final_relres=res.final_relres, smoothing=[args.nu_pre, args.nu_post])
                log(f"  fgmres + FMG V({args.nu_pre},{args.nu_post}) {statistics.median(times):8.2f} ms "
                    f"{res.iterations:3d} it")
                del solver, phi_m
                torch.cuda.empty_cache()
            krylov_meshes[spec] = entry
            del aq, fq
            torch.cuda.empty_cache()

    # -- smoothers (Sec. 3.2): red-black symmetric Gauss-Seidel (the default,
    # full multigrid cycles on a cold solve; and with V-cycles) against the
    # paper's Chebyshev(2)+SSOR smoother (V-cycles), forward solve from zero;
    # renewal = hierarchy rebuild (+ the Chebyshev bound estimate) ----------
    smoothers = None
    if not c5 and not args.no_krylov and not args.no_smoothers:
        log("smoother comparison (mixed, forward solve from zero) ...")
        smoothers = {}
        phi = torch.empty_like(a0)
        for label, kw in (("rbgs_fmg", dict(nu_kw)), ("rbgs_vcycle", dict(nu_kw, cold_cycle="vcycle")),
                          ("chebyshev_vcycle", {"smoother": "chebyshev"})):
            solver = gm.GMGPoisson(a0, precision="mixed", **kw)
            res = solver.solve(f0, p.phi_bot, p.phi_top, args.tol, out=phi)
            times, renew = [], []
            for _ in range(3):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                res = solver.solve(f0, p.phi_bot, p.phi_top, args.tol, out=phi)
                e1.record()
                e1.synchronize()
                times.append(e0.elapsed_time(e1))
                e0.record()
                solver.update_coefficient(a0)
                e1.record()
                e1.synchronize()
                renew.append(e0.elapsed_time(e1))
            solver.profile(True)
            solver.profile_reset()
            solver.solve(f0, p.phi_bot, p.phi_top, args.tol, out=phi)
            prof = solver.profile_read()
            solver.profile(False)
            kernels = []
            for name, (tot, cnt) in sorted(prof.items(), key=lambda kv: -kv[1][0])[:8]:
                base, level = split_name(name)
                bpc = cheb_bytes_per_cell(base, level, 4) if level is not None and level >= 0 else None
                gbs = bpc * N / 8 ** level * cnt / (tot * 1e-3) / 1e9 if bpc else None
                kernels.append({"kernel": name, "ms": round(tot, 3), "launches": cnt,
                                "GBps": round(gbs) if gbs else None})
            smoothers[label] = dict(solve_ms=statistics.median(times), renewal_ms=statistics.median(renew),
                                    iterations=res.iterations, converged=res.converged,
                                    final_relres=res.final_relres, top_kernels=kernels)
            if label.startswith("chebyshev"):
                smoothers[label]["lambda_per_level"] = solver.chebyshev_estimates()
            log(f"  {label:17s} solve {smoothers[label]['solve_ms']:8.2f} ms  {res.iterations:3d} it  "
                f"renewal {smoothers[label]['renewal_ms']:7.2f} ms  top {kernels[0]['kernel']} "
                f"{kernels[0]['GBps']} GB/s")
            del solver
        del phi
        torch.cuda.empty_cache()

    if args.copy_calibration:
        src = torch.ones(1 << 27, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)  # 1 GiB read + 1 GiB written
        torch.cuda.synchronize()
        log("copy calibration: 1 GiB read + 1 GiB written by one device copy")
        del src, dst

    # -- per-kernel tables and rooflines from the event passes -------------
    def tables(run_out, s_bytes, its):
        ps = run_out["prof_steps"]
        # iterations of the solves inside the profiled pass (c3: the same every step)
        its_prof = [r.iterations for r in run_out["prof_solves"]] if c5 else its * ps
        table, total = kernel_table(run_out["prof"], ps, its_prof, s_bytes, N)
        if table:
            log(f"{'kernel':34s} {'ms/step':>9s} {'launch':>7s} {'avg ms':>9s} {'GB/s':>8s}")
            for name, ms_s, cnt, avg, gbs, _ in table:
                log(f"{name:34s} {ms_s:9.3f} {cnt:7.1f} {avg:9.4f} {gbs if gbs else float('nan'):8.0f}")
        traffic_ok = n == 512 and args.workload == "c3"
        roof = roofline_of(table, run_out["ms_per_step"], traffic_ok)
        model = (total / ps) / (run_out["ms_per_step"] * 1e-3) / 1e9 if total else None
        return table, roof, model

    table, roofline, model_gbs = tables(mixed, 4, its_mixed)
    fp64_table = fp64_roofline = fp64_model_gbs = None
    if fp64 is not None:
        log("fp64 kernels:")
        fp64_table, fp64_roofline, fp64_model_gbs = tables(fp64, 8, [r.iterations for r in fp64["solves"]])

    # -- CPU oracle baseline ------------------------------------------------
    cpu = None
    if not args.no_cpu_baseline:
        from oracle.fgmres import solve_poisson
        m = args.cpu_n
        q = make_config(cfg, n=m)
        log(f"cpu baseline: oracle fp64 solve at {m}^3 ...")
        t0 = time.perf_counter()
        res = solve_poisson(q.a, q.f, q.h, q.phi_bot, q.phi_top, tol=args.tol, precision="fp64")
        dt = time.perf_counter() - t0
        cpu = {"value": m ** 3 / dt, "unit": "cells/s", "cores": 1, "kind": "oracle",
               "sample": (f"one FP64 NumPy oracle solve to {args.tol:g} from a zero guess of the same "
                          f"workload {args.workload} generator at {m}^3 ({res.iterations} "
                          f"steps, {dt:.1f} s; NumPy element-wise work on one thread, host has "
                          f"{os.cpu_count()} cpus)")}
        log(f"cpu baseline: {dt:.1f}s, {res.iterations} steps")

    sps = mixed["solves_per_step"]
    value = sps * N / (mixed["ms_per_step"] * 1e-3)
    desc = {1: "constant a = 1, Gaussian source", 2: "filament, max(a)=1e3", 3: "filament, max(a)=1e4",
            4: "filament, max(a)=1e3, probe-box loss", 5: "two filaments, max(a)=1e4"}[cfg]
    if c5:
        cyc = "full multigrid cycle" if args.warm_cycle == "fmg" else "V-cycle"
        workload = (f"{desc} {n}^3 time loop, tol {args.tol:g}, FGMRES(10) + {cyc} (V({args.nu_pre},{args.nu_post}) "
                    "smoothing) mixed "
                    "(float32 cycle, float64 outer); step = advect the densities (roll) + coefficient "
                    "and right side of e18 from them + renewal + warm-started solve + E = -grad phi")
    else:
        workload = (f"{desc} {n}^3, tol {args.tol:g}, FGMRES(10) + full multigrid cycle (V({args.nu_pre},{args.nu_post}) "
                    "smoothing) mixed (float32 cycle, float64 outer); step = renewal + forward solve + "
                    "adjoint solve + dL/da, both from no initial guess")
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "cells/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": mixed["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {
            "workload": workload,
            "grid": [n, n, n],
            "levels": len(mixed["levels"]),
            "solves_per_step": sps,
        },
        "iterations": its_mixed,
        "final_relres": [r.final_relres for r in mixed["solves"]],
        "solve_ms": mixed["solve_ms"],
        "solve_cells_per_s": N / (mixed["solve_ms"] * 1e-3) if mixed["solve_ms"] else None,
        "setup_ms": mixed.get("setup_ms"),
        "setup_and_solve_cells_per_s": (N / ((mixed["setup_ms"] + mixed["solve_ms"]) * 1e-3)
                                        if mixed.get("setup_ms") and mixed["solve_ms"] else None),
        "model_gbs": model_gbs,
        "roofline": roofline,
        "kernels": kernel_rows(table),
        "cpu_baseline": cpu,
        "krylov_methods": krylov,
        "krylov_meshes": krylov_meshes,
        "smoothers": smoothers,
    }
    if fp64 is not None:
        line["fp64"] = {
            "ms_per_step": fp64["ms_per_step"],
            "value": sps * N / (fp64["ms_per_step"] * 1e-3),
            "solve_ms": fp64["solve_ms"],
            "setup_ms": fp64.get("setup_ms"),
            "solve_cells_per_s": N / (fp64["solve_ms"] * 1e-3) if fp64["solve_ms"] else None,
            "iterations": [r.iterations for r in fp64["solves"]],
            "final_relres": [r.final_relres for r in fp64["solves"]],
            "model_gbs": fp64_model_gbs,
            "roofline": fp64_roofline,
            "kernels": kernel_rows(fp64_table) if fp64_table else None,
        }
        line["mixed_speedup_vs_fp64"] = fp64["ms_per_step"] / mixed["ms_per_step"]
        if "phi" in mixed and "phi" in fp64:  # forward solutions of the two precisions
            d = (mixed["phi"] - fp64["phi"]).norm() / fp64["phi"].norm()
            line["phi_rel_diff_mixed_vs_fp64"] = float(d)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
