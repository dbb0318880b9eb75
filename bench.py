#!/usr/bin/env python3
"""Benchmark of the GMG-preconditioned FGMRES solve on one MI355X.

Workload: the 512^3 single-filament problem (max(a) = 1e4, f = 50 (n_p -
n_e)), unit cube, phi = 0 / 1 on the plates, tolerance 1e-8, FGMRES(10) with
one V(2,2)-cycle per step.  One benchmark step is one pass of the whole hot
path: coefficient renewal (hierarchy rebuild), the forward solve from a zero
guess, the adjoint solve for a fixed dL/dphi and the dL/da face-flux kernel.
Each step therefore holds two converged 1e-8 solves; ``value`` counts
cells x solves per second over the timed steps (inputs resident in HBM).

Prints one JSON line on stdout; progress goes to stderr.

  python bench.py [--steps K] [--warmup W] [--gpus 1] [--n 512]
"""
import argparse
import json
import os
import statistics
import sys
import time

os.environ.setdefault("OPENBLAS_NUM_THREADS", "1")  # the CPU oracle leg runs on one core

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "converged cells/s per 1e-8 Poisson solve + HBM GB/s, FP64 vs mixed, 512^3"
PEAK_HBM_GBS = 8000.0  # MI355X HBM3E


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 side-by-side run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-n", type=int, default=128, help="edge of the CPU-oracle sample grid")
    ap.add_argument("--no-profile", action="store_true", help="skip the per-kernel event pass")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a 1 GiB device copy (for hardware-counter scaling)")
    return ap.parse_args()


# ---------------------------------------------------------------------------
# Algorithmic (compulsory) bytes per finest-level cell of each kernel: every
# kernel reads each input once and writes each output once at element
# granularity.  s = bytes of the V-cycle precision; j = vectors in a
# multi-dot / multi-axpy launch; k = preconditioned vectors in an update.
# ---------------------------------------------------------------------------
def bytes_per_cell(name, s, nv=0):
    base = name.rsplit("_", 2)[0] if name.endswith(("_f32", "_f64")) else name
    if base == "gs":  # half-sweep: x (all) + a (all) + b (own colour) read, x (own colour) written
        return 3 * s
    if base == "gs_first":  # b_in (float64) + a read; x (and the float32 copy of b) written
        return 8 + s + s + (s if s == 4 else 0)
    if base == "resid_restrict":  # x, a, b read; coarse b (1/8) written
        return 3 * s + s / 8
    if base == "prolong_add":  # x, coarse x (1/8) read; x written
        return 2 * s + s / 8
    return None


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
    return None


def nv_sequence(iterations, restart):
    """Vectors per Arnoldi step j (j+1 within each restart cycle)."""
    seq = []
    for it in range(iterations):
        seq.append(it % restart + 1)
    return seq


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "sharding of this solver is a design, not part of this build.", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_1812_08606_amd as gm  # raises if the HIP library is missing
    from workloads import make_config, probe_box_mask

    dev = torch.device("cuda:0")
    n = args.n
    N = n ** 3
    t_gen = time.perf_counter()
    p = make_config(3, n=n)
    mask = torch.tensor(probe_box_mask(n), device=dev)
    a = torch.tensor(p.a, device=dev)
    f = torch.tensor(p.f, device=dev)
    del p.a, p.f
    log(f"inputs: filament {n}^3, max(a)=1e4, generated in {time.perf_counter() - t_gen:.1f}s")
    h = 1.0 / n

    def probe_loss(phi):
        idx = torch.nonzero(mask)
        k, j, i = idx[:, 0], idx[:, 1], idx[:, 2]
        gx = (phi[k, j, i + 1] - phi[k, j, i - 1]) / (2 * h)
        gy = (phi[k, j + 1, i] - phi[k, j - 1, i]) / (2 * h)
        gz = (phi[k + 1, j, i] - phi[k - 1, j, i]) / (2 * h)
        return ((gx ** 2 + gy ** 2 + gz ** 2) * h ** 3).sum()

    def run(precision):
        solver = gm.GMGPoisson(a, precision=precision)
        phi = torch.empty_like(a)
        lam = torch.empty_like(a)
        grad = torch.empty_like(a)
        # dL/dphi of the probe-box loss at the solution (fixed input of the backward)
        r = solver.solve(f, p.phi_bot, p.phi_top, args.tol, out=phi)
        leaf = phi.detach().clone().requires_grad_(True)
        probe_loss(leaf).backward()
        gphi = leaf.grad.detach().contiguous()
        del leaf

        info = {}

        def step():
            solver.update_coefficient(a)
            r1 = solver.solve(f, p.phi_bot, p.phi_top, args.tol, out=phi)
            r2 = solver.solve(gphi, 0.0, 0.0, args.tol, out=lam)
            solver.face_flux_grad_into(phi, lam, p.phi_bot, p.phi_top, grad)
            info["fwd"], info["adj"] = r1, r2

        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ms = (t1 - t0) * 1e3 / args.steps
        # forward solve alone, timed with events on the solver's stream
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        solve_ms = []
        for _ in range(3):
            e0.record()
            solver.solve(f, p.phi_bot, p.phi_top, args.tol, out=phi)
            e1.record()
            e1.synchronize()
            solve_ms.append(e0.elapsed_time(e1))
        prof = {}
        if not args.no_profile:
            solver.profile(True)
            solver.profile_reset()
            for _ in range(args.steps):
                step()
            prof = solver.profile_read()
            solver.profile(False)
        out = dict(ms_per_step=ms, solve_ms=statistics.median(solve_ms), fwd=info["fwd"], adj=info["adj"],
                   prof=prof, levels=solver.levels)
        del solver, phi, lam, grad, gphi
        torch.cuda.empty_cache()
        return out

    log("mixed precision run ...")
    mixed = run("mixed")
    fwd, adj = mixed["fwd"], mixed["adj"]
    log(f"mixed: {mixed['ms_per_step']:.2f} ms/step, forward {fwd.iterations} steps "
        f"(relres {fwd.final_relres:.2e}), adjoint {adj.iterations} steps, solve {mixed['solve_ms']:.2f} ms")
    fp64 = None
    if not args.no_fp64:
        log("fp64 run ...")
        fp64 = run("fp64")
        log(f"fp64: {fp64['ms_per_step']:.2f} ms/step, forward {fp64['fwd'].iterations} steps, "
            f"solve {fp64['solve_ms']:.2f} ms")

    if args.copy_calibration:
        src = torch.empty(1 << 27, dtype=torch.float64, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: 1 GiB read + 1 GiB written by one device copy")
        del src, dst

    # -- per-kernel roofline from the event pass --------------------------
    s = 4
    its_f, its_a = fwd.iterations, adj.iterations
    restart = 10
    nvs = nv_sequence(its_f, restart) + nv_sequence(its_a, restart)
    table = []
    total_bytes = 0.0
    for name, (tot_ms, cnt) in sorted(mixed["prof"].items(), key=lambda kv: -kv[1][0]):
        bpc = None
        if "_fine_" in name:
            bpc = bytes_per_cell(name, s)
            per_launch = None if bpc is None else bpc * N
            tb = None if per_launch is None else per_launch * cnt
        else:
            tb = None
            if name.startswith("op_multidot") or name == "axpy_norm":
                tb = sum(outer_bytes(name, nv, s) for nv in nvs) * N * args.steps
            elif name.startswith("update"):
                b_upd = 0.0
                for its in (its_f, its_a):
                    left = its
                    while left > 0:
                        k = min(left, restart)
                        b_upd += outer_bytes(name, k, s)
                        left -= k
                tb = b_upd * N * args.steps
            elif outer_bytes(name, 0, s) is not None:
                tb = outer_bytes(name, 0, s) * N * cnt
        gbs = tb / (tot_ms * 1e-3) / 1e9 if tb else None
        if tb:
            total_bytes += tb
        table.append((name, tot_ms / args.steps, cnt // max(args.steps, 1), tot_ms / cnt, gbs))
    if table:
        log(f"{'kernel':34s} {'ms/step':>9s} {'launch':>7s} {'avg ms':>9s} {'GB/s':>8s}")
        for name, ms_s, cnt, avg, gbs in table:
            log(f"{name:34s} {ms_s:9.3f} {cnt:7d} {avg:9.4f} {gbs if gbs else float('nan'):8.0f}")
    roofline = None
    dom = next((t for t in table if t[4] is not None), None)
    if dom is not None:
        name, ms_s, cnt, avg_ms, gbs = dom
        roofline = {
            "bound": "hbm",
            "kernel": name,
            "achieved": round(gbs, 1),
            "peak": PEAK_HBM_GBS,
            "unit": "GB/s",
            "frac": round(gbs / PEAK_HBM_GBS, 4),
            "traffic": None,
            "avg_launch_ms": round(avg_ms, 5),
            "bytes_per_launch": bytes_per_cell(name, s) * N if "_fine_" in name else None,
            "share_of_step": round(ms_s / mixed["ms_per_step"], 3),
        }

    # -- CPU oracle baseline ------------------------------------------------
    cpu = None
    if not args.no_cpu_baseline:
        from oracle.fgmres import solve_poisson
        m = args.cpu_n
        q = make_config(3, n=m)
        log(f"cpu baseline: oracle fp64 solve at {m}^3 ...")
        t0 = time.perf_counter()
        res = solve_poisson(q.a, q.f, q.h, q.phi_bot, q.phi_top, tol=args.tol, precision="fp64")
        dt = time.perf_counter() - t0
        cpu = {"value": m ** 3 / dt, "unit": "cells/s", "cores": 1, "kind": "oracle",
               "sample": (f"one FP64 NumPy oracle solve to {args.tol:g} of the same filament generator at "
                          f"{m}^3 ({res.iterations} steps, {dt:.1f} s; NumPy element-wise work on one "
                          f"thread, host has {os.cpu_count()} cpus)")}
        log(f"cpu baseline: {dt:.1f}s, {res.iterations} steps")

    value = 2 * N / (mixed["ms_per_step"] * 1e-3)
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
            "workload": (f"filament {n}^3, max(a)=1e4, tol {args.tol:g}, FGMRES(10) + V(2,2) mixed "
                         "(float32 V-cycle, float64 outer); step = renewal + forward solve + adjoint "
                         "solve + dL/da"),
            "grid": [n, n, n],
            "levels": len(mixed["levels"]),
            "solves_per_step": 2,
        },
        "iterations": {"forward": its_f, "adjoint": its_a},
        "final_relres": fwd.final_relres,
        "solve_ms": mixed["solve_ms"],
        "solve_cells_per_s": N / (mixed["solve_ms"] * 1e-3),
        "model_gbs": (total_bytes / args.steps) / (mixed["ms_per_step"] * 1e-3) / 1e9 if total_bytes else None,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    if fp64 is not None:
        line["fp64"] = {
            "ms_per_step": fp64["ms_per_step"],
            "value": 2 * N / (fp64["ms_per_step"] * 1e-3),
            "solve_ms": fp64["solve_ms"],
            "solve_cells_per_s": N / (fp64["solve_ms"] * 1e-3),
            "iterations": {"forward": fp64["fwd"].iterations, "adjoint": fp64["adj"].iterations},
            "final_relres": fp64["fwd"].final_relres,
        }
        line["mixed_speedup_vs_fp64"] = fp64["solve_ms"] / mixed["solve_ms"]
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
