#!/usr/bin/env python
"""Throughput of the real-shifted multigrid Helmholtz solver on one MI355X.

Workload: 2D 1024 x 1024 cells, layered medium (8 layers, velocity 1.5-4.5, +-10 %
noise smoothed over 20 cells), 10 points per wavelength at the largest slowness,
20-cell absorbing layer, point source at the centre; FGMRES(20) to a relative
residual of 1e-6, preconditioned by the 3-level W(1,1) cycle (damped Jacobi 0.8)
with the real-shifted coarsest Galerkin operator (alpha* of the grid-to-grid
dispersion analysis), a level-2 real shift and a complex shift of the
preconditioner.

One step = one pass of the whole path on resident inputs: numerical setup
(coefficients, Galerkin operators, coarsest factorisation) + solve, with the
FP32-complex cycle inside FP64 FGMRES.  `value` = steps per second.  The FP64-cycle
path, solve-only rates, per-kernel-class HIP-event timings, the roofline figure of
the dominant kernel class and the FP64 CPU oracle timed on a bounded sample of the
same workload are reported in the same JSON line.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_2d_1024_layered.json")


def measured_traffic(cls):
    """HBM bytes per launch of a kernel class from the committed FETCH_SIZE/WRITE_SIZE runs.

    The record stores the SHA-256 of the kernel sources it was taken on; once any of them
    has changed the counters no longer describe the kernels and None is returned."""
    import hashlib
    try:
        rec = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    for f, h in rec.get("source_sha256", {}).items():
        path = os.path.join(ROOT, "paper_2604_19501_amd", "csrc", f)
        if not os.path.exists(path) or hashlib.sha256(open(path, "rb").read()).hexdigest() != h:
            return None
    c = rec.get("classes", {}).get(cls)
    return None if c is None else c["bytes_per_launch"]


def workload(n):
    import synth
    return synth.config2(n)


def make_solver(p, prec):
    from paper_2604_19501_amd import from_problem
    return from_problem(p, nu=(p.nu_pre, p.nu_post), cycle_prec=prec)


def timed_steps(s, p, q, steps, warmup, refactor=True):
    import torch
    its = []
    for _ in range(warmup):
        if refactor:
            s.refactor()
        x, info = s.solve(q, tol=p.tol, max_iter=2000)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        if refactor:
            s.refactor()
        x, info = s.solve(q, tol=p.tol, max_iter=2000)
        its.append(info["iterations"])
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    return dt, its, info, x


def bytes_model(cls, p, info, iters, restart):
    """algorithmic HBM bytes of one launch of a kernel class.

    Per-unit figures: fine node N1, level-2 node N2, factor entry / update entry of the
    coarsest elimination (info from helm_get_info), cb = bytes of a cycle complex."""
    d = p.dim
    N1, N2, N3 = info["N1"], info["N2"], info["N3"]
    cb = info["cycle_complex_bytes"]
    K = 3 ** d
    if cls == "l1_restrict":      # b (c128) + m (f32) per fine node, r2 per level-2 node
        return N1 * (16 + 4) + N2 * cb
    if cls == "l1_sweep":         # b (c128) + m (f32) + z out per fine node, e2 per level-2 node
        return N1 * (16 + 4 + cb) + N2 * cb
    if cls == "l2_sweep":         # coefficients (K) + b2 + x in + x out per level-2 node
        return N2 * cb * (K + 3)
    if cls == "l2_restrict":      # coefficients + b2 + x per level-2 node
        return N2 * cb * (K + 2)
    if cls == "nd_fwd":           # [A^-1; C A^-1] once, right-hand side gather, updates written and read
        per_solve = (info["L_entries"] * cb + N3 * (cb + 4) + info["upd_entries"] * (2 * cb + 4) + N3 * cb)
        return per_solve / info["fwd_launches"]
    if cls == "nd_bwd":           # -A^-1 B once, boundary gather, g read and x written
        per_solve = info["W_entries"] * cb + info["upd_entries"] * (cb + 4) + 2 * N3 * cb
        return per_solve / max(1, info["bwd_launches"])
    if cls == "arnoldi":          # two passes, each reading z, m and V_0..V_j; V_{j+1} written
        js = [k % restart for k in range(iters)]
        jm = sum(js) / max(1, len(js))
        return N1 * (2 * (cb + 8) + 16 + 32 * (jm + 1))
    return None


def cpu_baseline(p, its_gpu, budget_iters=20):
    """the FP64 oracle on the same workload: setup + the first FGMRES iterations, extrapolated."""
    from oracle import fgmres, multigrid
    t0 = time.perf_counter()
    H = multigrid.from_problem(p)
    t1 = time.perf_counter()
    r = fgmres.solve(H, p.rhs(), tol=p.tol, restart=p.restart, max_iter=budget_iters)
    t2 = time.perf_counter()
    per_it = (t2 - t1) / max(1, r.iterations)
    est = (t1 - t0) + per_it * its_gpu
    return {"value": 1.0 / est, "unit": "solves/s", "cores": 1, "kind": "oracle",
            "sample": "oracle setup (%.1f s) + first %d FGMRES iterations (%.2f s/iteration) of the same "
                      "1024^2 solve, extrapolated to %d iterations; scipy sparse kernels and SuperLU run "
                      "single-threaded" % (t1 - t0, r.iterations, per_it, its_gpu),
            "setup_s": t1 - t0, "s_per_iteration": per_it}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=1024)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--pmc-pass", action="store_true",
                    help="for hardware-counter runs: a 256 MiB device copy (calibrates FETCH_SIZE/WRITE_SIZE "
                         "against known bytes) followed by one setup+solve step, no timing output")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the solver has no multi-GPU path (requested --gpus %d)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    p = workload(args.n)
    q = torch.from_numpy(p.rhs()).cuda()
    if args.pmc_pass:
        a = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda")      # 256 MiB
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        s32 = make_solver(p, "f32")
        s32.refactor()
        x, info = s32.solve(q, tol=p.tol, max_iter=2000)
        torch.cuda.synchronize()
        print(json.dumps({"pmc_pass": True, "iterations": info["iterations"], "copy_bytes": 2 * a.numel() * 8}))
        return
    # mixed precision: FP32 cycle, FP64 FGMRES
    s32 = make_solver(p, "f32")
    dt, its, info, x = timed_steps(s32, p, q, args.steps, args.warmup)
    dt_solve, _, _, _ = timed_steps(s32, p, q, args.steps, 0, refactor=False)
    # instrumented pass: per-kernel-class HIP-event timings on the solver's stream
    s32.set_timing(True)
    s32.refactor()
    s32.solve(q, tol=p.tol, max_iter=2000)
    torch.cuda.synchronize()
    kt = s32.kernel_times()
    s32.set_timing(False)
    sinfo = s32.info()
    # true residual recomputed by the library in FP64 on the final iterate
    res = info["true_rel_residual"]
    out = {
        "metric": "Helmholtz solves/sec at 1e-6 rel. residual (setup+solve per step, FP32 cycle / FP64 FGMRES)",
        "value": 1.0 / dt,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * dt,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64 cycle / c128 FGMRES",
        "data": "synthetic",
        "config": {"workload": "2D %dx%d layered medium, G=10 at max slowness, 20-cell absorbing layer, "
                               "centre point source, FGMRES(20) tol 1e-6, W(1,1) cycle, alpha=%.4f, "
                               "alpha2=%.3f, beta=%.2f" % (args.n, args.n, p.alpha, p.alpha2, p.beta),
                   "unknowns": p.N, "iterations": its[-1], "true_rel_residual": res},
        "solve_only_per_sec": 1.0 / dt_solve,
        "setup_ms": 1e3 * (dt - dt_solve),
        "kernel_ms": {k: round(v[0], 4) for k, v in kt.items()},
        "kernel_launches": {k: v[1] for k, v in kt.items()},
    }
    # FP64 cycle on the same inputs
    if not args.no_fp64:
        s32.close()
        del s32
        torch.cuda.empty_cache()
        s64 = make_solver(p, "f64")
        dt64, its64, info64, _ = timed_steps(s64, p, q, args.steps, args.warmup)
        dts64, _, _, _ = timed_steps(s64, p, q, args.steps, 0, refactor=False)
        out["fp64"] = {"value": 1.0 / dt64, "iterations": its64[-1], "solve_only_per_sec": 1.0 / dts64,
                       "true_rel_residual": info64["true_rel_residual"]}
        out["speedup_mixed_vs_fp64"] = dt64 / dt
        out["speedup_mixed_vs_fp64_solve_only"] = dts64 / dt_solve
        s64.close()
    # roofline of the dominant kernel class (by HIP-event time) with its algorithmic bytes
    gbs = {}
    for k, (ms, cnt) in kt.items():
        B = bytes_model(k, p, sinfo, its[-1], p.restart)
        if B is not None and cnt > 0 and ms > 0:
            gbs[k] = B / (ms / cnt / 1e3) / 1e9
    out["kernel_achieved_GBs"] = {k: round(v, 1) for k, v in gbs.items()}
    dom = max(kt.items(), key=lambda kv: kv[1][0])[0]
    ms, cnt = kt[dom]
    B = bytes_model(dom, p, sinfo, its[-1], p.restart)
    avg_s = ms / cnt / 1e3
    out["roofline"] = {"bound": "hbm", "achieved": B / avg_s / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": B / avg_s / 1e9 / HBM_PEAK_GBS, "traffic": measured_traffic(dom), "kernel": dom,
                       "bytes_per_launch": B, "avg_launch_us": avg_s * 1e6,
                       "share_of_instrumented_solve": ms / sum(v[0] for v in kt.values())}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(p, its[-1])
    print(json.dumps(out))


if __name__ == "__main__":
    main()
