#!/usr/bin/env python
"""Throughput of the real-shifted multigrid Helmholtz solver on one MI355X.

Default run: the headline workload plus two sub-records, one JSON line.

  headline  2D 1024 x 1024 cells, layered medium (8 layers, velocity 1.5-4.5, +-10 % noise
            smoothed over 20 cells), 10 points per wavelength at the largest slowness,
            20-cell absorbing layer, point source at the centre; FGMRES(20) to a relative
            residual of 1e-6, preconditioned by the 3-level W(1,1) cycle (damped Jacobi 0.8)
            with the real-shifted coarsest Galerkin operator, a level-2 real shift and a
            complex shift of the preconditioner.  One step = numerical set-up (coefficients,
            Galerkin operators, coarsest factorisation) + solve on resident inputs, FP32
            cycle inside FP64 FGMRES; value = steps per second.  Beside it: the FP64-cycle
            rate, per-kernel-class timings, the roofline of the dominant class and the FP64
            CPU oracle's full solve of the same system (time, iterations, and the GPU
            solutions' relative difference to the oracle's).
  workloads.cfg3  3D 256^3 layered (6 layers, noise over 8 cells), G = 12, 7-point stencil,
            27-point Galerkin, W(1,1) with damping 0.6/0.4: set-up + solve steps, mixed and
            FP64, the true residual recomputed with the oracle's assembled operator, and the
            oracle timed on the same recipe at 96^3.
  workloads.cfg4  96 instances (32 each of 256^2, 512^2, 768^2), 4 frequencies, 8 sources
            each: the 768 solves of one batch per step, mixed and FP64, and the oracle's
            full solves of one source per grid size (iterations and difference).

Single workloads (same one-line contract): --workload cfg1 | cfg2 | cfg3 | cfg4 | cfg5
(cfg1: 2D 128^2 homogeneous; cfg5: 3D 128^3 misfit gradient).

    python bench.py [--workload suite] [--steps K] [--warmup W] [--gpus 1]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_2d_1024_layered.json")
METRIC = "Helmholtz solves/sec at 1e-6 rel. residual (setup+solve per step, FP32 cycle / FP64 FGMRES)"


def measured_traffic(cls):
    """HBM bytes per launch of a kernel class from the committed FETCH_SIZE/WRITE_SIZE runs.

    The record stores the SHA-256 of the kernel sources it was taken on; once any of them
    has changed the counters no longer describe the kernels and None is returned."""
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


def cpu_info():
    model = platform.processor() or "unknown"
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                model = ln.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return model, len(os.sched_getaffinity(0))


def make_solver(p, prec, **kw):
    from paper_2604_19501_amd import from_problem
    return from_problem(p, nu=(p.nu_pre, p.nu_post), cycle_prec=prec, **kw)


def sync():
    import torch
    torch.cuda.synchronize()


def free_gpu():
    import gc
    import torch
    gc.collect()
    torch.cuda.empty_cache()


def timed_steps(s, p, q, steps, warmup, refactor=True):
    its = []
    info = x = None
    for _ in range(warmup):
        if refactor:
            s.refactor()
        x, info = s.solve(q, tol=p.tol, max_iter=3000)
    sync()
    t0 = time.perf_counter()
    for _ in range(steps):
        if refactor:
            s.refactor()
        x, info = s.solve(q, tol=p.tol, max_iter=3000)
        its.append(info["iterations"])
    sync()
    return (time.perf_counter() - t0) / steps, its, info, x


def bytes_model(cls, p, info, iters, restart, nr=1):
    """algorithmic HBM bytes of one launch of a kernel class.

    Per-unit figures: fine node N1, level-2 node N2, factor entry / update entry of the
    coarsest elimination (info from helm_get_info), cb = bytes of a cycle complex.  nr
    right-hand sides iterated in lock-step share the operator data (m, the level-2
    coefficients, the factors and the gather indices) and bring their own vectors."""
    d = p.dim
    N1, N2, N3 = info["N1"], info["N2"], info["N3"]
    cb = info["cycle_complex_bytes"]
    K = 3 ** d
    U = info["upd_entries"]
    if getattr(p, "stack", "p5") == "compact" and cls in ("l1_restrict", "l1_sweep", "l2_restrict", "l2_sweep"):
        # the compact stack's plain kernels (one node per thread, neighbours from cache):
        # Jacobi sweeps read x, b, m and write x; a restriction class launch is either the
        # residual (x, b, m in, r out) or the transfer (r in, the coarse right-hand side
        # out): the class's bytes per launch are the two launches' mean
        K2 = info["planes2"]
        mb = cb // 2                            # m in the cycle's real precision
        if cls == "l1_sweep":
            return N1 * ((cb + 16 + cb) * nr + mb)
        if cls == "l1_restrict":
            return (N1 * ((cb + 16 + cb) * nr + mb) + (N1 * cb + N2 * cb) * nr) / 2
        if cls == "l2_sweep":
            return N2 * cb * (K2 + 3 * nr)
        if cls == "l2_restrict":
            return (N2 * cb * (K2 + 3 * nr) + (N2 + N3) * cb * nr) / 2
    # the level-1 diagonal: precomputed complex FP32 (the FP32 cycle) or m in FP64 (8 B either way)
    if cls == "l1_restrict":      # b (c128) per fine node and r2 per level-2 node per rhs; the diagonal
        return N1 * (16 * nr + 8) + N2 * cb * nr
    if cls == "l1_sweep":         # b (c128) + z out per fine node and e2 per level-2 node per rhs; diagonal
        return N1 * ((16 + cb) * nr + 8) + N2 * cb * nr
    # level-2 coefficients: the 3D FP32 cycle stores the complex-symmetric operator's centre
    # and the directions after it (14 planes), otherwise all K
    S = K // 2 + 1 if (cb == 8 and d == 3) else K
    if cls == "l2_sweep":         # coefficients + b2, x in, x out per level-2 node
        return N2 * cb * (S + 3 * nr)
    if cls == "l2_restrict":      # coefficients + b2, x per level-2 node
        return N2 * cb * (S + 2 * nr)
    if cls == "l2_chain":         # two sweeps and a residual in one pass: coefficients + b2, x in,
        return N2 * cb * (S + 3 * nr) + 2 * N3 * cb * nr      # x out; e in and b3 out per level-3 node
    if cls == "cycle_tail":       # the level-1 sweep's bytes; level-2 coefficients, x2 and b2; e3
        return N1 * ((16 + cb) * nr + 8) + N2 * cb * (S + 2 * nr) + N3 * cb * nr
    nb = info.get("coarse_complex_bytes", cb)     # the coarsest solve's precision
    if cls == "nd_fwd":           # [A^-1; C A^-1] once, right-hand side gather, updates written and read
        per_solve = info["L_entries"] * nb + 4 * (N3 + U) + nr * (2 * N3 * nb + 2 * U * nb)
        return per_solve / info["fwd_launches"]
    if cls == "nd_bwd":           # -A^-1 B once, boundary gather, g read and x written
        per_solve = info["W_entries"] * nb + 4 * U + nr * (U * nb + 2 * N3 * nb)
        return per_solve / max(1, info["bwd_launches"])
    if cls == "arnoldi":          # two passes, each reading z, m and V_0..V_j; V_{j+1} written
        js = [k % restart for k in range(iters)]
        jm = sum(js) / max(1, len(js))
        return N1 * (2 * 8 + nr * (2 * cb + 16 + 32 * (jm + 1)))
    return None


def roofline_of(kt, B_of, traffic_of=lambda cls: None):
    """per-class achieved GB/s and the roofline record of the class with the most time;
    kt = {class: (ms, launches)}, B_of(class) = algorithmic bytes per launch"""
    gbs = {}
    for k, (ms, cnt) in kt.items():
        B = B_of(k)
        if B is not None and cnt > 0 and ms > 0:
            gbs[k] = B / (ms / cnt / 1e3) / 1e9
    dom = max(kt.items(), key=lambda kv: kv[1][0])[0]
    ms, cnt = kt[dom]
    B = B_of(dom)
    avg_s = ms / cnt / 1e3
    roof = {"bound": "hbm", "achieved": B / avg_s / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": B / avg_s / 1e9 / HBM_PEAK_GBS, "traffic": traffic_of(dom), "kernel": dom, "bytes_per_launch": B,
            "avg_launch_us": avg_s * 1e6, "share_of_instrumented_solve": ms / sum(v[0] for v in kt.values())}
    return {k: round(v, 1) for k, v in gbs.items()}, roof


def instrumented(s, p, q, its, traffic=False):
    """per-kernel-class HIP-event timings of one set-up + solve on the solver's stream (the
    library holds the stream before each iteration so that the events time the kernels,
    not the host's enqueue gaps), and the roofline figures of every class and of the
    dominant one"""
    s.set_timing(True)
    s.refactor()
    s.solve(q, tol=p.tol, max_iter=3000)
    sync()
    kt = s.kernel_times()
    s.set_timing(False)
    sinfo = s.info()
    gbs, roof = roofline_of(kt, lambda k: bytes_model(k, p, sinfo, its, p.restart),
                            (lambda k: measured_traffic(k)) if traffic else (lambda k: None))
    return ({k: round(v[0], 4) for k, v in kt.items()}, {k: v[1] for k, v in kt.items()}, gbs, roof, sinfo)


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


# ------------------------------------------------------------------ oracle baselines
def oracle_full_solve(p, rhs=None, budget=None):
    """the oracle's set-up and complete FGMRES solve, on one host thread (scipy's sparse
    kernels and SuperLU are single-threaded; BLAS is held to one thread): (set-up s,
    solve s, result)"""
    from threadpoolctl import threadpool_limits
    from oracle import fgmres, multigrid
    with threadpool_limits(1):
        t0 = time.perf_counter()
        H = multigrid.from_problem(p)
        t1 = time.perf_counter()
        r = fgmres.solve(H, p.rhs() if rhs is None else rhs, tol=p.tol, restart=p.restart,
                         max_iter=budget or 3000)
        t2 = time.perf_counter()
    return t1 - t0, t2 - t1, r


def host_fields():
    model, avail = cpu_info()
    return {"cores": 1, "cpu_model": model, "host_cores_available": avail}


# ------------------------------------------------------------------ workloads
def run_single(args, p, label, with_fp64, traffic=False):
    """mixed steps (set-up + solve), solve-only rate, instrumented roofline; FP64 steps"""
    import torch
    q = torch.from_numpy(p.rhs()).cuda()
    s = make_solver(p, "f32")
    dt, its, info, x32 = timed_steps(s, p, q, args.steps, args.warmup)
    dt_solve, _, _, _ = timed_steps(s, p, q, args.steps, 0, refactor=False)
    kms, kl, gbs, roof, sinfo = instrumented(s, p, q, its[-1], traffic)
    out = {
        "metric": METRIC, "value": 1.0 / dt, "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * dt, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "c64 cycle / c128 FGMRES", "data": "synthetic",
        "config": {"workload": label, "unknowns": p.N, "iterations": its[-1],
                   "true_rel_residual": info["true_rel_residual"],
                   "nd_schedule": {"leaf": sinfo["nd_leaf"], "root": sinfo["nd_root"], "cuts": sinfo["nd_cuts"],
                                   "tuned": bool(sinfo["nd_tuned"])}},
        "solve_only_per_sec": 1.0 / dt_solve, "setup_ms": 1e3 * (dt - dt_solve),
        "kernel_ms": kms, "kernel_launches": kl, "kernel_achieved_GBs": gbs, "roofline": roof,
    }
    xs = {"f32": x32.cpu().numpy()}
    s.close()
    del s
    free_gpu()
    if with_fp64:
        s64 = make_solver(p, "f64")
        dt64, its64, info64, x64 = timed_steps(s64, p, q, args.steps, args.warmup)
        dts64, _, _, _ = timed_steps(s64, p, q, args.steps, 0, refactor=False)
        out["fp64"] = {"value": 1.0 / dt64, "iterations": its64[-1], "solve_only_per_sec": 1.0 / dts64,
                       "true_rel_residual": info64["true_rel_residual"]}
        out["speedup_mixed_vs_fp64"] = dt64 / dt
        out["speedup_mixed_vs_fp64_solve_only"] = dts64 / dt_solve
        xs["f64"] = x64.cpu().numpy()
        s64.close()
        del s64
        free_gpu()
    return out, xs


def label_cfg2(p):
    return ("2D %dx%d layered medium, G=10 at max slowness, 20-cell absorbing layer, centre point source, "
            "FGMRES(20) tol 1e-6, W(1,1) cycle, alpha=%.4f, alpha2=%.3f, beta=%.2f"
            % (p.n[0], p.n[1], p.alpha, p.alpha2, p.beta))


def workload_cfg2(args, p=None):
    import synth
    p = p or synth.config2(args.n)
    out, xs = run_single(args, p, label_cfg2(p), not args.no_fp64, traffic=(p.n[0] == 1024))
    if not args.no_cpu_baseline:
        print("[bench] %s GPU part done, oracle solve" % p.name, file=sys.stderr, flush=True)
        setup, solve, r = oracle_full_solve(p)
        out["cpu_baseline"] = dict(
            value=1.0 / (setup + solve), unit="solves/s", kind="oracle",
            sample="the oracle's complete solve of the same system (set-up %.2f s: Galerkin products and a "
                   "sparse LU of the coarsest operator; FGMRES %.1f s for %d iterations)"
                   % (setup, solve, r.iterations),
            iterations=r.iterations, setup_s=setup, solve_s=solve, **host_fields())
        out["oracle_parity"] = {
            "iterations_oracle": r.iterations, "iterations_gpu_mixed": out["config"]["iterations"],
            "rel_diff_to_oracle_solution_mixed": rel(xs["f32"], r.x),
            "oracle_true_rel_residual": r.true_rel_residual}
        if "f64" in xs:
            out["oracle_parity"]["iterations_gpu_fp64"] = out["fp64"]["iterations"]
            out["oracle_parity"]["rel_diff_to_oracle_solution_fp64"] = rel(xs["f64"], r.x)
    return out


def workload_cfg1(args):
    import synth
    p = synth.config1(128)
    label = ("2D 128x128 homogeneous, kappa = 1, G=12, 16-cell absorbing layer, centre point source, "
             "FGMRES(20) tol 1e-6, W(2,2) cycle, alpha=%.4f, beta=0" % p.alpha)
    out, xs = run_single(args, p, label, not args.no_fp64)
    if not args.no_cpu_baseline:
        setup, solve, r = oracle_full_solve(p)
        out["cpu_baseline"] = dict(value=1.0 / (setup + solve), unit="solves/s", kind="oracle",
                                   sample="the oracle's complete solve of the same system (%d iterations)"
                                          % r.iterations, **host_fields())
        out["oracle_parity"] = {"iterations_oracle": r.iterations,
                                "rel_diff_to_oracle_solution_mixed": rel(xs["f32"], r.x)}
    return out


def workload_cfg3(args):
    import synth
    from oracle import operators as ops
    p = synth.config3(256)
    label = ("3D 256^3 layered medium (6 layers, noise smoothed over 8 cells), G=12 at max slowness, 12-cell "
             "absorbing layer on five faces, source 10 cells below the top face, FGMRES(20) tol 1e-6, W(1,1) with "
             "damping 0.6/0.4, alpha=%.4f, beta=%.2f" % (p.alpha, p.beta))
    out, xs = run_single(args, p, label, not args.no_fp64)
    print("[bench] cfg3 GPU part done", file=sys.stderr, flush=True)
    # the true residual of the GPU solutions with the oracle's own assembled operator (a
    # property that holds at any size; the whole oracle solve does not fit a bench run)
    sig = ops.layer_sigma(p.n, p.layer, p.sigma_max)
    H = ops.helmholtz(p.n, p.h, p.slowness.ravel() ** 2, p.omega, sig)
    q = p.rhs()
    out["oracle_parity"] = {"true_rel_residual_oracle_operator_mixed": rel(H @ xs["f32"], q)}
    if "f64" in xs:
        out["oracle_parity"]["true_rel_residual_oracle_operator_fp64"] = rel(H @ xs["f64"], q)
        out["oracle_parity"]["rel_diff_mixed_to_fp64"] = rel(xs["f32"], xs["f64"])
    del H
    if not args.no_cpu_baseline:
        ps = synth.config3(96)
        setup, solve, r = oracle_full_solve(ps)
        scale = p.N / ps.N
        per_it = solve / max(1, r.iterations)
        est = (setup + per_it * out["config"]["iterations"]) * scale
        out["cpu_baseline"] = dict(
            value=1.0 / est, unit="solves/s", kind="oracle",
            sample="the oracle's complete solve of the same recipe at 96^3 (%d unknowns: set-up %.2f s, %d "
                   "iterations at %.3f s each), extrapolated to the GPU's %d iterations and scaled by the unknown "
                   "count to 256^3 (x%.1f)" % (ps.N, setup, r.iterations, per_it, out["config"]["iterations"], scale),
            **host_fields())
    return out


def workload_cfg4(args):
    import torch
    import synth
    from paper_2604_19501_amd.batched import BatchedSolver, instance_dict
    per = args.batch_per_size
    probs = [synth.config4_instance(i, per_size=per) for i in range(3 * per)]
    rhs, inst = [], []
    for i, p in enumerate(probs):
        for k in range(len(p.sources)):
            rhs.append(torch.from_numpy(p.rhs(k)).cuda())
            inst.append(i)
    res = {}
    for prec in ("f32", "f64"):
        if prec == "f64" and args.no_fp64:
            continue
        t0 = time.perf_counter()
        b = BatchedSolver([instance_dict(p) for p in probs], nu=(1, 1), cycle_prec=prec, max_rhs=8)
        sync()
        t_setup = time.perf_counter() - t0
        for _ in range(args.warmup):
            xs, infos = b.solve(rhs, inst, tol=1e-6, max_iter=3000)
        sync()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            xs, infos = b.solve(rhs, inst, tol=1e-6, max_iter=3000)
        sync()
        dt = (time.perf_counter() - t0) / args.steps
        print("[bench] batch %s: %.1f solves/s" % (prec, len(rhs) / dt), file=sys.stderr, flush=True)
        res[prec] = dict(dt=dt, infos=infos, setup=t_setup, xs=[xs[size_idx * per * 8].cpu().numpy()
                                                                 for size_idx in range(3)])
        if prec == "f32":
            # per-class HIP-event timings of one lock-step group at full width: the first
            # 768^2 instance with its first source in all 8 slots
            ii = 2 * per
            pi = probs[ii]
            q0 = torch.from_numpy(pi.rhs(0)).cuda()
            b.set_timing(True)
            _, inf8 = b.solve([q0] * 8, [ii] * 8, tol=1e-6, max_iter=3000)
            sync()
            kt = b.kernel_times()
            b.set_timing(False)
            info_i = b.instance_info(ii)
            it8 = inf8[0]["iterations"]
            gbs, roof = roofline_of(kt, lambda k: bytes_model(k, pi, info_i, it8, pi.restart, nr=8))
            roof["measured_on"] = ("one 768^2 instance, 8 lock-step right-hand sides (%d iterations), per-launch "
                                   "HIP events on its stream" % it8)
            res[prec]["timing"] = (kt, gbs, roof)
        b.close()
        del b, xs
        free_gpu()
    m = res["f32"]
    infos = m["infos"]
    its = [i["iterations"] for i in infos]
    kt, gbs, roof = m["timing"]
    out = {
        "metric": "batched Helmholtz solves/sec at 1e-6 rel. residual (solve-only, batch set-up reported apart, "
                  "FP32 cycle / FP64 FGMRES)",
        "value": len(rhs) / m["dt"], "unit": "solves/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * m["dt"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "c64 cycle / c128 FGMRES", "data": "synthetic",
        "config": {"workload": "%d instances (%d each of 256^2, 512^2, 768^2), G cycling 10, 10.67, 11.33, 12, "
                               "8 seeded point sources each, layered media seeded 4000+i, W(1,1), FGMRES(20) tol 1e-6"
                               % (3 * per, per), "solves_per_step": len(rhs), "fine_unknowns": sum(p.N for p in probs),
                   "iterations_mean": float(np.mean(its)), "iterations_max": int(max(its)),
                   "worst_true_rel_residual": max(i["true_rel_residual"] for i in infos),
                   "status_nonzero": sum(1 for i in infos if i["status"] != 0)},
        "batch_setup_s": m["setup"],
        "kernel_ms": {k: round(v[0], 4) for k, v in kt.items()},
        "kernel_launches": {k: v[1] for k, v in kt.items()},
        "kernel_achieved_GBs": gbs, "roofline": roof,
    }
    if "f64" in res:
        d = res["f64"]
        out["fp64"] = {"value": len(rhs) / d["dt"], "iterations_mean": float(np.mean([i["iterations"]
                                                                                     for i in d["infos"]])),
                       "batch_setup_s": d["setup"]}
        out["speedup_mixed_vs_fp64"] = d["dt"] / m["dt"]
    if not args.no_cpu_baseline:
        tot, sample, par = 0.0, [], []
        for size_idx in range(3):
            i = size_idx * per
            p = probs[i]
            setup, solve, r = oracle_full_solve(p, rhs=p.rhs(0))
            print("[bench] oracle %s: %d iterations, %.1f s" % (p.name, r.iterations, setup + solve),
                  file=sys.stderr, flush=True)
            j = inst.index(i)
            par.append({"instance": p.name, "iterations_oracle": r.iterations, "iterations_gpu": its[j],
                        "rel_diff_to_oracle_solution_mixed": rel(m["xs"][size_idx], r.x)})
            if "f64" in res:
                par[-1]["rel_diff_to_oracle_solution_fp64"] = rel(res["f64"]["xs"][size_idx], r.x)
            ti = [its[k] for k in range(len(rhs)) if inst[k] == i]
            per_it = solve / max(1, r.iterations)
            # every instance of this size: set-up once, its solves at the GPU's iteration counts
            tot += per * (setup + per_it * float(np.mean(ti)) * len(p.sources))
            sample.append("%d^2: set-up %.2f s, %d iterations at %.3f s" % (p.n[0], setup, r.iterations, per_it))
        out["cpu_baseline"] = dict(
            value=len(rhs) / tot, unit="solves/s", kind="oracle",
            sample="the oracle's complete solve of the first source of the first instance of each size ("
                   + "; ".join(sample) + "), extrapolated to the batch at the GPU's mean iteration counts, "
                   "set-ups included", **host_fields())
        out["oracle_parity"] = par
    return out


def workload_cfg5(args):
    import torch
    import synth
    from paper_2604_19501_amd import from_problem
    from paper_2604_19501_amd.autograd import helmholtz_misfit
    p, m_ref, rec = synth.config5(128)
    s = from_problem(p, cycle_prec="f32", max_rhs=16)          # the 16 sources in lock-step
    src = [torch.from_numpy(synth.point_rhs(p.n, pos)).cuda() for pos in p.sources]
    recs = torch.from_numpy(rec).cuda()
    s.refactor(m=torch.from_numpy(m_ref.ravel()).cuda())
    us, _ = s.solve_many(src, tol=1e-10, max_iter=3000)
    data = [u[recs].clone() for u in us]
    m0 = torch.from_numpy(p.slowness.ravel() ** 2).cuda()

    def step():
        m = m0.clone().requires_grad_(True)
        loss = helmholtz_misfit(m, s, src, recs, data, tol=1e-10, max_iter=3000)
        loss.backward()
        return loss, m.grad

    for _ in range(args.warmup):
        step()
    sync()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        loss, g = step()
    sync()
    dt = (time.perf_counter() - t0) / args.steps
    s.set_timing(True)
    u, info = s.solve(src[0], tol=1e-10, max_iter=3000)
    sync()
    kt = s.kernel_times()
    s.set_timing(False)
    sinfo = s.info()
    gbs, roof = roofline_of(kt, lambda k: bytes_model(k, p, sinfo, info["iterations"], p.restart))
    roof["measured_on"] = "the first forward solve at the evaluation point (%d iterations)" % info["iterations"]
    out = {
        "metric": "misfit gradient evaluations/sec (set-up + 16 forward + 16 adjoint solves at tol 1e-10, each "
                  "set in lock-step, + gradient, FP32 cycle / FP64 FGMRES)",
        "value": 1.0 / dt, "unit": "gradients/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * dt, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "c64 cycle / c128 FGMRES", "data": "synthetic",
        "config": {"workload": "3D 128^3 least-squares misfit, 16 point sources on a 4x4 lattice of the top plane, "
                               "receivers on all 16641 top-plane nodes, data from a seeded layered reference medium, "
                               "evaluated at its smoothing (16 cells), G=12, W(1,1) with damping 0.6/0.4, beta=%.2f"
                               % p.beta, "unknowns": p.N,
                   "loss": float(loss), "grad_norm": float(torch.linalg.norm(g)),
                   "iterations_first_forward": info["iterations"]},
        "kernel_ms": {k: round(v[0], 4) for k, v in kt.items()},
        "kernel_launches": {k: v[1] for k, v in kt.items()},
        "kernel_achieved_GBs": gbs,
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        setup, solve, r = oracle_full_solve(p, rhs=synth.point_rhs(p.n, p.sources[0]), budget=10)
        per_it = solve / max(1, r.iterations)
        est = setup + per_it * info["iterations"] * 2 * len(src)
        out["cpu_baseline"] = dict(value=1.0 / est, unit="gradients/s", kind="oracle",
                                   sample="oracle set-up (%.2f s) + 10 FGMRES iterations (%.3f s/iteration) of one "
                                          "forward solve, extrapolated to 32 solves of %d iterations each"
                                          % (setup, per_it, info["iterations"]), **host_fields())
    s.close()
    return out


def workload_paper(args):
    """the paper's own stack (compact fourth-order 9-point operator, cubic transfers, alpha*
    of Table 1) on Fig. 4b's homogeneous G = 12 problem at 1024^2, with the oracle's complete
    solve of the same system"""
    import synth
    p = synth.paper_stack((1024, 1024), "cubic")
    label = ("2D 1024x1024 homogeneous, G=12, 20-cell absorbing layer, centre point source, the paper's compact "
             "fourth-order 9-point operator with cubic transfers (25- and 49-point Galerkin levels), alpha=%.4f "
             "(Table 1), FGMRES(20) tol 1e-6, W(1,1) cycle, Jacobi 0.89" % p.alpha)
    out, xs = run_single(args, p, label, not args.no_fp64)
    if not args.no_cpu_baseline:
        print("[bench] %s GPU part done, oracle solve" % p.name, file=sys.stderr, flush=True)
        setup, solve, r = oracle_full_solve(p)
        out["cpu_baseline"] = dict(
            value=1.0 / (setup + solve), unit="solves/s", kind="oracle",
            sample="the oracle's complete solve of the same system (set-up %.1f s: Galerkin products and a "
                   "sparse LU of the 49-point coarsest operator; FGMRES %.1f s for %d iterations)"
                   % (setup, solve, r.iterations),
            iterations=r.iterations, setup_s=setup, solve_s=solve, **host_fields())
        out["oracle_parity"] = {
            "iterations_oracle": r.iterations, "iterations_gpu_mixed": out["config"]["iterations"],
            "rel_diff_to_oracle_solution_mixed": rel(xs["f32"], r.x),
            "paper_iterations_fig_4b": "6-8"}
        if "f64" in xs:
            out["oracle_parity"]["iterations_gpu_fp64"] = out["fp64"]["iterations"]
            out["oracle_parity"]["rel_diff_to_oracle_solution_fp64"] = rel(xs["f64"], r.x)
    return out


def workload_paper3d(args):
    """the paper's 3D stack on a stand-in of its largest 3D grid (Table 5: 192x192x72 cells,
    G = 12): GPU timing, the true residual of the GPU solution under the oracle's operator,
    and the oracle's complete solve of the same recipe at 96x96x40 scaled to this grid"""
    import synth
    from oracle import operators as ops
    p = synth.paper_3d((192, 192, 72), 12.0)
    label = ("3D 192x192x72 layered stand-in (8 sharp layers, noise smoothed over 4 cells), G=12, 12-cell "
             "absorbing layer on five faces, source at the centre of the top face, the paper's compact 19-point "
             "operator with level-dependent transfers (125-point Galerkin levels), alpha=%.4f (Table 2), "
             "FGMRES(20) tol 1e-6, W(1,1) cycle, Jacobi 0.6/0.4" % p.alpha)
    out, xs = run_single(args, p, label, not args.no_fp64)
    sigma = ops.layer_sigma(p.n, p.layer, p.sigma_max)
    Hc = ops.helmholtz_compact(p.n, p.h, p.slowness.ravel() ** 2, p.omega, sigma)
    b = p.rhs()
    out["oracle_parity"] = {"true_rel_residual_oracle_operator_mixed":
                            float(np.linalg.norm(b - Hc @ xs["f32"]) / np.linalg.norm(b)),
                            "paper_iterations_table_5": 10}
    if "f64" in xs:
        out["oracle_parity"]["true_rel_residual_oracle_operator_fp64"] = float(
            np.linalg.norm(b - Hc @ xs["f64"]) / np.linalg.norm(b))
    if not args.no_cpu_baseline:
        print("[bench] %s GPU part done, oracle sample" % p.name, file=sys.stderr, flush=True)
        ps = synth.paper_3d((96, 96, 40), 12.0)
        setup, solve, r = oracle_full_solve(ps)
        scale = p.N / ps.N
        its = out["config"]["iterations"]
        est = scale * (setup + solve * its / max(1, r.iterations))
        out["cpu_baseline"] = dict(
            value=1.0 / est, unit="solves/s", kind="oracle",
            sample="the oracle's complete solve of the same recipe at 96x96x40 (%d unknowns: set-up %.1f s, "
                   "%d iterations in %.1f s), scaled to the GPU's %d iterations and by the unknown count to "
                   "192x192x72 (x%.1f)" % (ps.N, setup, r.iterations, solve, its, scale), **host_fields())
    return out


def workload_suite(args):
    """the headline (1024^2 layered, mixed vs FP64, oracle full solve) with the 256^3, the
    batched and the paper-stack workloads as sub-records"""
    out = workload_cfg2(args)
    print("[bench] cfg2 done: %.3f solves/s" % out["value"], file=sys.stderr, flush=True)
    sub = {}
    # the sub-records time at most 3 steps after 1 warm-up (each step of the batch is 768
    # solves), so that the whole run stays within a few minutes
    sargs = argparse.Namespace(**vars(args))
    sargs.steps, sargs.warmup = min(args.steps, 3), min(args.warmup, 1)
    for name, fn in (("cfg3", workload_cfg3), ("cfg4", workload_cfg4), ("paper", workload_paper),
                     ("paper3d", workload_paper3d)):
        free_gpu()
        t0 = time.perf_counter()
        sub[name] = fn(sargs)
        sub[name]["wall_s"] = time.perf_counter() - t0
        print("[bench] %s done in %.1f s: %.3f %s" % (name, sub[name]["wall_s"], sub[name]["value"],
                                                     sub[name]["unit"]), file=sys.stderr, flush=True)
    out["workloads"] = sub
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=("suite", "cfg1", "cfg2", "cfg3", "cfg4", "cfg5", "paper", "paper3d"),
                    default="suite")
    ap.add_argument("--n", type=int, default=1024, help="cells per axis of the cfg2 workload")
    ap.add_argument("--batch-per-size", type=int, default=32, help="cfg4: instances per grid size")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--pmc-pass", action="store_true",
                    help="for hardware-counter runs: a 256 MiB device copy (calibrates FETCH_SIZE/WRITE_SIZE "
                         "against known bytes) followed by one setup+solve step of the cfg2 workload (cfg3 with "
                         "--workload cfg3)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the solver has no multi-GPU path (requested --gpus %d)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.pmc_pass:
        import synth
        p = synth.config3(256) if args.workload == "cfg3" else synth.config2(args.n)
        q = torch.from_numpy(p.rhs()).cuda()
        a = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda")      # 256 MiB
        b = torch.empty_like(a)
        b.copy_(a)
        sync()
        s32 = make_solver(p, "f32")
        s32.refactor()
        x, info = s32.solve(q, tol=p.tol, max_iter=3000)
        sync()
        print(json.dumps({"pmc_pass": True, "iterations": info["iterations"], "copy_bytes": 2 * a.numel() * 8}))
        return
    out = {"suite": workload_suite, "cfg1": workload_cfg1, "cfg2": workload_cfg2, "cfg3": workload_cfg3,
           "cfg4": workload_cfg4, "cfg5": workload_cfg5, "paper": workload_paper,
           "paper3d": workload_paper3d}[args.workload](args)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
