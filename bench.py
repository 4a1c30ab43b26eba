#!/usr/bin/env python
"""Throughput of the real-shifted multigrid Helmholtz solver on one MI355X.

Default workload (--workload cfg2): 2D 1024 x 1024 cells, layered medium (8 layers,
velocity 1.5-4.5, +-10 % noise smoothed over 20 cells), 10 points per wavelength at the
largest slowness, 20-cell absorbing layer, point source at the centre; FGMRES(20) to a
relative residual of 1e-6, preconditioned by the 3-level W(1,1) cycle (damped Jacobi 0.8)
with the real-shifted coarsest Galerkin operator (alpha* of the grid-to-grid dispersion
analysis), a level-2 real shift and a complex shift of the preconditioner.  One step =
numerical set-up (coefficients, Galerkin operators, coarsest factorisation) + solve on
resident inputs, FP32-complex cycle inside FP64 FGMRES; value = steps per second.

Other workloads (same one-line JSON contract):
  cfg1  2D 128^2 homogeneous, G = 12, W(2,2), set-up + solve
  cfg3  3D 256^3 layered, G = 12, 7-point stencil, 27-point Galerkin, W(1,1) damping
        0.6/0.4, set-up + solve
  cfg4  96 instances (32 each of 256^2, 512^2, 768^2), 4 frequencies, 8 sources each:
        the 768 solves of one batch per step (the batch's set-up is reported apart)
  cfg5  3D 128^3 least-squares misfit: 16 sources, receivers on the top plane; one step =
        set-up at m + 16 forward + 16 adjoint solves (tol 1e-10) + the gradient

The line also carries the FP64-cycle rate (cfg1, cfg2), per-kernel-class HIP-event
timings, the roofline of the dominant kernel class and the FP64 CPU oracle timed on a
bounded sample of the same workload.

    python bench.py [--workload cfg2] [--steps K] [--warmup W] [--gpus 1]
"""
from __future__ import annotations

import argparse
import hashlib
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


def make_solver(p, prec):
    from paper_2604_19501_amd import from_problem
    return from_problem(p, nu=(p.nu_pre, p.nu_post), cycle_prec=prec)


def sync():
    import torch
    torch.cuda.synchronize()


def timed_steps(s, p, q, steps, warmup, refactor=True):
    its = []
    info = None
    for _ in range(warmup):
        if refactor:
            s.refactor()
        x, info = s.solve(q, tol=p.tol, max_iter=2000)
    sync()
    t0 = time.perf_counter()
    for _ in range(steps):
        if refactor:
            s.refactor()
        x, info = s.solve(q, tol=p.tol, max_iter=2000)
        its.append(info["iterations"])
    sync()
    return (time.perf_counter() - t0) / steps, its, info


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
    if cls == "l1_restrict":      # b (c128) per fine node and r2 per level-2 node per rhs; m (f32)
        return N1 * (16 * nr + 4) + N2 * cb * nr
    if cls == "l1_sweep":         # b (c128) + z out per fine node and e2 per level-2 node per rhs; m
        return N1 * ((16 + cb) * nr + 4) + N2 * cb * nr
    # level-2 coefficients: the 3D FP32 cycle stores the complex-symmetric operator's centre
    # and the directions after it (14 planes), otherwise all K
    S = K // 2 + 1 if (cb == 8 and d == 3) else K
    if cls == "l2_sweep":         # coefficients + b2, x in, x out per level-2 node
        return N2 * cb * (S + 3 * nr)
    if cls == "l2_restrict":      # coefficients + b2, x per level-2 node
        return N2 * cb * (S + 2 * nr)
    if cls == "nd_fwd":           # [A^-1; C A^-1] once, right-hand side gather, updates written and read
        per_solve = info["L_entries"] * cb + 4 * (N3 + U) + nr * (2 * N3 * cb + 2 * U * cb)
        return per_solve / info["fwd_launches"]
    if cls == "nd_bwd":           # -A^-1 B once, boundary gather, g read and x written
        per_solve = info["W_entries"] * cb + 4 * U + nr * (U * cb + 2 * N3 * cb)
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


def instrumented(s, p, q, its):
    """per-kernel-class HIP-event timings of one set-up + solve on the solver's stream, and
    the roofline figures of every class and of the dominant one"""
    s.set_timing(True)
    s.refactor()
    s.solve(q, tol=p.tol, max_iter=2000)
    sync()
    kt = s.kernel_times()
    s.set_timing(False)
    sinfo = s.info()
    gbs, roof = roofline_of(kt, lambda k: bytes_model(k, p, sinfo, its, p.restart),
                            lambda k: measured_traffic(k) if (p.dim == 2 and p.n[0] == 1024) else None)
    return ({k: round(v[0], 4) for k, v in kt.items()}, {k: v[1] for k, v in kt.items()}, gbs, roof, sinfo)


# ------------------------------------------------------------------ oracle baselines
def oracle_solve_sample(p, budget_iters=20, rhs=None, tol=None):
    """oracle set-up + the first FGMRES iterations of the same solve: (set-up s, s/iteration, iterations)"""
    from oracle import fgmres, multigrid
    t0 = time.perf_counter()
    H = multigrid.from_problem(p)
    t1 = time.perf_counter()
    r = fgmres.solve(H, p.rhs() if rhs is None else rhs, tol=p.tol if tol is None else tol, restart=p.restart,
                     max_iter=budget_iters)
    t2 = time.perf_counter()
    return t1 - t0, (t2 - t1) / max(1, r.iterations), r.iterations


def cpu_baseline_single(p, its_gpu, label):
    setup, per_it, n_it = oracle_solve_sample(p)
    est = setup + per_it * its_gpu
    return {"value": 1.0 / est, "unit": "solves/s", "cores": 1, "kind": "oracle",
            "sample": "oracle set-up (%.2f s) + first %d FGMRES iterations (%.3f s/iteration) of the same %s "
                      "solve, extrapolated to %d iterations; scipy sparse kernels and SuperLU run single-threaded"
                      % (setup, n_it, per_it, label.split(",")[0], its_gpu),
            "setup_s": setup, "s_per_iteration": per_it}


# ------------------------------------------------------------------ workloads
def run_single(args, p, label, metric, with_fp64, cpu_sample=None):
    import torch
    q = torch.from_numpy(p.rhs()).cuda()
    s = make_solver(p, "f32")
    dt, its, info = timed_steps(s, p, q, args.steps, args.warmup)
    dt_solve, _, _ = timed_steps(s, p, q, args.steps, 0, refactor=False)
    kms, kl, gbs, roof, sinfo = instrumented(s, p, q, its[-1])
    out = {
        "metric": metric, "value": 1.0 / dt, "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * dt, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "c64 cycle / c128 FGMRES", "data": "synthetic",
        "config": {"workload": label, "unknowns": p.N, "iterations": its[-1],
                   "true_rel_residual": info["true_rel_residual"],
                   "nd_schedule": {"leaf": sinfo["nd_leaf"], "root": sinfo["nd_root"], "cuts": sinfo["nd_cuts"],
                                   "tuned": bool(sinfo["nd_tuned"])}},
        "solve_only_per_sec": 1.0 / dt_solve, "setup_ms": 1e3 * (dt - dt_solve),
        "kernel_ms": kms, "kernel_launches": kl, "kernel_achieved_GBs": gbs, "roofline": roof,
    }
    s.close()
    del s
    torch.cuda.empty_cache()
    if with_fp64:
        s64 = make_solver(p, "f64")
        dt64, its64, info64 = timed_steps(s64, p, q, args.steps, args.warmup)
        dts64, _, _ = timed_steps(s64, p, q, args.steps, 0, refactor=False)
        out["fp64"] = {"value": 1.0 / dt64, "iterations": its64[-1], "solve_only_per_sec": 1.0 / dts64,
                       "true_rel_residual": info64["true_rel_residual"]}
        out["speedup_mixed_vs_fp64"] = dt64 / dt
        out["speedup_mixed_vs_fp64_solve_only"] = dts64 / dt_solve
        s64.close()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_sample(its[-1]) if cpu_sample else cpu_baseline_single(p, its[-1], label)
    return out


def workload_cfg1(args):
    import synth
    p = synth.config1(128)
    label = ("2D 128x128 homogeneous, kappa = 1, G=12, 16-cell absorbing layer, centre point source, "
             "FGMRES(20) tol 1e-6, W(2,2) cycle, alpha=%.4f, beta=0" % p.alpha)
    return run_single(args, p, label, "Helmholtz solves/sec at 1e-6 rel. residual (setup+solve per step, "
                      "FP32 cycle / FP64 FGMRES)", not args.no_fp64)


def workload_cfg2(args):
    import synth
    p = synth.config2(args.n)
    label = ("2D %dx%d layered medium, G=10 at max slowness, 20-cell absorbing layer, centre point source, "
             "FGMRES(20) tol 1e-6, W(1,1) cycle, alpha=%.4f, alpha2=%.3f, beta=%.2f"
             % (args.n, args.n, p.alpha, p.alpha2, p.beta))
    return run_single(args, p, label, "Helmholtz solves/sec at 1e-6 rel. residual (setup+solve per step, "
                      "FP32 cycle / FP64 FGMRES)", not args.no_fp64)


def workload_cfg3(args):
    import synth
    p = synth.config3(256)
    label = ("3D 256^3 layered medium (6 layers, noise smoothed over 8 cells), G=12 at max slowness, 12-cell "
             "absorbing layer on five faces, source 10 cells below the top face, FGMRES(20) tol 1e-6, W(1,1) with "
             "damping 0.6/0.4, alpha=%.4f, beta=%.2f" % (p.alpha, p.beta))

    def cpu_sample(its_gpu):
        ps = synth.config3(96)
        setup, per_it, n_it = oracle_solve_sample(ps)
        scale = p.N / ps.N
        est = (setup + per_it * its_gpu) * scale
        return {"value": 1.0 / est, "unit": "solves/s", "cores": 1, "kind": "oracle",
                "sample": "oracle on the same recipe at 96^3 (%d unknowns): set-up %.2f s + first %d FGMRES "
                          "iterations (%.3f s/iteration), extrapolated to %d iterations and scaled by the unknown "
                          "count to 256^3 (x%.1f)" % (ps.N, setup, n_it, per_it, its_gpu, scale)}
    return run_single(args, p, label, "Helmholtz solves/sec at 1e-6 rel. residual (setup+solve per step, "
                      "FP32 cycle / FP64 FGMRES)", False, cpu_sample)


def workload_cfg4(args):
    import torch
    import synth
    from paper_2604_19501_amd.batched import BatchedSolver, instance_dict
    per = args.batch_per_size
    probs = [synth.config4_instance(i, per_size=per) for i in range(3 * per)]
    t0 = time.perf_counter()
    b = BatchedSolver([instance_dict(p) for p in probs], nu=(1, 1), cycle_prec="f32", max_rhs=8)
    sync()
    t_setup = time.perf_counter() - t0
    rhs, inst = [], []
    for i, p in enumerate(probs):
        for k in range(len(p.sources)):
            rhs.append(torch.from_numpy(p.rhs(k)).cuda())
            inst.append(i)
    sync()
    for _ in range(args.warmup):
        xs, infos = b.solve(rhs, inst, tol=1e-6, max_iter=2000)
    sync()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        xs, infos = b.solve(rhs, inst, tol=1e-6, max_iter=2000)
    sync()
    dt = (time.perf_counter() - t0) / args.steps
    its = [i["iterations"] for i in infos]
    worst = max(i["true_rel_residual"] for i in infos)
    nodes = sum(p.N for p in probs)
    out = {
        "metric": "batched Helmholtz solves/sec at 1e-6 rel. residual (solve-only, batch set-up reported apart, "
                  "FP32 cycle / FP64 FGMRES)",
        "value": len(rhs) / dt, "unit": "solves/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * dt, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "c64 cycle / c128 FGMRES", "data": "synthetic",
        "config": {"workload": "%d instances (%d each of 256^2, 512^2, 768^2), G cycling 10, 10.67, 11.33, 12, "
                               "8 seeded point sources each, layered media seeded 4000+i, W(1,1), FGMRES(20) tol 1e-6"
                               % (3 * per, per), "solves_per_step": len(rhs), "fine_unknowns": nodes,
                   "iterations_mean": float(np.mean(its)), "iterations_max": int(max(its)),
                   "worst_true_rel_residual": worst, "status_nonzero": sum(1 for i in infos if i["status"] != 0)},
        "batch_setup_s": t_setup,
    }
    # per-class HIP-event timings (graphs bypassed) of one lock-step group at full width: the
    # first 768^2 instance with its first source in all 8 slots, so every launch carries 8
    # active right-hand sides
    ii = 2 * per
    pi = probs[ii]
    q0 = torch.from_numpy(pi.rhs(0)).cuda()
    b.set_timing(True)
    _, inf8 = b.solve([q0] * 8, [ii] * 8, tol=1e-6, max_iter=2000)
    sync()
    kt = b.kernel_times()
    b.set_timing(False)
    info_i = b.instance_info(ii)
    it8 = inf8[0]["iterations"]
    gbs, roof = roofline_of(kt, lambda k: bytes_model(k, pi, info_i, it8, pi.restart, nr=8))
    roof["measured_on"] = ("one 768^2 instance, 8 lock-step right-hand sides (%d iterations), per-launch "
                           "HIP events on its stream" % it8)
    out["kernel_ms"] = {k: round(v[0], 4) for k, v in kt.items()}
    out["kernel_launches"] = {k: v[1] for k, v in kt.items()}
    out["kernel_achieved_GBs"] = gbs
    out["roofline"] = roof
    if not args.no_cpu_baseline:
        tot, sample = 0.0, []
        for size_idx in range(3):
            i = size_idx * per
            p = probs[i]
            ti = [its[j] for j in range(len(rhs)) if inst[j] == i]
            setup, per_it, _ = oracle_solve_sample(p, budget_iters=10, rhs=p.rhs(0))
            # every instance of this size: set-up once, its solves at the GPU's iteration counts
            tot += per * (setup + per_it * float(np.mean(ti)) * len(p.sources))
            sample.append("%d^2: set-up %.2f s, %.3f s/iteration" % (p.n[0], setup, per_it))
        out["cpu_baseline"] = {"value": len(rhs) / tot, "unit": "solves/s", "cores": 1, "kind": "oracle",
                               "sample": "oracle on the first instance of each size (set-up + 10 FGMRES "
                                         "iterations: " + "; ".join(sample) + "), extrapolated to the batch at "
                                         "the GPU's mean iteration counts, set-ups included"}
    b.close()
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
    # data from the reference medium, solved by the library (tol 1e-10)
    s.refactor(slowness=torch.from_numpy(np.sqrt(m_ref).ravel()).cuda())
    us, _ = s.solve_many(src, tol=1e-10, max_iter=2000)
    data = [u[recs].clone() for u in us]
    m0 = torch.from_numpy(p.slowness.ravel() ** 2).cuda()

    def step():
        m = m0.clone().requires_grad_(True)
        loss = helmholtz_misfit(m, s, src, recs, data, tol=1e-10, max_iter=2000)
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
    # per-class HIP-event timings of the first forward solve at the evaluation point
    s.set_timing(True)
    u, info = s.solve(src[0], tol=1e-10, max_iter=2000)
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
        setup, per_it, _ = oracle_solve_sample(p, budget_iters=10, rhs=synth.point_rhs(p.n, p.sources[0]), tol=1e-10)
        est = setup + per_it * info["iterations"] * 2 * len(src)
        out["cpu_baseline"] = {"value": 1.0 / est, "unit": "gradients/s", "cores": 1, "kind": "oracle",
                               "sample": "oracle set-up (%.2f s) + 10 FGMRES iterations (%.3f s/iteration) of one "
                                         "forward solve, extrapolated to 32 solves of %d iterations each"
                                         % (setup, per_it, info["iterations"])}
    s.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=("cfg1", "cfg2", "cfg3", "cfg4", "cfg5"), default="cfg2")
    ap.add_argument("--n", type=int, default=1024, help="cells per axis of the cfg2 workload")
    ap.add_argument("--batch-per-size", type=int, default=32, help="cfg4: instances per grid size")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--pmc-pass", action="store_true",
                    help="for hardware-counter runs: a 256 MiB device copy (calibrates FETCH_SIZE/WRITE_SIZE "
                         "against known bytes) followed by one setup+solve step of the cfg2 workload")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the solver has no multi-GPU path (requested --gpus %d)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.pmc_pass:
        import synth
        p = synth.config2(args.n)
        q = torch.from_numpy(p.rhs()).cuda()
        a = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda")      # 256 MiB
        b = torch.empty_like(a)
        b.copy_(a)
        sync()
        s32 = make_solver(p, "f32")
        s32.refactor()
        x, info = s32.solve(q, tol=p.tol, max_iter=2000)
        sync()
        print(json.dumps({"pmc_pass": True, "iterations": info["iterations"], "copy_bytes": 2 * a.numel() * 8}))
        return
    out = {"cfg1": workload_cfg1, "cfg2": workload_cfg2, "cfg3": workload_cfg3, "cfg4": workload_cfg4,
           "cfg5": workload_cfg5}[args.workload](args)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
