"""Autotuner of the coarsest-solve schedule.

The exact coarsest solve (nested dissection, see csrc/nd_plan.cpp) has five schedule
parameters that change its speed but not its result: the leaf box size, the size up to
which the top separators are merged into one root front, the dissection-tree heights whose
fronts are merged into their parents (HELM_ND_MERGE: fewer dependent levels, larger
fronts), the tree heights at which the tree-block launches end (HELM_ND_CUTS) and the
factor bytes per height from which a height takes split-K launches (HELM_ND_SPLITK_KB).  For a grid shape and cycle precision this
tool times FGMRES iterations of a seeded problem of that shape under every candidate
schedule and records the best-scoring one in a JSON cache, which libhelm reads when it plans a
context of that shape (file named by HELM_TUNE_CACHE; the package sets it to
tune_cache.json next to the library unless the caller set it).

    python -m paper_2604_19501_amd.tune --n 1024 1024 --prec f32 [--its 150] [--out FILE]
        [--stack compact --transfer cubic]

Each candidate is scored by its numerical set-up time (coefficients, Galerkin operators,
factorisation) plus --its times its per-iteration time: a larger root front shortens the
substitutions but lengthens the factorisation.  Both times are minima over repeats,
after a warm-up (which also captures the per-iteration graphs).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import time

import numpy as np
import torch

from . import _lib as L
from .solver import Solver


# merged-height sets: every second level (odd or even heights), two of every three, and
# every second level above the lower tree only; heights past the tree's are ignored
MERGES = {
    "none": "none",
    "odd": ",".join(str(h) for h in range(1, 40, 2)),
    "even": ",".join(str(h) for h in range(2, 40, 2)),
    "two_of_three": ",".join(str(h) for h in range(1, 40) if h % 3),
    "odd_from_5": ",".join(str(h) for h in range(5, 40, 2)),
}


SPLITK_DEFAULT_KB = 4096
SPLITK_OFF_KB = 1 << 30


def _candidates(dim: int):
    """(leaf, root, cuts, merge, splitk_kb) in two stages: the grid of leaf x root x cuts
    without merged heights, then every merged-height set with the cuts and both split-K
    thresholds under the best stage-one leaf sizes and root limits (_stage_two)."""
    if dim == 2:
        leaves, roots = (16, 32, 64), (100, 300, 600, 1100, 2200)
    else:
        leaves, roots = (8, 16), (1,)
    cuts = ["", "none"] + [str(h) for h in range(0, 7)] + ["2,4", "3,5", "2,5", "3,6", "1,3"]
    for leaf in leaves:
        for root in roots:
            for c in cuts:
                yield leaf, root, c, "none", SPLITK_DEFAULT_KB


def _stage_two(results, top=3):
    cuts = ["", "none"] + [str(h) for h in range(0, 5)] + ["1,3", "2,4", "1,2", "2,3"]
    seen = set()
    for r in sorted(results, key=lambda r: r["score_ms"]):
        lr = (r["leaf"], r["root"])
        if lr in seen:
            continue
        seen.add(lr)
        if len(seen) > top:
            break
        for name, m in MERGES.items():
            for sk in (SPLITK_DEFAULT_KB, SPLITK_OFF_KB):
                if name == "none" and sk == SPLITK_DEFAULT_KB:
                    continue           # stage one
                for c in cuts:
                    yield lr[0], lr[1], c, m, sk


def _problem(n, G=10.0, layer=8):
    """homogeneous medium, G points per wavelength, absorbing layer on every face; the
    schedule's cost does not depend on the medium's values."""
    dim = len(n)
    h = 1.0 / max(n)
    kappa = np.ones(tuple(k + 1 for k in reversed(n)))
    omega = 2.0 * math.pi / (G * h)
    return dim, h, kappa, omega, tuple((layer, layer) for _ in range(dim))


def coarsest_radius(stack="p5", transfer=None):
    """stencil radius of the coarsest operator: 1 for the 5/7-point stack; the compact
    stack's 49-point (cubic) or 25/125-point (level-dependent) operator: 3 or 2"""
    if stack != "compact":
        return 1
    return 3 if transfer == "cubic" else 2


def cache_key(n, prec, stack="p5", transfer=None):
    """the library's key: grid, the coarsest solve's precision (the cycle's for the 5/7-point
    stack; FP64 for the compact stack, whose coarsest factors are always FP64) and radius"""
    dim = len(n)
    r = coarsest_radius(stack, transfer)
    nd_prec = "f64" if stack == "compact" else prec
    return "nd:%d:%s:%s%s" % (dim, "x".join(str(k) for k in (tuple(n) + (0,) * (3 - dim))), nd_prec,
                              ":r%d" % r if r != 1 else "")


def time_schedule(n, prec, leaf, root, cuts, iters=30, repeats=2, merge="none", splitk_kb=SPLITK_DEFAULT_KB,
                  stack="p5", transfer=None, boxes="0,0,0,0"):
    """(seconds per FGMRES iteration, seconds per numerical set-up, plan info)"""
    env = {"HELM_ND_LEAF": str(leaf), "HELM_ND_ROOT": str(root), "HELM_ND_CUTS": cuts,
           "HELM_ND_MERGE": merge, "HELM_ND_SPLITK_KB": str(splitk_kb), "HELM_BOXES": boxes}
    saved = {k: os.environ.get(k) for k in env}
    os.environ.update(env)
    try:
        dim, h, kappa, omega, layer = _problem(n)
        s = Solver(n, h, kappa, omega, layer=layer, sigma_max=2.0, alpha=1.1, alpha2=1.0, beta=0.1,
                   nu=(1, 1), cycle_prec=prec, stack=stack, transfer=transfer)
        info = s.info()
        q = np.zeros(int(np.prod([k + 1 for k in n])), np.complex128)
        q[q.size // 2] = 1.0
        s.solve(q, tol=1e-300, max_iter=iters)
        best, setup = float("inf"), float("inf")
        for _ in range(repeats):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, it = s.solve(q, tol=1e-300, max_iter=iters)
            torch.cuda.synchronize()
            best = min(best, (time.perf_counter() - t0) / max(1, it["iterations"]))
            t0 = time.perf_counter()
            s.refactor()
            torch.cuda.synchronize()
            setup = min(setup, time.perf_counter() - t0)
        s.close()
        return best, setup, info
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
        torch.cuda.empty_cache()


def class_times(n, prec, sched, boxes, iters=30):
    """per-class kernel times (ms, HIP events on the solver's stream) of one solve of
    `iters` iterations under the schedule and the box variants"""
    env = {"HELM_ND_LEAF": str(sched["leaf"]), "HELM_ND_ROOT": str(sched["root"]), "HELM_ND_CUTS": sched["cuts"],
           "HELM_ND_MERGE": sched.get("merge", "none"),
           "HELM_ND_SPLITK_KB": str(sched.get("splitk_kb", SPLITK_DEFAULT_KB)), "HELM_BOXES": boxes}
    saved = {k: os.environ.get(k) for k in env}
    os.environ.update(env)
    try:
        dim, h, kappa, omega, layer = _problem(n)
        s = Solver(n, h, kappa, omega, layer=layer, sigma_max=2.0, alpha=1.1, alpha2=1.0, beta=0.1,
                   nu=(1, 1), cycle_prec=prec)
        q = np.zeros(int(np.prod([k + 1 for k in n])), np.complex128)
        q[q.size // 2] = 1.0
        s.solve(q, tol=1e-300, max_iter=iters)
        s.set_timing(True)
        s.solve(q, tol=1e-300, max_iter=iters)
        torch.cuda.synchronize()
        kt = {k: v[0] for k, v in s.kernel_times().items()}
        s.set_timing(False)
        s.close()
        return kt
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
        torch.cuda.empty_cache()


def tune_boxes(n, prec, sched, verbose=True):
    """stage three: the box shapes of the tiled cycle kernels (level-1 sweep, level-1
    restriction, level-2 sweep, level-2 restriction) under the given schedule.  Each class
    is timed by its own HIP events (whole iterations vary by about as much as one class's
    gain); a variant replaces the default when its class time is 2 % lower.  Returns (boxes
    string, {class: ms} of the choice)."""
    classes = ("l1_sweep", "l1_restrict", "l2_sweep", "l2_restrict")
    # 3D adds the z-marching tiles (sweeps 4 and 5, restrictions 3 and 4)
    nvar = (6, 5, 6, 5) if len(n) == 3 else (4, 3, 4, 3)
    base = class_times(n, prec, sched, "0,0,0,0")
    boxes = [0, 0, 0, 0]
    best_ms = {c: base[c] for c in classes}
    for v in range(1, max(nvar)):
        trial = [v if v < nvar[q] else 0 for q in range(4)]
        bx = ",".join(map(str, trial))
        kt = class_times(n, prec, sched, bx)
        for q, c in enumerate(classes):
            if trial[q] and kt[c] < 0.98 * best_ms[c]:
                boxes[q], best_ms[c] = trial[q], kt[c]
        if verbose:
            print("  boxes %s -> %s" % (bx, " ".join("%s %.3f" % (c, kt[c]) for c in classes)), flush=True)
    if verbose:
        print("  default -> %s" % " ".join("%s %.3f" % (c, base[c]) for c in classes), flush=True)
    return ",".join(map(str, boxes)), {c: round(best_ms[c], 4) for c in classes}

def tune(n, prec="f32", out=None, its=150, verbose=True, stack="p5", transfer=None):
    n = tuple(int(k) for k in n)
    dim = len(n)
    key = cache_key(n, prec, stack, transfer)
    results, seen = [], set()

    def run(cands):
        for leaf, root, cuts, merge, sk in cands:
            try:
                t, ts, info = time_schedule(n, prec, leaf, root, cuts, merge=merge, splitk_kb=sk, stack=stack,
                                            transfer=transfer)
            except L.HelmError as e:
                if verbose:
                    print("  leaf %d root %d cuts %r merge %r: %s" % (leaf, root, cuts, merge, e), flush=True)
                continue
            eff = (leaf, root, tuple(info["nd_cuts"]), tuple(info["nd_merge"]), info["fwd_launches"],
                   info["bwd_launches"])
            if eff in seen:            # the planner dropped cuts that do not fit: same schedule
                continue
            seen.add(eff)
            results.append({"leaf": leaf, "root": root, "cuts": ",".join(map(str, info["nd_cuts"])) or "none",
                            "merge": ",".join(map(str, info["nd_merge"])) or "none", "splitk_kb": sk,
                            "us_per_it": round(t * 1e6, 2), "setup_ms": round(ts * 1e3, 3),
                            "score_ms": round((ts + its * t) * 1e3, 3)})
            if verbose:
                print("  leaf %3d root %5d cuts %-8s merge %-12s split-K %10d KB -> %8.1f us/iteration, "
                      "set-up %8.2f ms, score %8.2f ms" % (leaf, root, results[-1]["cuts"], results[-1]["merge"][:12],
                                                          sk, t * 1e6, ts * 1e3, results[-1]["score_ms"]), flush=True)

    run(_candidates(dim))
    run(list(_stage_two(results, top=3 if dim == 2 else 1)))
    results.sort(key=lambda r: r["score_ms"])
    best = dict(results[0])
    best["boxes"] = "0,0,0,0"
    if stack == "p5":
        best["boxes"], best["box_class_ms"] = tune_boxes(n, prec, best, verbose)
    best["device"] = torch.cuda.get_device_name(0)
    best["score"] = "setup + %d iterations" % its
    best["runners_up"] = results[1:6]
    path = out or os.environ.get("HELM_TUNE_CACHE") or L.TUNE_CACHE
    cache = {}
    if os.path.exists(path):
        with open(path) as f:
            cache = json.load(f)
    cache[key] = best
    with open(path, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    if verbose:
        print("%s -> leaf %d root %d cuts %s merge %s (%.1f us/iteration, set-up %.2f ms), written to %s" % (
            key, best["leaf"], best["root"], best["cuts"], best["merge"], best["us_per_it"], best["setup_ms"],
            path), flush=True)
    return key, best


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, nargs="+", required=True, help="cells per axis (2 or 3 values)")
    ap.add_argument("--prec", choices=("f32", "f64"), default="f32")
    ap.add_argument("--out", default=None)
    ap.add_argument("--its", type=int, default=150, help="iterations per set-up in the score")
    ap.add_argument("--stack", choices=("p5", "compact"), default="p5")
    ap.add_argument("--transfer", choices=("cubic", "levdep"), default=None)
    ap.add_argument("--boxes-only", action="store_true",
                    help="only stage three (cycle-kernel boxes) under the cache entry's schedule")
    a = ap.parse_args()
    if a.boxes_only:
        n = tuple(a.n)
        key = cache_key(n, a.prec)
        path = a.out or os.environ.get("HELM_TUNE_CACHE") or L.TUNE_CACHE
        cache = json.load(open(path))
        cache[key].pop("us_per_it_boxes", None)
        cache[key]["boxes"], cache[key]["box_class_ms"] = tune_boxes(n, a.prec, cache[key])
        with open(path, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        print("%s -> boxes %s %s" % (key, cache[key]["boxes"], cache[key]["box_class_ms"]))
        return
    tune(a.n, a.prec, a.out, a.its, stack=a.stack, transfer=a.transfer)


if __name__ == "__main__":
    main()
