"""Convergence factor of the cycle used as a solver, against the real shift alpha.

The analogue of the paper's comparison of the dispersion-optimal shift with the shift
that makes the multigrid cycle converge fastest (Sec. 4.3, Fig. 3), for this library's
stack (5-point stencil, full weighting, bilinear interpolation): for a homogeneous medium
with an absorbing layer at G points per wavelength, every alpha of a grid is set up
(helm_refactor) and the cycle is run as a stationary solver (helm_iterate); the
convergence factor is the geometric mean residual reduction per cycle over the cycles
after the first `skip`.  A factor above 1 means the cycle diverges at that shift.

    python -m paper_2604_19501_amd.sweep --n 128 --G 12 [--nu 2] [--lo 1.0 --hi 1.25 --step 0.005]
"""
from __future__ import annotations

import argparse
import json
import math

import numpy as np

from . import _lib as L
from .solver import Solver


def homogeneous(n, G, layer=16):
    """unit slowness on an n^d grid (h = 1/n), omega for G points per wavelength"""
    dim = len(n)
    h = 1.0 / max(n)
    kappa = np.ones(tuple(k + 1 for k in reversed(n)))
    return dim, h, kappa, 2.0 * math.pi / (G * h), tuple((layer, layer) for _ in range(dim))


def factor(hist, skip=10, floor=1e-12):
    """geometric mean reduction per cycle after the first `skip` cycles, up to the cycle
    where the relative residual reaches `floor` (past it the FP64 residual stalls at the
    rounding level and the ratio no longer measures the cycle)"""
    h = np.asarray(hist, np.float64)
    below = np.nonzero(h < floor)[0]
    if len(below):
        h = h[:below[0] + 1]
    if len(h) < 2:
        return float("nan")
    k0 = min(skip, len(h) // 2)
    return float((h[-1] / h[k0 - 1 if k0 > 0 else 0]) ** (1.0 / max(1, len(h) - k0)))


def sweep(n, G, alphas, nu=2, jacobi=0.8, cycles=60, prec="f32", cycle=2):
    dim, h, kappa, omega, layer = homogeneous(tuple(n), G)
    s = Solver(tuple(n), h, kappa, omega, layer=layer, sigma_max=2.0, alpha=float(alphas[0]), alpha2=1.0,
               beta=0.0, cycle=cycle, nu=(nu, nu), jacobi=jacobi, cycle_prec=prec)
    q = np.zeros(int(np.prod([k + 1 for k in n])), np.complex128)
    q[q.size // 2] = 1.0
    out = []
    for a in alphas:
        s.refactor(alpha=float(a))
        _, info = s.iterate(q, tol=1e-300, max_iter=cycles, history=True)
        out.append({"alpha": round(float(a), 6), "factor": factor(info["history"]), "cycles": info["iterations"],
                    "final_rel_residual": info["true_rel_residual"]})
    s.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, nargs="+", required=True)
    ap.add_argument("--G", type=float, required=True)
    ap.add_argument("--nu", type=int, default=2)
    ap.add_argument("--lo", type=float, default=1.0)
    ap.add_argument("--hi", type=float, default=1.25)
    ap.add_argument("--step", type=float, default=0.005)
    ap.add_argument("--cycles", type=int, default=60)
    a = ap.parse_args()
    alphas = a.lo + a.step * np.arange(int(round((a.hi - a.lo) / a.step)) + 1)
    res = sweep(a.n, a.G, alphas, nu=a.nu, cycles=a.cycles)
    best = min((r for r in res if math.isfinite(r["factor"])), key=lambda r: r["factor"])
    print(json.dumps({"n": a.n, "G": a.G, "nu": a.nu, "best": best, "sweep": res}))


if __name__ == "__main__":
    main()
