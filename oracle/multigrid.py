"""3-level real-shifted multigrid cycle (oracle).

Test infrastructure only (see the package docstring).

Levels (Sec. 3):
  A1 = H_beta               fine operator of the preconditioner (complex shift beta, Sec. 5.1.1)
  A2 = R1 A1 P1             Galerkin, eq. (2.2)  (optionally from H_beta^{alpha2})
  A3 = R2 (R1 H_beta^alpha P1) P2     real-shifted coarsest Galerkin operator, eq. (3.6)
and A3 is solved exactly (Sec. 2: "exact solution on a coarser grid"; Sec. 3.1).

The cycle follows the two-grid algorithm of Sec. 2 (pre-relax, restrict the
residual, coarse solve, correct, post-relax) applied recursively; gamma = 1 gives
a V-cycle and gamma = 2 a W-cycle (two recursive calls, the second on the
updated residual).  Relaxation is damped Jacobi x <- x + w D^{-1}(b - A x)
(Sec. 5.1).  `stationary` uses the cycle as a solver on its own.
"""
from __future__ import annotations

from typing import Optional

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import operators as ops


class Hierarchy:
    """stack 'p5fw': the 5/7-point operator with full weighting and linear interpolation;
    'compact': the paper's compact fourth-order operator (eqs. (3.1)/(3.2)) with the transfers
    named by `transfer` ('cubic', eq. (3.3); 'levdep', eq. (3.4); 'fw')."""

    def __init__(self, n, h, m, omega, layer, sigma_max, alpha=1.0, beta=0.0,
                 alpha2=1.0, cycle=2, nu_pre=1, nu_post=1, jacobi=(0.8, 0.8),
                 conj=False, r_scale=1.0, p_scale=1.0, stack="p5fw", transfer=None):
        n = tuple(int(k) for k in n)
        assert all(k % 4 == 0 for k in n), "three levels need n divisible by 4"
        self.n1, self.n2, self.n3 = n, ops.coarse(n), ops.coarse(ops.coarse(n))
        self.h = h
        self.sigma = ops.layer_sigma(n, layer, sigma_max)
        self.m = np.asarray(m, np.float64).ravel()
        self.omega = omega
        op = ops.helmholtz if stack == "p5fw" else ops.helmholtz_compact
        transfer = transfer or ("fw" if stack == "p5fw" else "cubic")
        # the operator the outer Krylov method solves (no shifts)
        self.H = op(n, h, self.m, omega, self.sigma)
        A1 = op(n, h, self.m, omega, self.sigma, beta=beta)
        A1_a2 = A1 if alpha2 == 1.0 else op(n, h, self.m, omega, self.sigma, beta=beta, alpha=alpha2)
        A1_a = op(n, h, self.m, omega, self.sigma, beta=beta, alpha=alpha)
        R1, P1 = ops.transfers(self.n1, transfer, 1)
        R2, P2 = ops.transfers(self.n2, transfer, 2)
        self.R1 = r_scale * R1
        self.P1 = p_scale * P1
        self.R2 = r_scale * R2
        self.P2 = p_scale * P2
        A2 = ops.galerkin(self.R1, A1_a2, self.P1)
        A3 = ops.galerkin(self.R2, ops.galerkin(self.R1, A1_a, self.P1), self.P2)
        if conj:
            self.H = self.H.conjugate().tocsr()
            A1, A2, A3 = A1.conjugate().tocsr(), A2.conjugate().tocsr(), A3.conjugate().tocsr()
        self.A = [A1.tocsr(), A2.tocsr(), A3.tocsr()]
        self.R = [self.R1, self.R2]
        self.P = [self.P1, self.P2]
        self.D = [A1.diagonal(), A2.diagonal()]
        self.lu3 = spla.splu(A3.tocsc())
        self.gamma = cycle
        self.nu_pre, self.nu_post = nu_pre, nu_post
        self.w = tuple(jacobi) if np.ndim(jacobi) else (jacobi, jacobi)

    def relax(self, lev: int, x: np.ndarray, b: np.ndarray, sweeps: int) -> np.ndarray:
        """damped Jacobi: x <- x + w D^{-1} (b - A x), `sweeps` times."""
        A, D, w = self.A[lev], self.D[lev], self.w[lev]
        for _ in range(sweeps):
            x = x + w * (b - A @ x) / D
        return x

    def coarse_solve(self, b: np.ndarray) -> np.ndarray:
        return self.lu3.solve(b)

    def cycle(self, lev: int, b: np.ndarray, x: Optional[np.ndarray] = None) -> np.ndarray:
        """one cycle on level `lev` (0 = fine) for A_lev x = b from initial guess x (default 0)."""
        if lev == 2:
            return self.coarse_solve(b)
        if x is None:
            x = np.zeros_like(b)
        A = self.A[lev]
        x = self.relax(lev, x, b, self.nu_pre)                 # 1. pre-relaxation
        bc = self.R[lev] @ (b - A @ x)                        # 2. restrict the residual
        if lev + 1 == 2:
            e = self.coarse_solve(bc)                         # 3. exact coarsest solve
        else:
            e = np.zeros_like(bc)
            for _ in range(self.gamma):                       # 3. gamma recursive calls
                e = e + self.cycle(lev + 1, bc - self.A[lev + 1] @ e)
        x = x + self.P[lev] @ e                               # 4. coarse-grid correction
        x = self.relax(lev, x, b, self.nu_post)               # 5. post-relaxation
        return x

    def precond(self, v: np.ndarray) -> np.ndarray:
        """M^{-1} v: one cycle on the fine level from a zero initial guess."""
        return self.cycle(0, v)


def stationary(hier: Hierarchy, b: np.ndarray, tol: float = 1e-6, max_iter: int = 500, x0=None):
    """the cycle used as a solver on its own (Sec. 5.1, the counts in parentheses of Table 3):
    the stationary iteration x <- x + M^{-1}(b - H x) until ||b - H x|| <= tol ||b||, or until
    the residual exceeds 1e8 ||b|| (divergence).  Returns (x, cycles, relative residual after
    every cycle)."""
    b = np.asarray(b, np.complex128)
    x = np.zeros_like(b) if x0 is None else np.array(x0, np.complex128)
    bn = np.linalg.norm(b)
    if bn == 0.0:
        return np.zeros_like(b), 0, []
    r = b - hier.H @ x
    rel = np.linalg.norm(r) / bn
    hist = []
    its = 0
    while rel > tol and its < max_iter:
        x = x + hier.precond(r)
        r = b - hier.H @ x
        rel = np.linalg.norm(r) / bn
        its += 1
        hist.append(rel)
        if not np.isfinite(rel) or rel > 1e8:
            break
    return x, its, hist


def from_problem(prob, conj=False, **kw) -> Hierarchy:
    compact = getattr(prob, "stack", "p5") == "compact"
    args = dict(alpha=prob.alpha, alpha2=getattr(prob, "alpha2", 1.0), beta=prob.beta, cycle=prob.cycle,
                nu_pre=prob.nu_pre,
                nu_post=prob.nu_post,
                jacobi=tuple(prob.jacobi) if np.ndim(prob.jacobi) else (prob.jacobi, prob.jacobi),
                stack="compact" if compact else "p5fw",
                transfer=getattr(prob, "transfer", None) if compact else None)
    args.update(kw)
    return Hierarchy(prob.n, prob.h, prob.slowness ** 2, prob.omega, prob.layer, prob.sigma_max,
                     conj=conj, **args)
