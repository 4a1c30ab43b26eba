"""Restarted right-preconditioned flexible GMRES (oracle).

Test infrastructure only (see the package docstring).

The outer solver of the paper's experiments (Sec. 5: FGMRES(20), stopping at a
relative residual below 1e-6) in its textbook form (Saad, 1993):

  r0 = b - H x0, beta0 = ||r0||, v1 = r0 / beta0
  for j = 1..m:  z_j = M^{-1} v_j;  w = H z_j;
                 modified Gram-Schmidt against v_1..v_j -> h_{ij};
                 h_{j+1,j} = ||w||;  v_{j+1} = w / h_{j+1,j};
                 Givens rotations reduce the Hessenberg matrix; |g_{j+1}| is the
                 residual norm of the least-squares problem.
  x = x0 + Z_m y_m, y_m = argmin || beta0 e1 - Hbar y ||;  restart from the true residual.

The iteration count is the number of preconditioner applications.
"""
from __future__ import annotations

import dataclasses
from typing import Callable, List

import numpy as np


@dataclasses.dataclass
class Result:
    x: np.ndarray
    iterations: int
    restarts: int
    converged: bool
    history: List[float]          # estimated relative residual after every iteration
    true_rel_residual: float


def givens(a: complex, b: complex):
    """rotation G = [[c, s], [-conj(s), c]] with real c such that G [a, b]^T = [r, 0]^T."""
    if b == 0:
        return 1.0, 0.0 + 0.0j, a
    if a == 0:
        return 0.0, np.conj(b) / abs(b), abs(b) + 0j
    t = np.hypot(abs(a), abs(b))
    c = abs(a) / t
    s = (a / abs(a)) * np.conj(b) / t
    r = (a / abs(a)) * t
    return c, s, r


def fgmres(apply_H: Callable, precond: Callable, b: np.ndarray, x0=None, tol=1e-6,
           restart=20, max_iter=500, trace=None) -> Result:
    """trace: optional list; every restart cycle appends a dict with the cycle's starting
    iterate, its preconditioned directions Z (N x k), the iterate it returns and the
    Givens estimate at its end (a record for tests, no effect on the arithmetic)."""
    b = np.asarray(b, np.complex128)
    x = np.zeros_like(b) if x0 is None else np.array(x0, np.complex128)
    bnorm = np.linalg.norm(b)
    hist: List[float] = []
    if bnorm == 0.0:
        return Result(np.zeros_like(b), 0, 0, True, hist, 0.0)
    its, cycles = 0, 0
    converged = False
    r = b - apply_H(x)
    while True:
        beta0 = np.linalg.norm(r)
        if beta0 / bnorm <= tol:                         # true residual decides
            converged = True
            break
        if its >= max_iter:
            break
        cycles += 1
        m = restart
        V = [r / beta0]
        Z = []
        Hh = np.zeros((m + 1, m), np.complex128)
        cs = np.zeros(m)
        sn = np.zeros(m, np.complex128)
        g = np.zeros(m + 1, np.complex128)
        g[0] = beta0
        k = 0
        for j in range(m):
            z = precond(V[j])
            Z.append(z)
            w = apply_H(z)
            for i in range(j + 1):                       # modified Gram-Schmidt
                Hh[i, j] = np.vdot(V[i], w)
                w = w - Hh[i, j] * V[i]
            Hh[j + 1, j] = np.linalg.norm(w)
            its += 1
            k = j + 1
            for i in range(j):                           # previous rotations
                t = cs[i] * Hh[i, j] + sn[i] * Hh[i + 1, j]
                Hh[i + 1, j] = -np.conj(sn[i]) * Hh[i, j] + cs[i] * Hh[i + 1, j]
                Hh[i, j] = t
            c, s, rr = givens(Hh[j, j], Hh[j + 1, j])
            cs[j], sn[j] = c, s
            Hh[j, j] = rr
            Hh[j + 1, j] = 0.0
            g[j + 1] = -np.conj(s) * g[j]
            g[j] = c * g[j]
            est = abs(g[j + 1]) / bnorm
            hist.append(est)
            if est <= tol or its >= max_iter:
                break
            V.append(w / np.linalg.norm(w))
        # y = R^{-1} g by back substitution on the k x k upper triangle
        y = np.zeros(k, np.complex128)
        for i in range(k - 1, -1, -1):
            y[i] = (g[i] - Hh[i, i + 1:k] @ y[i + 1:k]) / Hh[i, i]
        x_start = x
        for i in range(k):
            x = x + y[i] * Z[i]
        if trace is not None:
            trace.append(dict(x_start=x_start.copy(), Z=np.stack(Z[:k], 1), x_end=x.copy(),
                              est=abs(g[k]) / bnorm, k=k))
        r = b - apply_H(x)
    return Result(x, its, max(cycles - 1, 0), converged, hist, float(np.linalg.norm(r) / bnorm))


def solve(hier, b, tol=1e-6, restart=20, max_iter=500, x0=None, trace=None) -> Result:
    """FGMRES on the hierarchy's outer operator H, preconditioned by one cycle."""
    return fgmres(lambda v: hier.H @ v, hier.precond, b, x0=x0, tol=tol, restart=restart,
                  max_iter=max_iter, trace=trace)
