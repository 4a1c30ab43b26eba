"""Differentiable least-squares misfit of Helmholtz solves w.r.t. squared slowness.

    loss = helmholtz_misfit(m, solver, sources, receivers, data, tol=1e-10)
    loss.backward()          # m.grad = dL/dm

For H(m) = -Lap_h - omega^2 m (1 - i sigma) (eq. (1.1) with the absorbing layer),
sources q_s, receivers given as flat node indices (sampling operator P) and data d_s,

    L(m) = 1/2 sum_s || P u_s - d_s ||^2,   H(m) u_s = q_s.

The medium is handed to the library as m itself (helm_refactor_m).  The backward pass
first sets the solver up for the forward pass's medium again if it has been refactored
since (another loss evaluated with the same solver), then solves the adjoint systems
H^H lambda_s = P^T (P u_s - d_s) with the same preconditioner on the conjugate-transpose
operator (op = HELM_OP_C) and forms dL/dm_j = sum_s omega^2 Re(conj(lambda_s[j]) (1 - i sigma_j) u_s[j]) in the library's
gradient kernel.  A solver built with max_rhs > 1 solves the sources, and then the
adjoint systems, in lock-step groups (Solver.solve_many); each solution equals the one of
a separate solve.  Every solve and the gradient run in libhelm; this module only orders
the calls.
"""
from __future__ import annotations

from typing import Sequence

import torch

from . import _lib as L
from .solver import Solver


def _solve_all(solver: Solver, rhs, tol, max_iter, op, what):
    """solutions of op(H) x = rhs[k]: lock-step groups when the solver has the capacity"""
    if getattr(solver, "max_rhs", 1) > 1 and len(rhs) > 1:
        xs, infos = solver.solve_many(rhs, tol=tol, max_iter=max_iter, op=op)
    else:
        xs, infos = [], []
        for q in rhs:
            x, info = solver.solve(q, tol=tol, max_iter=max_iter, op=op)
            xs.append(x)
            infos.append(info)
    for k, info in enumerate(infos):
        if info["status"] != 0:
            raise L.HelmError(info["status"], "%s solve %d" % (what, k))
    return xs


class _Misfit(torch.autograd.Function):
    @staticmethod
    def forward(ctx, m, solver: Solver, sources, receivers, data, tol, max_iter):
        md = m.detach().to(torch.float64).contiguous().clone()
        solver.refactor(m=md)
        # the medium, frequency and shifts the forward solves used: the backward pass needs the
        # same operator, and the solver may have been set up for another medium meanwhile
        ctx.m_saved, ctx.version = md, solver.medium_version
        ctx.omega = solver.omega
        ctx.shift = (solver.shift.alpha, solver.shift.alpha2, solver.shift.beta)
        us, res = [], []
        loss = torch.zeros((), dtype=torch.float64, device=m.device)
        sols = _solve_all(solver, sources, tol, max_iter, L.HELM_OP_N, "forward")
        for s, u in enumerate(sols):
            r = u[receivers] - data[s]
            loss = loss + 0.5 * torch.sum(r.real ** 2 + r.imag ** 2)
            us.append(u)
            res.append(r)
        ctx.solver, ctx.us, ctx.res, ctx.receivers = solver, us, res, receivers
        ctx.tol, ctx.max_iter, ctx.N = tol, max_iter, m.numel()
        return loss

    @staticmethod
    def backward(ctx, gout):
        solver = ctx.solver
        if solver.medium_version != ctx.version:        # refactored since this forward pass
            a, a2, b = ctx.shift
            solver.refactor(m=ctx.m_saved, omega=ctx.omega, alpha=a, alpha2=a2, beta=b)
        rhss = []
        for r in ctx.res:
            rhs = torch.zeros(ctx.N, dtype=torch.complex128, device=r.device)
            rhs.index_put_((ctx.receivers,), r, accumulate=True)
            rhss.append(rhs)
        lams = _solve_all(solver, rhss, ctx.tol, ctx.max_iter, L.HELM_OP_C, "adjoint")
        g = solver.grad_m(ctx.us, lams)
        return gout * g, None, None, None, None, None, None


def helmholtz_misfit(m: torch.Tensor, solver: Solver, sources: Sequence[torch.Tensor], receivers: torch.Tensor,
                     data: Sequence[torch.Tensor], tol: float = 1e-10, max_iter: int = 1000) -> torch.Tensor:
    """L(m) = 1/2 sum_s ||P u_s - d_s||^2 with u_s = H(m)^{-1} q_s; differentiable in m (float64, N1)."""
    return _Misfit.apply(m, solver, list(sources), receivers, list(data), tol, max_iter)


class HelmholtzLoss(torch.nn.Module):
    """module form of helmholtz_misfit for a fixed solver, source set, receiver set and data."""

    def __init__(self, solver: Solver, sources, receivers, data, tol: float = 1e-10, max_iter: int = 1000):
        super().__init__()
        self.solver, self.sources, self.receivers, self.data = solver, list(sources), receivers, list(data)
        self.tol, self.max_iter = tol, max_iter

    def forward(self, m):
        return helmholtz_misfit(m, self.solver, self.sources, self.receivers, self.data, self.tol, self.max_iter)
