"""Least-squares misfit, adjoint solve and gradient w.r.t. squared slowness (oracle).

Test infrastructure only (see the package docstring).

For sources q_s, receivers given as flat node indices (the sampling operator P
picks those entries), and data d_s:

    H(m) u_s = q_s,   L(m) = 1/2 sum_s || P u_s - d_s ||^2.

H(m) = -Lap_h - diag(omega^2 m (1 - i sigma)) (the operator of eq. (1.1) with the
absorbing layer), so dH/dm_j = -omega^2 (1 - i sigma_j) e_j e_j^T and

    dL/dm_j = Re sum_s conj(lam_s[j]) omega^2 (1 - i sigma_j) u_s[j],
    H^H lam_s = P^T (P u_s - d_s).

H is complex symmetric (H^T = H), so H^H = conj(H).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from . import operators as ops


def _factor(n, h, m, omega, layer, sigma_max):
    sigma = ops.layer_sigma(n, layer, sigma_max)
    H = ops.helmholtz(n, h, m, omega, sigma)
    return H, sigma


def forward_exact(n, h, m, omega, layer, sigma_max, Q):
    """u_s = H^{-1} q_s for the columns of Q (N x S), sparse LU."""
    H, _ = _factor(n, h, m, omega, layer, sigma_max)
    lu = spla.splu(H.tocsc())
    return np.stack([lu.solve(Q[:, s]) for s in range(Q.shape[1])], 1)


def misfit(U, rec, D):
    R = U[rec, :] - D
    return 0.5 * float(np.sum(np.abs(R) ** 2))


def gradient_exact(n, h, m, omega, layer, sigma_max, Q, rec, D):
    """(L, dL/dm) with forward and adjoint solves by sparse LU (the plain definition)."""
    H, sigma = _factor(n, h, m, omega, layer, sigma_max)
    lu = spla.splu(H.tocsc())
    luH = spla.splu(H.conjugate().tocsc())
    N = H.shape[0]
    g = np.zeros(N)
    L = 0.0
    for s in range(Q.shape[1]):
        u = lu.solve(Q[:, s])
        r = u[rec] - D[:, s]
        L += 0.5 * float(np.sum(np.abs(r) ** 2))
        rhs = np.zeros(N, np.complex128)
        np.add.at(rhs, rec, r)
        lam = luH.solve(rhs)
        g += (omega ** 2) * np.real(np.conj(lam) * (1.0 - 1j * sigma) * u)
    return L, g
