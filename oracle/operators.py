"""Assembled sparse operators of the oracle (complex128).

Test infrastructure only (see the package docstring).

Discretisation (Sec. 1, eq. (1.1); Sec. 3.1 operator split H = -Lap_h - k^2 M_h with
M_h = I for the second-order stencil used here):

* nodes 0..n_a on every axis a (all of them are unknowns), spacing h, zero values
  one node beyond each end (Dirichlet ghost);
* -Lap_h = Kronecker sum over the axes of tridiag(-1, 2, -1)/h^2;
* k^2(x) = omega^2 m(x), m = slowness^2, and inside the absorbing layer the
  coefficient is damped:  c = omega^2 m (1 - i sigma(x)),
  sigma = sigma_max * sum_a (depth_a / L_a)^2 with depth_a the distance in cells
  into the layer of width L_a on that face (quadratic profile);
* complex shift beta (CSLP-type, Sec. 1 and 5.1.1):  c_beta = (1 - i beta) c;
* real shift alpha (eq. (3.5)):  k -> alpha k, i.e. c_alpha = alpha^2 c_beta.

Transfers (contract stack): 1-D full weighting R = [1 2 1]/4 on coarse nodes
I = 0..n/2 (fine node 2I and its neighbours, truncated at the ends) and
P = 2 R^T (linear interpolation); in d dimensions the Kronecker products, so
P = 2^d R^T.  Galerkin coarsening is eq. (2.2): A_c = R A P.

The paper's own stack (Sec. 3.1) is here too: the compact fourth-order 9-point (2D, eq.
(3.1)) and 19-point (3D, eq. (3.2)) operators H = L_h - M_h diag(c), and the high-order
transfers R = (x) [1 4 6 4 1]/16 (eq. (3.3)) and their level-dependent variant with full
weighting from level 2 to 3 (eq. (3.4)), prolongation 2^d R^T in every case.
"""
from __future__ import annotations

from typing import Sequence, Tuple

import numpy as np
import scipy.sparse as sp


def nodes(n: Sequence[int]) -> Tuple[int, ...]:
    return tuple(int(k) + 1 for k in n)


def kron_axes(mats):
    """operator acting with mats[a] on grid axis a, x-fastest flat ordering.

    flat = i0 + N0*(i1 + N1*i2): the slowest index is the last axis, so the
    Kronecker chain is kron(M_{d-1}, ..., kron(M_1, M_0))."""
    out = sp.csr_matrix(mats[0])
    for M in mats[1:]:
        out = sp.kron(sp.csr_matrix(M), out, format="csr")
    return out


def lap1d(n: int, h: float) -> sp.csr_matrix:
    """1-D second difference tridiag(-1, 2, -1)/h^2 on nodes 0..n (zero ghost values)."""
    N = n + 1
    main = np.full(N, 2.0)
    off = -np.ones(N - 1)
    return sp.diags([off, main, off], [-1, 0, 1], format="csr") / (h * h)


def neg_laplacian(n: Sequence[int], h: float) -> sp.csr_matrix:
    d = len(n)
    Ns = nodes(n)
    out = None
    for a in range(d):
        mats = [sp.identity(Ns[b], format="csr") for b in range(d)]
        mats[a] = lap1d(n[a], h)
        term = kron_axes(mats)
        out = term if out is None else out + term
    return out.tocsr()


def compact_laplacian(n: Sequence[int], h: float) -> sp.csr_matrix:
    """the fourth-order compact Laplacian of eq. (3.1) (2D) / eq. (3.2) (3D) with zero ghost
    values, as Kronecker products of T = tridiag(-1, 2, -1)/h^2: L5 - (h^2/6) T (x) T in 2D and
    L7 - (h^2/6)(T(x)T(x)I + T(x)I(x)T + I(x)T(x)T) in 3D (L5, L7: the 5/7-point sums)."""
    d = len(n)
    Ns = nodes(n)
    T = [lap1d(n[a], h) for a in range(d)]
    Id = [sp.identity(Ns[a], format="csr") for a in range(d)]
    out = neg_laplacian(n, h)
    for a in range(d):
        for b in range(a + 1, d):
            mats = list(Id)
            mats[a], mats[b] = T[a], T[b]
            out = out - (h * h / 6.0) * kron_axes(mats)
    return out.tocsr()


def compact_mass(n: Sequence[int], h: float) -> sp.csr_matrix:
    """the mass operator of eqs. (3.1)/(3.2): I - (h^2/12) L5 (2D, [0 1 0; 1 8 1; 0 1 0]/12)
    and I - (h^2/12) L7 (3D, centre 6/12 and the six face neighbours 1/12)."""
    N = int(np.prod(nodes(n)))
    return (sp.identity(N, format="csr") - (h * h / 12.0) * neg_laplacian(n, h)).tocsr()


def helmholtz_compact(n, h, m, omega, sigma, beta=0.0, alpha=1.0) -> sp.csr_matrix:
    """H = L_h - M_h diag(c), the compact fourth-order operator with the zeroth-order
    coefficient c of `coefficient` (eq. (1.1), (3.1)/(3.2), the shifts of (3.5))."""
    c = coefficient(m, omega, sigma, beta, alpha)
    L = compact_laplacian(n, h).astype(np.complex128)
    return (L - compact_mass(n, h).astype(np.complex128) @ sp.diags(c)).tocsr()


def restriction1d_cubic(n: int) -> sp.csr_matrix:
    """the high-order restriction [1 4 6 4 1]/16 (eq. (3.3)) from nodes 0..n onto 0..n/2"""
    assert n % 2 == 0
    nc = n // 2
    rows, cols, vals = [], [], []
    for I in range(nc + 1):
        for o, w in ((-2, 1 / 16), (-1, 4 / 16), (0, 6 / 16), (1, 4 / 16), (2, 1 / 16)):
            f = 2 * I + o
            if 0 <= f <= n:
                rows.append(I)
                cols.append(f)
                vals.append(w)
    return sp.csr_matrix((vals, (rows, cols)), shape=(nc + 1, n + 1))


def transfers(n: Sequence[int], kind: str, level: int):
    """(R, P) between level `level` (1 = fine, grid n) and the next: kind 'fw' (full
    weighting, linear interpolation), 'cubic' (eq. (3.3) both ways) or 'levdep' (eq. (3.4):
    cubic except the restriction from level 2 to 3, which is full weighting); P = 2^d R^T of
    the interpolating restriction in every case."""
    d = len(n)
    cub = kron_axes([restriction1d_cubic(k) for k in n])
    fw = restriction(n)
    if kind == "fw":
        R, Rp = fw, fw
    elif kind == "cubic":
        R, Rp = cub, cub
    elif kind == "levdep":
        R, Rp = (cub if level == 1 else fw), cub
    else:
        raise ValueError(kind)
    return R.tocsr(), ((2.0 ** d) * Rp.T).tocsr()


def layer_sigma(n: Sequence[int], layer, sigma_max: float) -> np.ndarray:
    """sigma(x) on the flat node vector: sigma_max * sum_a (depth_a/L_a)^2."""
    d = len(n)
    prof = []
    for a in range(d):
        i = np.arange(n[a] + 1, dtype=np.float64)
        lo, hi = layer[a]
        t = np.zeros_like(i)
        if lo > 0:
            t += (np.maximum(lo - i, 0.0) / lo) ** 2
        if hi > 0:
            t += (np.maximum(i - (n[a] - hi), 0.0) / hi) ** 2
        prof.append(t)
    # broadcast to the numpy node shape (axis a -> numpy axis d-1-a)
    tot = np.zeros(tuple(reversed(nodes(n))))
    for a in range(d):
        shape = [1] * d
        shape[d - 1 - a] = n[a] + 1
        tot = tot + prof[a].reshape(shape)
    return sigma_max * tot.ravel()


def coefficient(m: np.ndarray, omega: float, sigma: np.ndarray, beta: float = 0.0,
                alpha: float = 1.0) -> np.ndarray:
    """zeroth-order coefficient alpha^2 (1 - i beta) omega^2 m (1 - i sigma), flat."""
    return (alpha ** 2) * (1.0 - 1j * beta) * (omega ** 2) * np.asarray(m, np.float64).ravel() \
        * (1.0 - 1j * sigma)


def helmholtz(n, h, m, omega, sigma, beta=0.0, alpha=1.0) -> sp.csr_matrix:
    """H = -Lap_h - diag(c) with c as in `coefficient` (eq. (1.1), (3.5))."""
    c = coefficient(m, omega, sigma, beta, alpha)
    return (neg_laplacian(n, h).astype(np.complex128) - sp.diags(c)).tocsr()


def restriction1d(n: int) -> sp.csr_matrix:
    """full weighting [1 2 1]/4 from nodes 0..n onto coarse nodes 0..n/2."""
    assert n % 2 == 0
    nc = n // 2
    rows, cols, vals = [], [], []
    for I in range(nc + 1):
        for o, w in ((-1, 0.25), (0, 0.5), (1, 0.25)):
            f = 2 * I + o
            if 0 <= f <= n:
                rows.append(I)
                cols.append(f)
                vals.append(w)
    return sp.csr_matrix((vals, (rows, cols)), shape=(nc + 1, n + 1))


def restriction(n: Sequence[int]) -> sp.csr_matrix:
    return kron_axes([restriction1d(k) for k in n])


def prolongation(n: Sequence[int]) -> sp.csr_matrix:
    """P = 2^d R^T: d-linear interpolation from the coarse nodes."""
    d = len(n)
    return ((2.0 ** d) * restriction(n).T).tocsr()


def galerkin(R, A, P) -> sp.csr_matrix:
    """eq. (2.2): A_c = R A P."""
    return (R @ A @ P).tocsr()


def coarse(n: Sequence[int]) -> Tuple[int, ...]:
    return tuple(int(k) // 2 for k in n)


def stencil_apply_loops(n, h, m, omega, sigma, x, beta=0.0, alpha=1.0):
    """H x by explicit loops over nodes and the 5/7-point neighbours (tiny grids only).

    An independent construction of the same operator, used to cross-check the
    Kronecker assembly on small grids."""
    d = len(n)
    Ns = nodes(n)
    c = coefficient(m, omega, sigma, beta, alpha)
    y = np.zeros_like(x, dtype=np.complex128)
    strides = [1]
    for a in range(1, d):
        strides.append(strides[-1] * Ns[a - 1])
    for f in range(len(x)):
        idx = []
        r = f
        for a in range(d):
            idx.append(r % Ns[a])
            r //= Ns[a]
        acc = (2.0 * d / (h * h) - c[f]) * x[f]
        for a in range(d):
            for s in (-1, 1):
                j = idx[a] + s
                if 0 <= j <= n[a]:
                    acc -= x[f + s * strides[a]] / (h * h)
        y[f] = acc
    return y
