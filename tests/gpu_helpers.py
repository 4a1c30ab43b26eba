"""Shared helpers of the GPU parity tests (oracle-side views of the same inputs)."""
import numpy as np

import synth
from oracle import multigrid, operators as ops


def stencil_arrays(A, n_lev, r=1):
    """((2r+1)^d, N) array of a sparse operator of stencil radius r: entry k of row i is
    A[i, i + offset_k], offset k = (d0+r) + (2r+1) (d1+r) [+ (2r+1)^2 (d2+r)], zero where the
    neighbour is outside the grid."""
    d = len(n_lev)
    Ns = [k + 1 for k in n_lev]
    N = int(np.prod(Ns))
    w = 2 * r + 1
    K = w ** d
    out = np.zeros((K, N), np.complex128)
    A = A.tocoo()
    i, j = A.row, A.col
    ci = [i % Ns[0], (i // Ns[0]) % Ns[1]] + ([i // (Ns[0] * Ns[1])] if d == 3 else [])
    cj = [j % Ns[0], (j // Ns[0]) % Ns[1]] + ([j // (Ns[0] * Ns[1])] if d == 3 else [])
    off = [cj[a] - ci[a] for a in range(d)]
    assert all(np.all(np.abs(o) <= r) for o in off), "operator wider than radius %d" % r
    k = (off[0] + r) + w * (off[1] + r)
    if d == 3:
        k = k + w * w * (off[2] + r)
    out[k, i] = A.data
    return out


def small_problem(dim, n=None, seed=7, beta=0.03, alpha2=1.0):
    """layered medium with absorbing layers on every face, a few cells per level."""
    if dim == 2:
        n = n or 32
        p = synth.config2(n, seed=seed)
    else:
        n = n or 16
        p = synth.config3(n, seed=seed)
    p.beta = beta
    p.alpha2 = alpha2
    return p


def rect_problem(n, seed=11, G=10.0, beta=0.05, alpha2=1.03):
    """layered medium on a non-square grid (several kernel tiles per axis with ragged
    last tiles); layer of 4 cells on every face."""
    dim = len(n)
    h = 1.0 / max(n)
    kap = synth.layered_slowness(n, 4, 3.0, seed)
    layer = tuple((4, 4) for _ in range(dim))
    return synth.Problem("rect_%s" % "x".join(map(str, n)), dim, tuple(n), h, kap,
                         synth.omega_for_G(G, h, kap.max()), layer, synth.SIGMA_MAX,
                         synth.alpha_for(dim, 10.0), beta, [tuple(k // 2 for k in n)], G, alpha2=alpha2)


def oracle_hierarchy(p, **kw):
    args = dict(alpha2=getattr(p, "alpha2", 1.0))
    args.update(kw)
    return multigrid.from_problem(p, **args)


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def maxabs_rel(a, b):
    """element-wise relative difference max_i |a_i - b_i| / max_i |b_i|: a single wrong node
    shows here at its own size instead of being averaged over the grid as in `rel`."""
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))
