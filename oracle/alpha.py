"""Grid-to-grid dispersion analysis and the optimal real shift (oracle side).

Test infrastructure only (see the package docstring).

Follows Sec. 4 of the paper:

* a constant-coefficient stencil s (h = 1, dimensionless wavenumber kh = 2 pi / G)
  has the symbol  S(theta) = sum_k s_k exp(i k.theta)  (eq. (4.3)); for the
  symmetric stencils here that is  sum_k s_k cos(k.theta);
* the discrete radius r(phi) in direction phi is the distance from the origin to
  the first sign change of S along the ray theta = r u(phi) (Sec. 4.1);
* the Galerkin stencil of R A P is the full convolution r * s * p sampled at even
  offsets (Sec. 4.2, stencil convolution and down-sampling); applying it twice
  with the real-shifted fine stencil (k -> alpha k, eq. (3.5)) gives the stencil
  of H_4h^alpha (eq. (3.6));
* e_g(alpha, phi) = V_1 / (4 V_3) - 1 = r_3 / (4 r_1) - 1  (eq. (4.8) with
  eq. (4.6): the velocity ratio is the inverse radius ratio);
* alpha* = argmin_alpha max_phi |e_g(alpha, phi)|  (eq. (4.10)) by exhaustive
  search with alpha step 5e-4, phi in [0, pi/4] step 0.1 (2D) and azimuth
  [0, pi/4] x polar [pi/2 - arccos(1/sqrt 3), pi/2] step 0.1 (3D), and the ray
  sampled at 1e-3 (Sec. 4.3);
* n_crit bounds  G/(4 e_g) <= n_crit <= G/(2 e_g)  (eq. (4.9)).

Stacks: 'p5' / 'p7' second-order 5/7-point stencil (M = I), 'c9' / 'c19' the
compact fourth-order stencils of eq. (3.1)/(3.2); transfers 'fw' (full weighting
[1 2 1]/4 with linear interpolation), 'cubic' ([1 4 6 4 1]/16, eq. (3.3)) and
'levdep' (cubic except the level-2 -> 3 restriction [1 2 1]/4, eq. (3.4)).  The
prolongation is 2^d R^T; its scale does not move the zero set of the symbol.
"""
from __future__ import annotations

import math
from typing import Tuple

import numpy as np
from scipy.optimize import brentq
from scipy.signal import convolve


def _outer(vs):
    out = np.asarray(vs[0], np.float64)
    for v in vs[1:]:
        out = np.multiply.outer(out, np.asarray(v, np.float64))
    return out


def fine_stencil(kind: str, kh: float) -> np.ndarray:
    """L - (kh)^2 M as a 3^d array indexed [..., dy, dx] (h = 1)."""
    if kind in ("p5", "p7"):
        d = 2 if kind == "p5" else 3
        L = np.zeros((3,) * d)
        M = np.zeros((3,) * d)
        c = (1,) * d
        L[c] = 2.0 * d
        M[c] = 1.0
        for a in range(d):
            for s in (0, 2):
                idx = list(c)
                idx[a] = s
                L[tuple(idx)] = -1.0
        return L - kh * kh * M
    if kind == "c9":                               # eq. (3.1)
        L = np.array([[-1, -4, -1], [-4, 20, -4], [-1, -4, -1]], np.float64) / 6.0
        M = np.array([[0, 1, 0], [1, 8, 1], [0, 1, 0]], np.float64) / 12.0
        return L - kh * kh * M
    if kind == "c19":                              # eq. (3.2)
        outer = np.array([[0, 1, 0], [1, 2, 1], [0, 1, 0]], np.float64)
        mid = np.array([[1, 2, 1], [2, -24, 2], [1, 2, 1]], np.float64)
        L = -np.stack([outer, mid, outer]) / 6.0
        mo = np.array([[0, 0, 0], [0, 1, 0], [0, 0, 0]], np.float64)
        mm = np.array([[0, 1, 0], [1, 6, 1], [0, 1, 0]], np.float64)
        M = np.stack([mo, mm, mo]) / 12.0
        return L - kh * kh * M
    raise ValueError(kind)


def transfer_1d(kind: str, level: int) -> Tuple[np.ndarray, np.ndarray]:
    """(restriction, prolongation) 1-D stencils between level and level+1 (level 1 = fine)."""
    fw = np.array([1, 2, 1], np.float64) / 4.0
    cub = np.array([1, 4, 6, 4, 1], np.float64) / 16.0
    if kind == "fw":
        return fw, 2.0 * fw
    if kind == "cubic":
        return cub, 2.0 * cub
    if kind == "levdep":
        return (cub if level == 1 else fw), 2.0 * cub
    raise ValueError(kind)


def galerkin_stencil(s: np.ndarray, r1: np.ndarray, p1: np.ndarray) -> np.ndarray:
    """stencil of R A P: even-offset samples of the full convolution r * s * p."""
    d = s.ndim
    r = _outer([r1] * d)
    p = _outer([p1] * d)
    full = convolve(convolve(r, s), p)
    c = (full.shape[0] - 1) // 2
    half = c // 2
    sl = tuple(slice(c - 2 * half, c + 2 * half + 1, 2) for _ in range(d))
    return full[sl]


def coarse_stencil(kind: str, transfer: str, kh: float, alpha: float) -> np.ndarray:
    """stencil of H_4h^alpha = R2 (R1 H^alpha P1) P2 (eq. (3.6))."""
    s = fine_stencil(kind, alpha * kh)
    r, p = transfer_1d(transfer, 1)
    s2 = galerkin_stencil(s, r, p)
    r, p = transfer_1d(transfer, 2)
    return galerkin_stencil(s2, r, p)


def symbol(st: np.ndarray, theta: np.ndarray) -> np.ndarray:
    """S(theta) = sum_k s_k cos(k.theta) for theta of shape (..., d)."""
    d = st.ndim
    c = (st.shape[0] - 1) // 2
    offs = np.stack(np.meshgrid(*[np.arange(-c, c + 1)] * d, indexing="ij"), -1).reshape(-1, d)
    w = st.reshape(-1)
    keep = w != 0
    offs, w = offs[keep], w[keep]
    # stencil array is indexed [..., dy, dx]: offset component j pairs with theta[d-1-j]
    th = theta[..., ::-1]
    ph = th @ offs.T.astype(np.float64)
    return np.cos(ph) @ w


def directions(dim: int, step: float = 0.1) -> np.ndarray:
    if dim == 2:
        phis = np.arange(0.0, math.pi / 4 + 1e-12, step)
        return np.stack([np.cos(phis), np.sin(phis)], -1)
    az = np.arange(0.0, math.pi / 4 + 1e-12, step)
    pol = np.arange(math.pi / 2 - math.acos(1 / math.sqrt(3)), math.pi / 2 + 1e-12, step)
    out = []
    for p in pol:
        for a in az:
            out.append([math.sin(p) * math.cos(a), math.sin(p) * math.sin(a), math.cos(p)])
    return np.array(out)


def ray_radius(st: np.ndarray, u: np.ndarray, dr: float = 1e-3, rmax=None,
               mode: str = "root") -> float:
    """distance to the first sign change of the symbol along r*u, sampled from r = 0.

    mode 'root' refines the bracket by brentq; 'after' / 'before' return the first
    sample past / the last sample before the change.  Samples are taken on the
    grid k*dr up to rmax (scanned in chunks so the scan stops at the first change)."""
    if rmax is None:                       # the ray leaves [-pi, pi]^d at pi / max|u_i|
        rmax = math.pi / float(np.max(np.abs(u)))
    s0 = None
    k0 = 0
    nmax = int(round(rmax / dr))
    chunk = 256
    while k0 <= nmax:
        ks = np.arange(k0, min(k0 + chunk, nmax + 1))
        rs = ks * dr
        vals = symbol(st, rs[:, None] * u[None, :])
        if s0 is None:
            s0 = np.sign(vals[0])
        ch = np.nonzero(np.sign(vals) != s0)[0]
        if len(ch):
            k = int(ks[ch[0]])
            if mode == "after":
                return k * dr
            if mode == "before":
                return (k - 1) * dr
            f = lambda r: float(symbol(st, (r * u)[None, :])[0])
            return float(brentq(f, (k - 1) * dr, k * dr, xtol=1e-14))
        k0 += chunk
    return float("nan")


def _fine_radii(kind: str, G: float, mode: str) -> np.ndarray:
    dim = 2 if kind in ("p5", "c9") else 3
    s1 = fine_stencil(kind, 2.0 * math.pi / G)
    return np.array([ray_radius(s1, u, mode=mode) for u in directions(dim)])


def eg(kind: str, transfer: str, G: float, alpha: float, mode: str = "root",
       r1=None) -> np.ndarray:
    """e_g(alpha, phi) over the sampled directions (eq. (4.8))."""
    dim = 2 if kind in ("p5", "c9") else 3
    kh = 2.0 * math.pi / G
    if r1 is None:
        r1 = _fine_radii(kind, G, mode)
    s3 = coarse_stencil(kind, transfer, kh, alpha)
    r3 = np.array([ray_radius(s3, u, mode=mode) for u in directions(dim)])
    return r3 / (4.0 * r1) - 1.0


def alpha_star(kind: str, transfer: str, G: float, lo: float = 1.0, hi: float = 1.2,
               step: float = 5e-4, mode: str = "root", exhaustive: bool = False):
    """(alpha*, max_phi |e_g(alpha*)|) (eq. (4.10)).

    exhaustive=True scans every alpha on the 5e-4 grid; otherwise the grid is
    scanned at 10x the step first and then at the full resolution around the best
    coarse value (the same answer when the objective is unimodal in alpha)."""
    r1 = _fine_radii(kind, G, mode)
    def obj(a):
        e = np.abs(eg(kind, transfer, G, a, mode, r1))
        return float(np.max(e)) if np.all(np.isfinite(e)) else float("inf")
    grid = lo + step * np.arange(int(round((hi - lo) / step)) + 1)
    if exhaustive:
        cand = grid
    else:
        coarse_pts = grid[::10]
        vals = [obj(a) for a in coarse_pts]
        b = int(np.argmin(vals))
        lo_i = max(0, 10 * b - 10)
        hi_i = min(len(grid) - 1, 10 * b + 10)
        cand = grid[lo_i:hi_i + 1]
    best_a, best_e = None, float("inf")
    for a in cand:
        e = obj(a)
        if e < best_e - 1e-15:
            best_a, best_e = float(round(a, 6)), e
    return best_a, best_e


def level2_stencil(kind: str, transfer: str, kh: float, alpha2: float) -> np.ndarray:
    """stencil of the level-2 Galerkin operator R1 H^alpha2 P1 (the second shift of Remark 4.1)."""
    s = fine_stencil(kind, alpha2 * kh)
    r, p = transfer_1d(transfer, 1)
    return galerkin_stencil(s, r, p)


def eg_level2(kind: str, transfer: str, G: float, alpha2: float, mode: str = "root",
              r1=None) -> np.ndarray:
    """grid-1-to-grid-2 analogue of eq. (4.8): e = r_2 / (2 r_1) - 1 over the sampled directions."""
    dim = 2 if kind in ("p5", "c9") else 3
    kh = 2.0 * math.pi / G
    if r1 is None:
        r1 = _fine_radii(kind, G, mode)
    s2 = level2_stencil(kind, transfer, kh, alpha2)
    r2 = np.array([ray_radius(s2, u, mode=mode) for u in directions(dim)])
    return r2 / (2.0 * r1) - 1.0


def alpha2_star(kind: str, transfer: str, G: float, lo: float = 1.0, hi: float = 1.1,
                step: float = 5e-4, mode: str = "root"):
    """(alpha2*, max |e|): the level-2 shift minimising the worst grid-1-to-grid-2 error."""
    r1 = _fine_radii(kind, G, mode)
    best_a, best_e = None, float("inf")
    for a in lo + step * np.arange(int(round((hi - lo) / step)) + 1):
        e = np.abs(eg_level2(kind, transfer, G, a, mode, r1))
        v = float(np.max(e)) if np.all(np.isfinite(e)) else float("inf")
        if v < best_e - 1e-15:
            best_a, best_e = float(round(a, 6)), v
    return best_a, best_e


def ncrit_bounds(G: float, e: float) -> Tuple[float, float]:
    """eq. (4.9): G/(4 e_g) <= n_crit <= G/(2 e_g)."""
    return G / (4.0 * e), G / (2.0 * e)
