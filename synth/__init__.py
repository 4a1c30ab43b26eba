"""Seeded synthetic inputs for the real-shifted multigrid Helmholtz solver.

This module is shared by the FP64 CPU oracle and by the GPU library's tests and
benchmark.  It holds *inputs only*: media (slowness fields), source positions,
receiver sets and the frozen run parameters of each workload.  It contains none
of the method's arithmetic (no operator, transfer, smoother, Galerkin product or
Krylov step): both sides build those independently from these inputs.

Array convention (both sides): a grid with ``n[a]`` cells along axis ``a`` has
``n[a]+1`` nodes; node arrays are stored x-fastest, i.e. the flat index of node
``(i0, i1[, i2])`` is ``i0 + (n0+1)*(i1 + (n1+1)*i2)``.  As a numpy array that is
C order with shape ``(n2+1, n1+1, n0+1)`` (3D) or ``(n1+1, n0+1)`` (2D); grid axis
``a`` is numpy axis ``d-1-a``.  The depth axis is the last grid axis (y in 2D,
z in 3D); its low end (index 0) is the "top" face.

Workload recipes (synthetic stand-ins for the layered geophysical media of the
paper's 2D and 3D experiments, Sec. 5.1.2 and 5.2):

* layered medium: ``n_layers`` horizontal layers with velocities drawn uniformly
  in [1.5, 4.5] and sorted to increase with depth, interfaces at sorted uniform
  depths, times ``1 + 0.1*xi`` where ``xi`` is uniform white noise smoothed by a
  Gaussian of ``sigma`` cells and scaled to max |xi| = 1; clipped to [1.5, 4.5];
  slowness = 1/velocity.
* the angular frequency is fixed by the number of grid points per wavelength G
  at the largest slowness: omega = 2*pi / (G * h * kappa_max).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

VMIN, VMAX = 1.5, 4.5


def node_shape(n: Sequence[int]) -> Tuple[int, ...]:
    """numpy shape (C order, x fastest) of the node array of a grid with n cells."""
    return tuple(int(k) + 1 for k in reversed(list(n)))


def flat_index(n: Sequence[int], idx: Sequence[int]) -> int:
    """flat x-fastest index of node idx on a grid with n cells per axis."""
    f, stride = 0, 1
    for a in range(len(n)):
        f += int(idx[a]) * stride
        stride *= int(n[a]) + 1
    return f


def _gaussian_smooth(a: np.ndarray, sigma: float) -> np.ndarray:
    from scipy.ndimage import gaussian_filter
    return gaussian_filter(a, sigma=sigma, mode="nearest")


def layered_slowness(n: Sequence[int], n_layers: int, sigma_cells: float, seed: int,
                     noise: float = 0.1) -> np.ndarray:
    """Layered + smoothed-noise slowness on the nodes of a grid with n cells.

    Returns float64 array of node_shape(n)."""
    rng = np.random.default_rng(seed)
    shape = node_shape(n)
    nz = shape[0]  # depth = last grid axis = numpy axis 0
    interfaces = np.sort(rng.uniform(0.0, nz - 1, n_layers - 1))
    v_layers = np.sort(rng.uniform(VMIN, VMAX, n_layers))
    z = np.arange(nz, dtype=np.float64)
    vz = v_layers[np.searchsorted(interfaces, z)]
    v = np.broadcast_to(vz.reshape((nz,) + (1,) * (len(shape) - 1)), shape).astype(np.float64)
    xi = rng.uniform(-1.0, 1.0, shape)
    xi = _gaussian_smooth(xi, sigma_cells)
    xi /= np.abs(xi).max()
    v = np.clip(v * (1.0 + noise * xi), VMIN, VMAX)
    return 1.0 / v


def constant_slowness(n: Sequence[int], value: float = 1.0) -> np.ndarray:
    return np.full(node_shape(n), float(value), dtype=np.float64)


def omega_for_G(G: float, h: float, kappa_max: float) -> float:
    """angular frequency giving G grid points per wavelength at slowness kappa_max."""
    return 2.0 * math.pi / (G * h * kappa_max)


def random_sources(n: Sequence[int], layers, count: int, seed: int) -> List[Tuple[int, ...]]:
    """count distinct node positions drawn uniformly outside the absorbing layers."""
    rng = np.random.default_rng(seed)
    out: List[Tuple[int, ...]] = []
    seen = set()
    while len(out) < count:
        p = tuple(int(rng.integers(layers[a][0], n[a] - layers[a][1] + 1)) for a in range(len(n)))
        if p not in seen:
            seen.add(p)
            out.append(p)
    return out


def point_rhs(n: Sequence[int], pos: Sequence[int], value: complex = 1.0) -> np.ndarray:
    """complex128 flat right-hand side with one unit point source."""
    N = int(np.prod([k + 1 for k in n]))
    q = np.zeros(N, dtype=np.complex128)
    q[flat_index(n, pos)] = value
    return q


# Real shifts alpha* = argmin_alpha max_phi |e_g| for the contract stack
# (2nd-order 5/7-point stencil, full-weighting restriction, bi/trilinear
# prolongation), computed by the grid-to-grid dispersion analysis of Sec. 4.2
# (eq. 4.8 and 4.10) with alpha sampled at 5e-4 and the ray root refined.
# These constants are *inputs*; tests/golden/make_alpha.py regenerates them and
# tests/test_oracle_alpha.py checks that the analysis reproduces them.
ALPHA_STAR = {
    (2, 10.0): 1.1445, (2, 32.0 / 3.0): 1.1370, (2, 34.0 / 3.0): 1.1275, (2, 12.0): 1.1170,
    (3, 10.0): 1.1265, (3, 11.0): 1.1145, (3, 12.0): 1.1010,
}


def alpha_for(dim: int, G: float) -> float:
    for (d, g), a in ALPHA_STAR.items():
        if d == dim and abs(g - G) < 1e-9:
            return a
    raise KeyError((dim, G))


@dataclasses.dataclass
class Problem:
    """One Helmholtz instance: grid, medium, frequency, layer and multigrid parameters."""
    name: str
    dim: int
    n: Tuple[int, ...]
    h: float
    slowness: np.ndarray          # float64, node_shape(n)
    omega: float
    layer: Tuple[Tuple[int, int], ...]   # absorbing layer width in cells per (axis, low/high face)
    sigma_max: float
    alpha: float
    beta: float
    sources: List[Tuple[int, ...]]
    G: float
    alpha2: float = 1.0     # real shift of the level-2 Galerkin operator
    cycle: int = 2          # 1 = V, 2 = W
    nu_pre: int = 2
    nu_post: int = 2
    jacobi: object = 0.8    # damping weight, or (level 1, level 2)
    restart: int = 20
    tol: float = 1e-6
    stack: str = "p5"       # "p5" (5/7-point, full weighting) or "compact" (the paper's stack)
    transfer: Optional[str] = None   # compact stack: "cubic" or "levdep"

    @property
    def N(self) -> int:
        return int(np.prod([k + 1 for k in self.n]))

    def rhs(self, k: int = 0) -> np.ndarray:
        return point_rhs(self.n, self.sources[k])


SIGMA_MAX = 2.0


def config1(n: int = 128) -> Problem:
    """2D homogeneous: kappa = 1, G = 12, 16-cell layer on all faces, source at the centre."""
    dim, G = 2, 12.0
    h = 1.0 / n
    L = 16 if n >= 64 else max(2, n // 8)
    return Problem("cfg1_2d_homog_%d" % n, dim, (n, n), h, constant_slowness((n, n)),
                   omega_for_G(G, h, 1.0), ((L, L), (L, L)), SIGMA_MAX, alpha_for(dim, G), 0.0,
                   [(n // 2, n // 2)], G)


# level-2 real shifts: the same grid-to-grid analysis between levels 1 and 2
# (e = r_2 / (2 r_1) - 1) for the contract stack; used where both coarse grids are shifted.
# Regenerated by tests/golden/make_alpha.py like ALPHA_STAR.
ALPHA2_STAR = {
    (2, 10.0): 1.0360, (2, 32.0 / 3.0): 1.0315, (2, 34.0 / 3.0): 1.0280, (2, 12.0): 1.0255,
    (3, 10.0): 1.0315, (3, 11.0): 1.0260, (3, 12.0): 1.0220,
}


def alpha2_for(dim: int, G: float) -> float:
    for (d, g), a in ALPHA2_STAR.items():
        if d == dim and abs(g - G) < 1e-9:
            return a
    raise KeyError((dim, G))

CFG2_BETA = 0.1


def config2(n: int = 1024, seed: int = 2000) -> Problem:
    """2D layered: 8 layers + noise smoothed over 20 cells, G = 10 at the largest slowness,
    20-cell layer on all faces, source at the centre; real shifts on both coarse grids plus a
    complex shift of the preconditioner, W(1,1) cycle."""
    dim, G = 2, 10.0
    h = 1.0 / n
    sig = 20.0 * n / 1024.0 if n < 1024 else 20.0
    kap = layered_slowness((n, n), 8, sig, seed)
    L = 20 if n >= 128 else max(2, (20 * n) // 1024 + 2)
    return Problem("cfg2_2d_layered_%d" % n, dim, (n, n), h, kap, omega_for_G(G, h, kap.max()),
                   ((L, L), (L, L)), SIGMA_MAX, alpha_for(dim, G), CFG2_BETA, [(n // 2, n // 2)], G,
                   alpha2=alpha2_for(2, G), nu_pre=1, nu_post=1)


# 3D workloads: the paper's 3D smoothing (W(1,1), damping 0.6 on level 1 and 0.4 on level 2,
# Sec. 5.2) with a modest complex shift of the preconditioner
CFG3_JACOBI = (0.6, 0.4)
CFG3_BETA = 0.05


def config3(n: int = 256, seed: int = 3000) -> Problem:
    """3D layered: 6 layers + noise smoothed over 8 cells, G = 12, 12-cell layer on five faces
    (none on the top face), one source 10 cells below the centre of the top face."""
    dim, G = 3, 12.0
    h = 1.0 / n
    sig = 8.0 * n / 256.0 if n < 256 else 8.0
    kap = layered_slowness((n, n, n), 6, sig, seed)
    L = 12 if n >= 64 else max(2, (12 * n) // 256 + 2)
    depth = min(10, n // 2)
    return Problem("cfg3_3d_layered_%d" % n, dim, (n, n, n), h, kap, omega_for_G(G, h, kap.max()),
                   ((L, L), (L, L), (0, L)), SIGMA_MAX, alpha_for(dim, G), CFG3_BETA,
                   [(n // 2, n // 2, depth)], G, nu_pre=1, nu_post=1, jacobi=CFG3_JACOBI)


CFG4_SIZES = (256, 512, 768)
CFG4_G = (10.0, 32.0 / 3.0, 34.0 / 3.0, 12.0)


def config4_instance(i: int, per_size: int = 32, sizes=CFG4_SIZES, n_src: int = 8) -> Problem:
    """instance i of the batched 2D workload: sizes in blocks of per_size, frequency index
    i mod 4 (G from 10 to 12), layered medium seeded 4000+i, 8 seeded random sources;
    the same shifts and (1,1) smoothing as the 1024^2 layered workload."""
    n = sizes[(i // per_size) % len(sizes)]
    G = CFG4_G[i % 4]
    dim = 2
    h = 1.0 / n
    kap = layered_slowness((n, n), 8, 20.0 * n / 1024.0 if n < 1024 else 20.0, 4000 + i)
    L = 20
    srcs = random_sources((n, n), ((L, L), (L, L)), n_src, 40000 + i)
    return Problem("cfg4_inst%d_%d" % (i, n), dim, (n, n), h, kap, omega_for_G(G, h, kap.max()),
                   ((L, L), (L, L)), SIGMA_MAX, alpha_for(dim, G), CFG2_BETA, srcs, G,
                   alpha2=alpha2_for(dim, G), nu_pre=1, nu_post=1)


def config5(n: int = 128, seed: int = 5000, smooth_cells: float = 16.0):
    """3D inverse-problem workload: reference medium (config-3 generator), a smoothed copy as
    the evaluation point, 16 sources on a 4x4 lattice of the top node plane, receivers on
    every node of the top plane, G = 12, 12-cell layer on five faces.

    Returns (problem_at_m0, m_ref, receiver_flat_indices)."""
    dim, G = 3, 12.0
    h = 1.0 / n
    sig = 8.0 * n / 256.0
    kap_ref = layered_slowness((n, n, n), 6, sig, seed)
    m_ref = kap_ref ** 2
    m0 = _gaussian_smooth(m_ref, smooth_cells * n / 128.0)
    kap0 = np.sqrt(m0)
    L = 12 if n >= 64 else max(2, (12 * n) // 128 + 1)
    lat = [int(round(n * (k + 1) / 5.0)) for k in range(4)]
    srcs = [(a, b, 0) for b in lat for a in lat]
    kmax = max(kap_ref.max(), kap0.max())
    prob = Problem("cfg5_3d_grad_%d" % n, dim, (n, n, n), h, kap0, omega_for_G(G, h, kmax),
                   ((L, L), (L, L), (0, L)), SIGMA_MAX, alpha_for(dim, G), CFG3_BETA, srcs, G,
                   nu_pre=1, nu_post=1, jacobi=CFG3_JACOBI)
    rec = np.array([flat_index((n, n, n), (i0, i1, 0)) for i1 in range(n + 1) for i0 in range(n + 1)],
                   dtype=np.int64)
    return prob, m_ref, rec


def random_vector(N: int, seed: int, dtype=np.complex128) -> np.ndarray:
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    return v.astype(dtype)


# The paper's own discretisation (Sec. 3.1, 5.1, 5.2): compact fourth-order operator, cubic
# transfers in 2D and level-dependent ones in 3D, the real shift alpha* of Table 1 (2D) /
# Table 2 (3D) for the stack and G, W(1,1) cycle, damped Jacobi 0.89 on both levels in 2D
# and 0.6 / 0.4 in 3D, no complex shift, unit-square (cube) domain with a 20-cell absorbing
# layer (scaled down below 128 cells), point source at the centre.
PAPER_ALPHA = {
    (2, "cubic", 10.0): 1.014, (2, "cubic", 11.0): 1.0075, (2, "cubic", 12.0): 1.0045,
    (2, "levdep", 10.0): 1.029, (2, "levdep", 11.0): 1.019, (2, "levdep", 12.0): 1.0135,
    (3, "levdep", 10.0): 1.0245, (3, "levdep", 11.0): 1.0165, (3, "levdep", 12.0): 1.012,
}


def paper_stack(n: Sequence[int], transfer: Optional[str] = None, G: float = 12.0, lo: Optional[float] = None,
                alpha: Optional[float] = None, layer_cells: int = 20) -> Problem:
    """the paper's stack on a grid of n cells per axis.  Medium: homogeneous (Fig. 4b) or,
    with lo, Table 3's linear medium, whose slowness grows linearly with depth from lo at the
    top face to 1 at the bottom (the text's ranges read as slowness); G at the largest
    slowness."""
    n = tuple(int(k) for k in n)
    dim = len(n)
    transfer = transfer or ("cubic" if dim == 2 else "levdep")
    h = 1.0 / max(n)
    shape = node_shape(n)
    if lo is None:
        kap = np.ones(shape)
        name = "paper_homog"
    else:
        depth = np.linspace(0.0, 1.0, n[-1] + 1)
        prof = lo + (1.0 - lo) * depth
        kap = np.broadcast_to(prof.reshape((-1,) + (1,) * (dim - 1)), shape).copy()
        name = "paper_linear%g" % lo
    L = layer_cells if min(n) >= 128 else max(2, (layer_cells * min(n)) // 128)
    a = PAPER_ALPHA[(dim, transfer, float(G))] if alpha is None else alpha
    jac = (0.89, 0.89) if dim == 2 else (0.6, 0.4)
    return Problem("%s_%s_%s" % (name, transfer, "x".join(map(str, n))), dim, n, h, kap,
                   omega_for_G(G, h, float(kap.max())), tuple((L, L) for _ in range(dim)), SIGMA_MAX, a, 0.0,
                   [tuple(k // 2 for k in n)], G, nu_pre=1, nu_post=1, jacobi=jac, stack="compact",
                   transfer=transfer)


def paper_3d(n: Sequence[int] = (192, 192, 72), G: float = 12.0, seed: int = 6000) -> Problem:
    """stand-in for the paper's 3D layered-media experiment (Sec. 5.2, Table 5: grids of
    64x64x32 up to 192x192x72 cells, G = 12 and 10, no complex shift): a layered medium with
    sharp interfaces (8 layers, noise smoothed over 4 cells) on a shallow box, h from the
    horizontal extent, a 12-cell absorbing layer on the five faces other than the top one
    (none there), the source at the centre of the top face; the paper's 3D stack: compact
    19-point operator, level-dependent transfers, alpha* of Table 2, W(1,1) with Jacobi
    damping 0.6 / 0.4."""
    n = tuple(int(k) for k in n)
    h = 1.0 / max(n)
    kap = layered_slowness(n, 8, 4.0, seed)
    L = 12 if min(n) >= 64 else max(2, min(n) // 6)
    return Problem("paper3d_%s" % "x".join(map(str, n)), 3, n, h, kap, omega_for_G(G, h, float(kap.max())),
                   ((L, L), (L, L), (0, L)), SIGMA_MAX, PAPER_ALPHA[(3, "levdep", float(G))], 0.0,
                   [(n[0] // 2, n[1] // 2, 0)], G, nu_pre=1, nu_post=1, jacobi=(0.6, 0.4), stack="compact",
                   transfer="levdep")
