"""Pins of the oracle's operators against facts fixed by the paper and by mathematics.

* plane-wave symbol of the 5/7-point operator (Sec. 4.1, the second-order analogue
  of eq. (4.4)): h^2 (H phi)/phi = 2d - 2 sum cos(theta_i) - (kh)^2 at interior nodes,
  and H phi = 0 on the discrete dispersion relation;
* an explicit loop construction of H on tiny grids;
* closed forms of the Galerkin operators eq. (2.2) / eq. (3.6) for constant k,
  from 1-D Galerkin matrices worked out by hand (boundary rows included);
* the real-shift identity eq. (3.7);
* second-order convergence for a smooth manufactured solution.
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import synth
from oracle import operators as ops


def _grid_coords(n):
    d = len(n)
    axes = [np.arange(k + 1) for k in n]
    mesh = np.meshgrid(*axes[::-1], indexing="ij")   # numpy axes: slowest first
    return [mesh[d - 1 - a].ravel() for a in range(d)]


@pytest.mark.parametrize("n", [(12, 10), (8, 6, 10)])
def test_plane_wave_symbol(n):
    d = len(n)
    h = 0.1
    omega = 7.0
    m = np.full(int(np.prod([k + 1 for k in n])), 1.3)
    sigma = np.zeros_like(m)
    H = ops.helmholtz(n, h, m, omega, sigma)
    X = _grid_coords(n)
    interior = np.ones_like(X[0], bool)
    for a in range(d):
        interior &= (X[a] >= 1) & (X[a] <= n[a] - 1)
    kh2 = omega * omega * 1.3 * h * h
    rng = np.random.default_rng(1)
    for _ in range(4):
        th = rng.uniform(-math.pi, math.pi, d)
        phi = np.exp(1j * sum(th[a] * X[a] for a in range(d)))
        ratio = (h * h) * (H @ phi)[interior] / phi[interior]
        expect = 2 * d - 2 * np.sum(np.cos(th)) - kh2
        assert np.allclose(ratio, expect, rtol=0, atol=1e-11)
    # a wave on the discrete dispersion relation is annihilated at interior nodes
    th = np.zeros(d)
    th[0] = math.acos(1.0 - kh2 / 2.0)
    phi = np.exp(1j * th[0] * X[0])
    assert np.max(np.abs((H @ phi)[interior])) < 1e-9 / (h * h)


@pytest.mark.parametrize("n", [(4, 6), (4, 2, 4)])
def test_kronecker_assembly_matches_loops(n):
    h, omega = 0.25, 3.0
    N = int(np.prod([k + 1 for k in n]))
    rng = np.random.default_rng(3)
    m = rng.uniform(0.2, 1.0, N)
    layer = tuple((1, 2) for _ in n)
    sigma = ops.layer_sigma(n, layer, 2.0)
    x = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    H = ops.helmholtz(n, h, m, omega, sigma, beta=0.05, alpha=1.1)
    y = ops.stencil_apply_loops(n, h, m, omega, sigma, x, beta=0.05, alpha=1.1)
    assert np.allclose(H @ x, y, rtol=1e-14, atol=1e-12)
    assert abs(H - H.T).max() == 0.0          # complex symmetric


def test_layer_profile():
    n = (20, 20)
    s = ops.layer_sigma(n, ((4, 4), (0, 5)), 2.0).reshape(21, 21)   # [y, x]
    assert s[10, 10] == 0.0
    assert s[10, 0] == pytest.approx(2.0)          # outermost node of a 4-cell layer
    assert s[10, 2] == pytest.approx(2.0 * (2 / 4) ** 2)
    assert s[0, 10] == 0.0                         # no layer on the top face
    assert s[20, 10] == pytest.approx(2.0)
    assert s[20, 0] == pytest.approx(4.0)          # corner: both axes add


def _hand_1d(nc, level):
    """1-D Galerkin mass/stiffness matrices on nc+1 coarse nodes (worked out by hand for
    full weighting and linear interpolation with a zero ghost node beyond each end).
    level 2: M = tridiag(1/8, 3/4, 1/8) with corner 5/8, T = (2h)^-2 tridiag(-1,2,-1)
    with corner 3; level 3: M = tridiag(5,22,5)/32 with corner 15/32, T = (4h)^-2
    tridiag(-1,2,-1) with corner 5."""
    N = nc + 1
    if level == 2:
        M = sp.diags([np.full(N - 1, 1 / 8), np.full(N, 3 / 4), np.full(N - 1, 1 / 8)], [-1, 0, 1]).tolil()
        M[0, 0] = M[N - 1, N - 1] = 5 / 8
        T = sp.diags([-np.ones(N - 1), np.full(N, 2.0), -np.ones(N - 1)], [-1, 0, 1]).tolil()
        T[0, 0] = T[N - 1, N - 1] = 3.0
    else:
        M = sp.diags([np.full(N - 1, 5 / 32), np.full(N, 22 / 32), np.full(N - 1, 5 / 32)], [-1, 0, 1]).tolil()
        M[0, 0] = M[N - 1, N - 1] = 15 / 32
        T = sp.diags([-np.ones(N - 1), np.full(N, 2.0), -np.ones(N - 1)], [-1, 0, 1]).tolil()
        T[0, 0] = T[N - 1, N - 1] = 5.0
    return M.tocsr(), T.tocsr()


def _tensor(n_c, level, H, c):
    d = len(n_c)
    scale = (2.0 ** (level - 1) * H) ** -2
    Ms, Ts = zip(*[_hand_1d(k, level) for k in n_c])
    out = None
    for a in range(d):
        mats = list(Ms)
        mats[a] = Ts[a] * scale
        t = ops.kron_axes(mats)
        out = t if out is None else out + t
    return out - c * ops.kron_axes(list(Ms))


@pytest.mark.parametrize("n", [(16, 8), (8, 8, 12)])
def test_galerkin_closed_form(n):
    h, omega, kap, alpha, beta = 1.0 / 16, 20.0, 0.9, 1.12, 0.03
    N = int(np.prod([k + 1 for k in n]))
    m = np.full(N, kap * kap)
    sigma = np.zeros(N)
    Hb = ops.helmholtz(n, h, m, omega, sigma, beta=beta)
    Hba = ops.helmholtz(n, h, m, omega, sigma, beta=beta, alpha=alpha)
    n2 = ops.coarse(n)
    R1, P1 = ops.restriction(n), ops.prolongation(n)
    R2, P2 = ops.restriction(n2), ops.prolongation(n2)
    A2 = ops.galerkin(R1, Hb, P1)
    A3 = ops.galerkin(R2, ops.galerkin(R1, Hba, P1), P2)
    c = (1 - 1j * beta) * omega ** 2 * kap ** 2
    ref2 = _tensor(n2, 2, h, c)
    ref3 = _tensor(ops.coarse(n2), 3, h, alpha ** 2 * c)
    assert abs(A2 - ref2).max() <= 1e-12 * abs(ref2).max()
    assert abs(A3 - ref3).max() <= 1e-12 * abs(ref3).max()
    # stencil sizes: 9 (2D) / 27 (3D) points per interior coarse row
    assert A2.getnnz(axis=1).max() == 3 ** len(n)


def test_real_shift_identity():
    """eq. (3.7): the shift enters the coarsest operator as (1 - alpha^2) times the doubly
    Galerkin-coarsened mass term; linear in the coefficient, so it holds for variable media."""
    n = (16, 12)
    h, omega = 1.0 / 16, 25.0
    N = 17 * 13
    rng = np.random.default_rng(5)
    m = rng.uniform(0.1, 1.0, N)
    sigma = ops.layer_sigma(n, ((3, 3), (3, 3)), 2.0)
    alpha, beta = 1.117, 0.03
    R1, P1 = ops.restriction(n), ops.prolongation(n)
    n2 = ops.coarse(n)
    R2, P2 = ops.restriction(n2), ops.prolongation(n2)
    A3 = R2 @ R1 @ ops.helmholtz(n, h, m, omega, sigma, beta=beta) @ P1 @ P2
    A3a = R2 @ R1 @ ops.helmholtz(n, h, m, omega, sigma, beta=beta, alpha=alpha) @ P1 @ P2
    cb = ops.coefficient(m, omega, sigma, beta)
    M3 = R2 @ R1 @ sp.diags(cb) @ P1 @ P2
    diff = A3a - A3 - (1 - alpha ** 2) * M3
    assert abs(diff).max() <= 1e-12 * abs(A3).max()


def test_second_order_convergence():
    """smooth solution with zero values one node beyond the boundary, sigma = 0, k = 8:
    the discrete error decays as h^2 (textbook second order)."""
    errs = []
    for nn in (14, 30, 62):       # h = 1/16, 1/32, 1/64
        n = (nn, nn)
        h = 1.0 / (nn + 2)            # ghost nodes i = -1 and i = n + 1 sit at x = 0 and x = 1
        k = 8.0
        X = _grid_coords(n)
        x, y = (X[0] + 1) * h, (X[1] + 1) * h
        u = np.sin(math.pi * x) * np.sin(2 * math.pi * y)
        lam = math.pi ** 2 + (2 * math.pi) ** 2
        q = (lam - k * k) * u
        H = ops.helmholtz(n, h, np.ones(len(u)), k, np.zeros(len(u)))
        uh = spla.spsolve(H.tocsc(), q.astype(np.complex128))
        errs.append(np.max(np.abs(uh - u)))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.5 < r1 < 4.5 and 3.7 < r2 < 4.3, errs
