"""Pins of the oracle's cycle and Krylov solver.

* Galerkin projection property of an exact coarse-grid correction (eq. (2.1), (2.2)):
  R (b - A (x + P A_c^{-1} R (b - A x))) = 0 when A_c = R A P, and the coarse-grid
  correction operator is idempotent;
* the cycle is invariant to rescaling R and P (Galerkin operators, Jacobi D^{-1},
  exact coarsest solve);
* k = 0 (Poisson): the W cycle as a stand-alone solver converges at a textbook rate;
* FGMRES reaches the dense direct solution on small grids and its estimated
  residual matches the true residual.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import synth
from oracle import fgmres, multigrid, operators as ops


def _hier(n=(16, 16), **kw):
    N = int(np.prod([k + 1 for k in n]))
    rng = np.random.default_rng(11)
    m = rng.uniform(0.3, 1.0, N)
    layer = tuple((2, 2) for _ in n)
    args = dict(alpha=1.0, beta=0.0, cycle=2, nu_pre=1, nu_post=1, jacobi=(0.8, 0.8))
    args.update(kw)
    return multigrid.Hierarchy(n, 1.0 / n[0], m, 18.0, layer, 2.0, **args)


@pytest.mark.parametrize("n", [(16, 16), (8, 8, 8)])
def test_coarse_correction_is_galerkin_projection(n):
    H = _hier(n, nu_pre=0, nu_post=0, cycle=1)
    rng = np.random.default_rng(2)
    N2 = H.A[1].shape[0]
    b = rng.standard_normal(N2) + 1j * rng.standard_normal(N2)
    # level-2 cycle without smoothing = P2 A3^{-1} R2 b
    x = H.cycle(1, b)
    r = H.R2 @ (b - H.A[1] @ x)
    assert np.linalg.norm(r) <= 1e-11 * np.linalg.norm(H.R2 @ b)
    # idempotence of the fine coarse-grid correction with an exact level-2 solve
    A = H.A[0].toarray()
    R, P = H.R1.toarray(), H.P1.toarray()
    Ac = R @ A @ P
    C = np.eye(A.shape[0]) - P @ np.linalg.solve(Ac, R @ A)
    assert np.allclose(C @ C, C, atol=1e-9)


def test_real_shifted_coarsest_is_not_projection_but_shifted_one():
    """with alpha != 1 the coarsest operator is the Galerkin image of the shifted
    operator (eq. (3.6)), so the projection property holds for that one instead."""
    H = _hier(nu_pre=0, nu_post=0, cycle=1, alpha=1.12)
    rng = np.random.default_rng(4)
    N2 = H.A[1].shape[0]
    b = rng.standard_normal(N2) + 1j * rng.standard_normal(N2)
    x = H.cycle(1, b)
    A2a = H.R1 @ ops.helmholtz(H.n1, H.h, H.m, H.omega, H.sigma, alpha=1.12) @ H.P1
    assert np.linalg.norm(H.R2 @ (b - A2a @ x)) <= 1e-11 * np.linalg.norm(H.R2 @ b)
    assert np.linalg.norm(H.R2 @ (b - H.A[1] @ x)) > 1e-3 * np.linalg.norm(H.R2 @ b)


def test_transfer_scaling_invariance():
    rng = np.random.default_rng(6)
    a = _hier(alpha=1.1, beta=0.03)
    b = _hier(alpha=1.1, beta=0.03, r_scale=2.0, p_scale=0.25)
    v = rng.standard_normal(a.A[0].shape[0]) + 1j * rng.standard_normal(a.A[0].shape[0])
    za, zb = a.precond(v), b.precond(v)
    assert np.linalg.norm(za - zb) <= 1e-12 * np.linalg.norm(za)


@pytest.mark.parametrize("n", [(32, 32), (16, 16, 16)])
def test_poisson_w_cycle_rate(n):
    N = int(np.prod([k + 1 for k in n]))
    H = multigrid.Hierarchy(n, 1.0 / n[0], np.ones(N), 0.0, tuple((0, 0) for _ in n), 0.0,
                            cycle=2, nu_pre=2, nu_post=2, jacobi=(0.8, 0.8))
    rng = np.random.default_rng(0)
    b = rng.standard_normal(N).astype(np.complex128)
    x = np.zeros(N, np.complex128)
    res = [np.linalg.norm(b)]
    for _ in range(8):
        x = x + H.precond(b - H.H @ x)
        res.append(np.linalg.norm(b - H.H @ x))
    rate = (res[-1] / res[2]) ** (1.0 / 6)
    assert rate < 0.3, rate


@pytest.mark.parametrize("n", [(16, 16), (8, 8, 8)])
def test_fgmres_matches_direct(n):
    prob = synth.config1(n[0]) if len(n) == 2 else None
    if prob is None:
        p3 = synth.config3(8)
        prob = p3
    H = multigrid.from_problem(prob, nu_pre=1, nu_post=1)
    b = prob.rhs()
    u = spla.spsolve(H.H.tocsc(), b)
    res = fgmres.solve(H, b, tol=1e-10, restart=20, max_iter=200)
    assert res.converged
    assert res.true_rel_residual <= 1e-10 * 1.01
    assert np.linalg.norm(res.x - u) / np.linalg.norm(u) < 1e-7
    # the Givens estimate is the true residual of the iterate (up to rounding)
    assert abs(res.history[-1] - res.true_rel_residual) < 1e-11


def test_fgmres_identity_preconditioner_is_gmres():
    """with M = I and no restart, FGMRES on an N x N system is exact after N steps."""
    rng = np.random.default_rng(7)
    N = 12
    A = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N)) + 5 * np.eye(N)
    b = rng.standard_normal(N) + 0j
    r = fgmres.fgmres(lambda v: A @ v, lambda v: v, b, tol=1e-14, restart=N, max_iter=N)
    assert np.linalg.norm(A @ r.x - b) / np.linalg.norm(b) < 1e-12
    # monotone residual estimates
    assert all(r.history[i + 1] <= r.history[i] * (1 + 1e-12) for i in range(len(r.history) - 1))


def test_fgmres_zero_rhs():
    H = _hier()
    r = fgmres.solve(H, np.zeros(H.H.shape[0], np.complex128))
    assert r.iterations == 0 and r.converged and np.all(r.x == 0)
