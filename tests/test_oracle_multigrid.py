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


# ---------------------------------------------------------------- restart branch of FGMRES
@pytest.mark.parametrize("restart", [3, 4])
def test_fgmres_restart_cycles_minimise_the_residual(restart):
    """restarted FGMRES (Saad 1993): every restart cycle returns the iterate of smallest
    residual norm over x_start + span(Z) of that cycle, checked against a dense least-squares
    solve on the stored directions; cycles chain (each starts from the previous end, with the
    true residual); the Givens estimate at a cycle's end is the true residual of its iterate;
    iterations and restarts add up over the cycles."""
    prob = synth.config1(16)
    H = multigrid.from_problem(prob, nu_pre=1, nu_post=1)
    b = prob.rhs()
    trace = []
    res = fgmres.solve(H, b, tol=1e-10, restart=restart, max_iter=400, trace=trace)
    assert res.converged and res.true_rel_residual <= 1e-10
    assert len(trace) >= 3                                    # several restarts happen
    assert res.restarts == len(trace) - 1
    assert res.iterations == sum(t["k"] for t in trace) == len(res.history)
    assert all(t["k"] == restart for t in trace[:-1])
    bn = np.linalg.norm(b)
    A = H.H.toarray()
    for c, t in enumerate(trace):
        if c > 0:
            assert np.array_equal(t["x_start"], trace[c - 1]["x_end"])
        r0 = b - A @ t["x_start"]
        y, *_ = np.linalg.lstsq(A @ t["Z"], r0, rcond=None)
        x_ls = t["x_start"] + t["Z"] @ y
        step = np.linalg.norm(t["x_end"] - t["x_start"])
        # (late cycles take steps near the rounding level of x itself)
        assert np.linalg.norm(t["x_end"] - x_ls) <= 1e-8 * step + 1e-13 * np.linalg.norm(t["x_end"]), c
        true_rel = np.linalg.norm(b - A @ t["x_end"]) / bn
        assert abs(t["est"] - true_rel) <= 1e-9 * max(true_rel, 1e-12) + 1e-14, (c, t["est"], true_rel)
    # restarting changes the iterates but not the limit: same solution as restart = 20
    ref = fgmres.solve(H, b, tol=1e-10, restart=20, max_iter=400)
    assert np.linalg.norm(res.x - ref.x) <= 1e-7 * np.linalg.norm(ref.x)
    assert res.iterations > ref.iterations


# ---------------------------------------------------------------- cycle composition, eq. (2.1)
def _dense_cycle_operator(H, gamma, nu1, nu2, w):
    """M^{-1} of the 3-level cycle from a zero guess, composed from the matrix form of the
    two-grid operator (eq. (2.1)): with S_l = I - w_l D_l^{-1} A_l,
      E_2 = S_2^nu2 (I - P_2 A_3^{-1} R_2 A_2) S_2^nu1,   B_2 = (I - E_2^gamma) A_2^{-1}
      (gamma cycles on level 2 from a zero guess, each on the updated residual),
      E_1 = S_1^nu2 (I - P_1 B_2 R_1 A_1) S_1^nu1,        M^{-1} = (I - E_1) A_1^{-1}."""
    A1, A2, A3 = (a.toarray() for a in H.A)
    R1, R2 = H.R1.toarray(), H.R2.toarray()
    P1, P2 = H.P1.toarray(), H.P2.toarray()
    mp = np.linalg.matrix_power
    I1, I2 = np.eye(A1.shape[0]), np.eye(A2.shape[0])
    S1 = I1 - w[0] * (A1 / np.diag(A1)[:, None])
    S2 = I2 - w[1] * (A2 / np.diag(A2)[:, None])
    E2 = mp(S2, nu2) @ (I2 - P2 @ np.linalg.solve(A3, R2 @ A2)) @ mp(S2, nu1)
    B2 = (I2 - mp(E2, gamma)) @ np.linalg.inv(A2)
    E1 = mp(S1, nu2) @ (I1 - P1 @ B2 @ R1 @ A1) @ mp(S1, nu1)
    return (I1 - E1) @ np.linalg.inv(A1)


@pytest.mark.parametrize("n,gamma,nu", [((8, 8), 2, (1, 2)), ((8, 8), 1, (2, 1)), ((8, 8), 2, (0, 1)),
                                        ((8, 4, 8), 2, (1, 2))])
def test_cycle_equals_dense_composition_of_eq_2_1(n, gamma, nu):
    """the recursive cycle (W: two level-2 visits, the second on the updated residual) equals,
    column by column, the dense operator composed from eq. (2.1) with per-level damping weights
    (0.6, 0.4), the level-2 shift alpha2 and the real-shifted coarsest operator."""
    H = _hier(n, alpha=1.12, alpha2=1.03, beta=0.05, cycle=gamma, nu_pre=nu[0], nu_post=nu[1],
              jacobi=(0.6, 0.4))
    Md = _dense_cycle_operator(H, gamma, nu[0], nu[1], (0.6, 0.4))
    N = H.A[0].shape[0]
    cols = np.stack([H.precond(np.eye(N, dtype=np.complex128)[:, j]) for j in range(N)], 1)
    assert np.max(np.abs(cols - Md)) <= 1e-12 * np.max(np.abs(Md))
    # the composition is sensitive to what it pins: swapped weights or sweep counts differ
    assert np.max(np.abs(_dense_cycle_operator(H, gamma, nu[0], nu[1], (0.4, 0.6)) - Md)) > 1e-3 * np.max(np.abs(Md))
    if nu[0] != nu[1]:
        assert np.max(np.abs(_dense_cycle_operator(H, gamma, nu[1], nu[0], (0.6, 0.4)) - Md)) > 1e-3 * np.max(np.abs(Md))
    assert np.max(np.abs(_dense_cycle_operator(H, 3 - gamma, nu[0], nu[1], (0.6, 0.4)) - Md)) > 1e-6 * np.max(np.abs(Md))



# ---------------------------------------------------------------- the cycle as a solver
def test_stationary_iteration_matches_its_closed_form():
    """k cycles of x <- x + M^{-1}(b - H x) from zero give x_k = (I - (I - M^{-1}H)^k) H^{-1} b,
    with M^{-1} the dense composition of eq. (2.1); the residual then contracts per cycle at
    the spectral radius of I - H M^{-1}."""
    H = _hier((8, 8), alpha=1.12, alpha2=1.03, beta=0.05, cycle=2, nu_pre=1, nu_post=1, jacobi=(0.6, 0.4))
    Md = _dense_cycle_operator(H, 2, 1, 1, (0.6, 0.4))
    A = H.H.toarray()
    N = A.shape[0]
    rng = np.random.default_rng(3)
    b = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    x, its, hist = multigrid.stationary(H, b, tol=1e-300, max_iter=6)
    E = np.eye(N) - Md @ A
    xk = (np.eye(N) - np.linalg.matrix_power(E, 6)) @ np.linalg.solve(A, b)
    assert its == 6 and len(hist) == 6
    assert np.linalg.norm(x - xk) <= 1e-11 * np.linalg.norm(xk)
    rho = np.max(np.abs(np.linalg.eigvals(np.eye(N) - A @ Md)))
    x, its, hist = multigrid.stationary(H, b, tol=1e-300, max_iter=60)
    rate = (hist[-1] / hist[-11]) ** 0.1
    assert abs(rate - rho) <= 0.05 * rho, (rate, rho)


def test_stationary_stops_on_divergence_and_at_zero():
    H = _hier((16, 16), alpha=1.6, cycle=2, nu_pre=3, nu_post=3, jacobi=(1.6, 1.6))     # unstable smoother
    b = np.ones(H.H.shape[0], np.complex128)
    x, its, hist = multigrid.stationary(H, b, tol=1e-6, max_iter=500)
    assert hist[-1] > 1e8 and its < 500
    x, its, hist = multigrid.stationary(H, np.zeros_like(b))
    assert its == 0 and not np.any(x)
