"""Pins of the oracle's adjoint and gradient.

* dot test <H x, y> = <x, H^H y> and <H^{-1} a, b> = <a, H^{-H} b> (H complex symmetric);
* the misfit gradient w.r.t. squared slowness against central finite differences.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import synth
from oracle import gradient, operators as ops


def _small(dim):
    if dim == 2:
        n = (16, 16)
    else:
        n = (8, 8, 8)
    N = int(np.prod([k + 1 for k in n]))
    rng = np.random.default_rng(21)
    m = rng.uniform(0.3, 1.0, N)
    layer = tuple((2, 2) for _ in n)
    return n, 1.0 / n[0], m, 12.0, layer, 2.0


@pytest.mark.parametrize("dim", [2, 3])
def test_adjoint_dot(dim):
    n, h, m, omega, layer, smax = _small(dim)
    sigma = ops.layer_sigma(n, layer, smax)
    H = ops.helmholtz(n, h, m, omega, sigma)
    rng = np.random.default_rng(1)
    N = H.shape[0]
    x = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    y = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    HH = H.conjugate().T
    assert abs(np.vdot(H @ x, y) - np.vdot(x, HH @ y)) <= 1e-13 * abs(np.vdot(H @ x, y))
    assert abs(HH - H.conjugate()).max() == 0
    lu, luH = spla.splu(H.tocsc()), spla.splu(H.conjugate().tocsc())
    assert abs(np.vdot(lu.solve(x), y) - np.vdot(x, luH.solve(y))) <= 1e-10 * abs(np.vdot(lu.solve(x), y))


@pytest.mark.parametrize("dim", [2, 3])
def test_gradient_finite_differences(dim):
    n, h, m, omega, layer, smax = _small(dim)
    N = len(m)
    rng = np.random.default_rng(3)
    S = 3
    Q = np.zeros((N, S), np.complex128)
    for s in range(S):
        Q[rng.integers(0, N), s] = 1.0
    rec = np.sort(rng.choice(N, size=N // 5, replace=False))
    m_ref = m * (1 + 0.1 * rng.standard_normal(N))
    D = gradient.forward_exact(n, h, m_ref, omega, layer, smax, Q)[rec, :]
    L, g = gradient.gradient_exact(n, h, m, omega, layer, smax, Q, rec, D)
    eps = 1e-4
    for k in range(4):
        v = rng.uniform(-1, 1, N)
        v /= np.abs(v).max()
        Lp = gradient.misfit(gradient.forward_exact(n, h, m + eps * v, omega, layer, smax, Q), rec, D)
        Lm = gradient.misfit(gradient.forward_exact(n, h, m - eps * v, omega, layer, smax, Q), rec, D)
        fd = (Lp - Lm) / (2 * eps)
        assert g @ v == pytest.approx(fd, rel=1e-6)
