"""Adjoint solve and misfit gradient w.r.t. squared slowness on the GPU.

* against the oracle's gradient (forward and adjoint by sparse LU, data from the
  oracle's forward solve on a reference medium): relative L2 difference <= 1e-5
  with GPU solves at tol 1e-10;
* against central finite differences of the GPU loss (step 1e-4, 20 seeded
  directions with max |v| = 1): relative agreement <= 1e-5;
* the full-size 128^3 workload (16 sources on the top face, receivers on the whole
  top face, zero data, the sources solved in lock-step): finite-difference agreement on
  20 seeded directions;
* a solver refactored for another medium between a loss and its backward pass gives the
  gradient of the medium the loss was evaluated at;
* lock-step source solves give the separate solves' loss and gradient bit for bit.
"""
import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu

pytest.importorskip("paper_2604_19501_amd._lib")
from paper_2604_19501_amd import from_problem  # noqa: E402
from paper_2604_19501_amd.autograd import helmholtz_misfit  # noqa: E402
from oracle import gradient as og  # noqa: E402


def _setup(dim, n, nsrc, seed=5):
    p = synth.config3(n, seed=seed) if dim == 3 else synth.config2(n, seed=seed)
    rng = np.random.default_rng(seed)
    N = p.N
    m_ref = p.slowness.ravel() ** 2
    m0 = m_ref * (1.0 + 0.05 * rng.uniform(-1, 1, N))
    Q = np.zeros((N, nsrc), np.complex128)
    for s in range(nsrc):
        Q[rng.integers(0, N), s] = 1.0
    rec = np.sort(rng.choice(N, size=max(8, N // 10), replace=False))
    return p, m_ref, m0, Q, rec


@pytest.mark.parametrize("dim,n", [(2, 32), (3, 16)])
def test_gradient_matches_oracle(dim, n):
    p, m_ref, m0, Q, rec = _setup(dim, n, 3)
    D = og.forward_exact(p.n, p.h, m_ref, p.omega, p.layer, p.sigma_max, Q)[rec, :]
    L_ref, g_ref = og.gradient_exact(p.n, p.h, m0, p.omega, p.layer, p.sigma_max, Q, rec, D)
    s = from_problem(p, cycle_prec="f32")
    m = torch.tensor(m0, dtype=torch.float64, device="cuda", requires_grad=True)
    src = [torch.from_numpy(Q[:, k]).cuda() for k in range(Q.shape[1])]
    data = [torch.from_numpy(D[:, k]).cuda() for k in range(D.shape[1])]
    recs = torch.from_numpy(rec).cuda()
    loss = helmholtz_misfit(m, s, src, recs, data, tol=1e-10)
    loss.backward()
    g = m.grad.cpu().numpy()
    assert abs(loss.item() - L_ref) <= 1e-7 * L_ref
    assert np.linalg.norm(g - g_ref) <= 1e-5 * np.linalg.norm(g_ref)


def _fd_check(p, m0, src, recs, data, ndir, seed, tol_rel=1e-5, max_rhs=1):
    s = from_problem(p, cycle_prec="f32", max_rhs=max_rhs)
    m = torch.tensor(m0, dtype=torch.float64, device="cuda", requires_grad=True)
    loss = helmholtz_misfit(m, s, src, recs, data, tol=1e-10)
    loss.backward()
    g = m.grad.detach().clone()
    rng = np.random.default_rng(seed)
    eps = 1e-4
    worst = 0.0
    for k in range(ndir):
        v = torch.from_numpy(rng.uniform(-1, 1, p.N)).cuda()
        v /= v.abs().max()
        with torch.no_grad():
            lp = helmholtz_misfit(m.detach() + eps * v, s, src, recs, data, tol=1e-10).item()
            lm = helmholtz_misfit(m.detach() - eps * v, s, src, recs, data, tol=1e-10).item()
        fd = (lp - lm) / (2 * eps)
        an = float(torch.dot(g, v))
        err = abs(fd - an) / max(abs(an), 1e-300)
        worst = max(worst, err)
        assert err <= tol_rel, (k, fd, an, err)
    return worst


def test_gradient_finite_differences_20_directions():
    p, m_ref, m0, Q, rec = _setup(2, 64, 2, seed=9)
    D = np.zeros((len(rec), 2), np.complex128)            # zero data: L = 1/2 sum ||P u_s||^2
    src = [torch.from_numpy(Q[:, k]).cuda() for k in range(2)]
    data = [torch.from_numpy(D[:, k]).cuda() for k in range(2)]
    w = _fd_check(p, m0, src, torch.from_numpy(rec).cuda(), data, 20, 11)
    print("worst relative FD mismatch over 20 directions: %.2e" % w)


def test_gradient_full_size_workload():
    """128^3, 16 sources on a 4x4 lattice of the top face, receivers on every top-face node."""
    p, m_ref, rec = synth.config5(128)
    m0 = p.slowness.ravel() ** 2
    src = [torch.from_numpy(synth.point_rhs(p.n, pos)).cuda() for pos in p.sources]
    data = [torch.zeros(len(rec), dtype=torch.complex128, device="cuda") for _ in p.sources]
    w = _fd_check(p, m0, src, torch.from_numpy(rec).cuda(), data, 20, 13, max_rhs=16)
    print("worst relative FD mismatch at 128^3 (lock-step sources): %.2e" % w)


def test_lockstep_misfit_equals_separate_solves():
    """a solver with room for 4 right-hand sides in lock-step (max_rhs = 4, groups of 4 and
    of 1 for 5 sources) gives the same loss and gradient, bit for bit, as separate solves"""
    p, m_ref, m0, Q, rec = _setup(3, 16, 5, seed=21)
    D = 0.5 * np.ones((len(rec), 5), np.complex128)
    src = [torch.from_numpy(Q[:, k]).cuda() for k in range(5)]
    data = [torch.from_numpy(D[:, k]).cuda() for k in range(5)]
    recs = torch.from_numpy(rec).cuda()
    out = []
    for mr in (1, 4):
        s = from_problem(p, cycle_prec="f32", max_rhs=mr)
        m = torch.tensor(m0, dtype=torch.float64, device="cuda", requires_grad=True)
        loss = helmholtz_misfit(m, s, src, recs, data, tol=1e-10)
        loss.backward()
        out.append((loss.detach().clone(), m.grad.detach().clone()))
        s.close()
    assert torch.equal(out[0][0], out[1][0])
    assert torch.equal(out[0][1], out[1][1])


def test_backward_after_the_solver_moved_to_another_medium():
    """two losses evaluated with one solver at different media, then backward on the first:
    the gradient equals (bit for bit) the one of a fresh solver at the first medium"""
    p, m_ref, m0, Q, rec = _setup(2, 32, 2, seed=17)
    D = np.zeros((len(rec), 2), np.complex128)
    src = [torch.from_numpy(Q[:, k]).cuda() for k in range(2)]
    data = [torch.from_numpy(D[:, k]).cuda() for k in range(2)]
    recs = torch.from_numpy(rec).cuda()
    s = from_problem(p, cycle_prec="f32")
    m1 = torch.tensor(m0, dtype=torch.float64, device="cuda", requires_grad=True)
    m2 = torch.tensor(m_ref, dtype=torch.float64, device="cuda", requires_grad=True)
    l1 = helmholtz_misfit(m1, s, src, recs, data, tol=1e-10)
    l2 = helmholtz_misfit(m2, s, src, recs, data, tol=1e-10)
    l1.backward()
    s2 = from_problem(p, cycle_prec="f32")
    m1b = torch.tensor(m0, dtype=torch.float64, device="cuda", requires_grad=True)
    l1b = helmholtz_misfit(m1b, s2, src, recs, data, tol=1e-10)
    l1b.backward()
    assert torch.equal(l1.detach(), l1b.detach())
    assert torch.equal(m1.grad, m1b.grad)
    l2.backward()                        # and back again for the second medium
    s2.refactor(m=torch.tensor(m_ref, dtype=torch.float64, device="cuda"))
    m2b = torch.tensor(m_ref, dtype=torch.float64, device="cuda", requires_grad=True)
    l2b = helmholtz_misfit(m2b, s2, src, recs, data, tol=1e-10)
    l2b.backward()
    assert torch.equal(m2.grad, m2b.grad)
    s.close()
    s2.close()
