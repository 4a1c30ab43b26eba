"""GPU-vs-oracle parity at the workloads' full sizes, through the C ABI.

* 2D 1024^2 layered workload (the benchmarked solve: about 170 iterations, eight
  restarts): FP64 and FP32 cycles against the oracle's FGMRES at tol 1e-6 (iterations
  +-1, true FP64 residual, relative difference to the oracle's solution within 1e-10
  (FP64 cycle) or 1e-6 (FP32 cycle) in norm and element by element, error against the
  exact solution of a sparse LU of H), and at tol 1e-10, where the solution must be
  within 1e-6 of the exact one in norm and element by element;
* 3D 128^3 with the 256^3 workload's recipe: the same checks, with the oracle's FGMRES
  solve carried on to tol 1e-12 as the reference solution (a sparse LU of the 3D fine
  operator does not fit);
* the 256^3 workload's coarsest level (65^3 unknowns, the large-front factorisation
  paths): the residual of the library's exact solve against the oracle's assembled
  real-shifted Galerkin operator (eq. (3.6)).

Tolerance derivation (stated with the design notes):
* two iterates that both meet ||b - Hx|| <= tol ||b|| differ from the exact solution
  u* by at most ||H^-1|| tol ||b||; for these media ||H^-1|| ||b|| / ||u*|| is measured
  at 20-200, so at tol 1e-6 the error against u* is bounded by 2e-4 for any method, and
  the GPU's error must stay within 3x the oracle's own (same Krylov method, same
  stopping rule) or 1e-7, whichever is larger;
* at tol 1e-10 the same argument bounds the error by 2e-8; the benchmark spec's bound of 1e-6
  is asserted, in the 2-norm and element-wise (max |x - u*| <= 1e-6 max |u*|).
"""
import time

import numpy as np
import pytest
import scipy.sparse.linalg as spla
import torch

import synth
from tests.gpu_helpers import maxabs_rel, oracle_hierarchy, rel

pytestmark = pytest.mark.gpu

L = pytest.importorskip("paper_2604_19501_amd._lib")
from paper_2604_19501_amd import from_problem  # noqa: E402
from oracle import fgmres, operators as ops  # noqa: E402


# relative difference to the oracle's FGMRES solution at the same tolerance, in the 2-norm
# and element-wise: the FP64 cycle computes the oracle's iterates up to rounding (measured
# 2e-15 at 1024^2 after eight restarts); the FP32 cycle perturbs each preconditioned
# direction by about 1e-7 relative, and FGMRES (which keeps the directions it used) carries
# that into the solution only through the least-squares weights (measured 4e-9 at 1024^2,
# 1e-11 at 128^3), so the benchmark spec's bound 1e-6 holds with a wide margin
DIFF = {"f64": 1e-10, "f32": 1e-6}


def _true_rel(H, q, x):
    return float(np.linalg.norm(q - H @ x) / np.linalg.norm(q))


def _gpu_solve(p, prec, tol):
    s = from_problem(p, nu=(p.nu_pre, p.nu_post), cycle_prec=prec)
    x, info = s.solve(p.rhs(), tol=tol, max_iter=3000)
    xg = x.cpu().numpy()
    s.close()
    torch.cuda.empty_cache()
    return xg, info


def _check_solves(p, H, ref6, ustar, label):
    q = p.rhs()
    e_orc = rel(ref6.x, ustar)
    print("%s oracle: %d iterations, %d restarts, error vs reference %.2e" % (label, ref6.iterations, ref6.restarts,
                                                                                 e_orc), flush=True)
    for prec in ("f64", "f32"):
        x6, i6 = _gpu_solve(p, prec, 1e-6)
        r6 = _true_rel(H.H, q, x6)
        e6 = rel(x6, ustar)
        print("%s %s tol 1e-6: %d iterations (oracle %d), true residual %.3e, error %.2e, diff to oracle %.2e"
              % (label, prec, i6["iterations"], ref6.iterations, r6, e6, rel(x6, ref6.x)), flush=True)
        assert i6["status"] == 0
        assert abs(i6["iterations"] - ref6.iterations) <= 1, (prec, i6["iterations"], ref6.iterations)
        assert r6 <= 1e-6
        assert e6 <= max(3.0 * e_orc, 1e-7), (prec, e6, e_orc)
        # the same iterate as the oracle's: same Krylov method, same stopping point
        d6, dm6 = rel(x6, ref6.x), maxabs_rel(x6, ref6.x)
        assert d6 <= DIFF[prec] and dm6 <= DIFF[prec], (prec, d6, dm6)
        x10, i10 = _gpu_solve(p, prec, 1e-10)
        r10 = _true_rel(H.H, q, x10)
        e10, m10 = rel(x10, ustar), maxabs_rel(x10, ustar)
        print("%s %s tol 1e-10: %d iterations, true residual %.3e, error %.2e (element-wise %.2e)"
              % (label, prec, i10["iterations"], r10, e10, m10), flush=True)
        assert i10["status"] == 0 and r10 <= 1e-10
        assert e10 <= 1e-6 and m10 <= 1e-6, (prec, e10, m10)


def test_solve_2d_1024_layered_against_oracle():
    p = synth.config2(1024)
    t0 = time.perf_counter()
    H = oracle_hierarchy(p, nu_pre=1, nu_post=1)
    ustar = spla.splu(H.H.tocsc()).solve(p.rhs())
    ref6 = fgmres.solve(H, p.rhs(), tol=1e-6, restart=p.restart, max_iter=2000)
    print("oracle 1024^2: %.1f s" % (time.perf_counter() - t0), flush=True)
    assert ref6.restarts >= 5           # the restart path is exercised
    _check_solves(p, H, ref6, ustar, "1024^2")


def test_solve_3d_128_layered_against_oracle():
    p = synth.config3(128)
    t0 = time.perf_counter()
    H = oracle_hierarchy(p, nu_pre=1, nu_post=1)
    ref6 = fgmres.solve(H, p.rhs(), tol=1e-6, restart=p.restart, max_iter=2000)
    ref12 = fgmres.solve(H, p.rhs(), tol=1e-12, restart=p.restart, max_iter=2000, x0=ref6.x)
    print("oracle 128^3: %.1f s (%d + %d iterations)" % (time.perf_counter() - t0, ref6.iterations,
                                                           ref12.iterations), flush=True)
    assert ref12.converged
    _check_solves(p, H, ref6, ref12.x, "128^3")


def _coarsest_operator(p):
    """the oracle's R2 (R1 H_beta^alpha P1) P2 (eq. (3.6)) without a factorisation"""
    n = p.n
    sig = ops.layer_sigma(n, p.layer, p.sigma_max)
    A = ops.helmholtz(n, p.h, p.slowness.ravel() ** 2, p.omega, sig, beta=p.beta, alpha=p.alpha)
    n2 = ops.coarse(n)
    A2 = ops.galerkin(ops.restriction(n), A, ops.prolongation(n))
    del A
    return ops.galerkin(ops.restriction(n2), A2, ops.prolongation(n2))


def test_coarse_solve_3d_256_against_oracle_operator():
    """e = A3^-1 r by the library's factors at 65^3 unknowns: ||A3 e - r|| / ||r|| with the
    oracle's assembled A3 (FP64 factors: backward-stable elimination, bound 1e-10; FP32
    factors and substitution: entries rounded to 6e-8 relative and O(100)-deep sums, bound
    1e-4).  Conjugate operator likewise."""
    p = synth.config3(256)
    t0 = time.perf_counter()
    A3 = _coarsest_operator(p)
    print("oracle A3 at 65^3: %.1f s, %d nonzeros" % (time.perf_counter() - t0, A3.nnz), flush=True)
    rng = np.random.default_rng(31)
    r = rng.standard_normal(A3.shape[0]) + 1j * rng.standard_normal(A3.shape[0])
    for prec, tol in (("f32", 1e-4), ("f64", 1e-10)):
        s = from_problem(p, nu=(1, 1), cycle_prec=prec)
        assert s.level_size(3) == A3.shape[0]
        e = s.coarse_solve(r).cpu().numpy()
        res = np.linalg.norm(A3 @ e - r) / np.linalg.norm(r)
        ec = s.coarse_solve(r, op=L.HELM_OP_C).cpu().numpy()
        resc = np.linalg.norm(A3.conjugate() @ ec - r) / np.linalg.norm(r)
        print("256^3 coarsest %s: residual %.2e, conjugate %.2e" % (prec, res, resc), flush=True)
        assert res <= tol and resc <= tol, (prec, res, resc)
        s.close()
        torch.cuda.empty_cache()
