"""Batched form: uneven grid sizes, several frequencies and right-hand sides per instance,
solved concurrently; every result equals the single-instance solve bit for bit and meets
the residual bound checked with the oracle's operator."""
import ctypes as C

import numpy as np
import pytest
import scipy.sparse.linalg as spla
import torch

import synth

pytestmark = pytest.mark.gpu

pytest.importorskip("paper_2604_19501_amd._lib")
from paper_2604_19501_amd import from_problem  # noqa: E402
from paper_2604_19501_amd.batched import BatchedSolver, instance_dict  # noqa: E402
from oracle import fgmres, multigrid, operators as ops  # noqa: E402
from tests.gpu_helpers import rel  # noqa: E402
from paper_2604_19501_amd import _lib as L  # noqa: E402


def test_batched_matches_single():
    probs = [synth.config4_instance(i, per_size=2, sizes=(64, 96, 128), n_src=3) for i in range(6)]
    b = BatchedSolver([instance_dict(p) for p in probs], nu=(1, 1), cycle_prec="f32", max_rhs=3)
    rhs, inst = [], []
    for i, p in enumerate(probs):
        for k in range(3):
            rhs.append(p.rhs(k))
            inst.append(i)
    xs, infos = b.solve(rhs, inst, tol=1e-6, max_iter=400)
    torch.cuda.synchronize()
    for i, p in enumerate(probs):
        assert b.instance_info(i)["N1"] == p.N
        assert L.lib.helm_level_size(b.ctx, i, 1) == p.N
    for j, (x, info, i) in enumerate(zip(xs, infos, inst)):
        p = probs[i]
        assert info["status"] == 0, (j, info)
        H = ops.helmholtz(p.n, p.h, p.slowness.ravel() ** 2, p.omega, ops.layer_sigma(p.n, p.layer, p.sigma_max))
        xg = x.cpu().numpy()
        res = np.linalg.norm(rhs[j] - H @ xg) / np.linalg.norm(rhs[j])
        assert res <= 1e-6
        s = from_problem(p, nu=(1, 1), cycle_prec="f32")
        x1, i1 = s.solve(rhs[j], tol=1e-6, max_iter=400)
        assert i1["iterations"] == info["iterations"]
        assert torch.equal(x1, x)
        s.close()


@pytest.mark.parametrize("max_iter", [400, 3])
def test_lockstep_groups_with_mixed_outcomes(max_iter):
    """five right-hand sides of one instance solved in lock-step groups of at most 2: a
    zero right-hand side (x = 0 at once), point sources at different places and a scaled
    copy; with max_iter = 3 the solves stop unconverged.  Every solution, status and
    iteration count equals the single solve's."""
    p = synth.config4_instance(1, per_size=2, sizes=(64, 96, 128), n_src=3)
    b = BatchedSolver([instance_dict(p)], nu=(1, 1), cycle_prec="f32", max_rhs=2)
    q = [p.rhs(0), np.zeros_like(p.rhs(0)), p.rhs(1), 1e3 * p.rhs(2), p.rhs(2)]
    xs, infos = b.solve(q, [0] * len(q), tol=1e-6, max_iter=max_iter)
    torch.cuda.synchronize()
    s = from_problem(p, nu=(1, 1), cycle_prec="f32")
    for j in range(len(q)):
        x1, i1 = s.solve(q[j], tol=1e-6, max_iter=max_iter)
        assert (i1["status"], i1["iterations"]) == (infos[j]["status"], infos[j]["iterations"]), j
        assert torch.equal(x1, xs[j]), j
    assert infos[1]["iterations"] == 0 and not torch.any(xs[1] != 0)
    if max_iter == 3:
        assert all(i["status"] == L.HELM_ENOCONV and i["iterations"] == 3 for k, i in enumerate(infos) if k != 1)
    s.close()
    b.close()


def test_batched_instances_against_oracle():
    """one instance of each grid size of the 96-instance workload (256^2 at G = 10, 512^2 at
    G = 10 2/3, 768^2 at G = 11 1/3), two of its sources solved in one lock-step group, against
    the oracle's FGMRES on that instance: iterations +-1, true residual <= 1e-6, error against
    the exact solution (sparse LU) within 3x the oracle's."""
    probs = [synth.config4_instance(i) for i in (0, 33, 66)]
    b = BatchedSolver([instance_dict(p) for p in probs], nu=(1, 1), cycle_prec="f32", max_rhs=2)
    rhs, inst = [], []
    for i, p in enumerate(probs):
        for k in range(2):
            rhs.append(p.rhs(k))
            inst.append(i)
    xs, infos = b.solve(rhs, inst, tol=1e-6, max_iter=1000)
    torch.cuda.synchronize()
    b.close()
    for i, p in enumerate(probs):
        H = multigrid.from_problem(p, nu_pre=1, nu_post=1)
        lu = spla.splu(H.H.tocsc())
        for k in range(2):
            j = 2 * i + k
            q = rhs[j]
            ref = fgmres.solve(H, q, tol=1e-6, restart=p.restart, max_iter=1000)
            ustar = lu.solve(q)
            xg = xs[j].cpu().numpy()
            res = np.linalg.norm(q - H.H @ xg) / np.linalg.norm(q)
            e_gpu, e_orc = rel(xg, ustar), rel(ref.x, ustar)
            print("%s source %d: %d iterations (oracle %d), residual %.2e, error %.2e (oracle %.2e)"
                  % (p.name, k, infos[j]["iterations"], ref.iterations, res, e_gpu, e_orc), flush=True)
            assert infos[j]["status"] == 0 and res <= 1e-6
            assert abs(infos[j]["iterations"] - ref.iterations) <= 1
            assert e_gpu <= max(3.0 * e_orc, 1e-7)
            assert rel(xg, ref.x) <= 1e-6          # FP32 cycle: the oracle's iterate to 1e-6


def test_single_instance_calls_refuse_a_batched_context():
    """the parent context of a batch holds no hierarchy of its own: every call that works on
    one hierarchy returns HELM_EINVAL for it before any device work"""
    probs = [synth.config4_instance(i, per_size=2, sizes=(64, 96, 128), n_src=1) for i in range(2)]
    b = BatchedSolver([instance_dict(p) for p in probs], nu=(1, 1), cycle_prec="f32", max_rhs=1)
    N = probs[0].N
    x = torch.zeros(N, dtype=torch.complex128, device="cuda")
    y = torch.zeros_like(x)
    g = torch.zeros(N, dtype=torch.float64, device="cuda")
    kap = torch.ones(N, dtype=torch.float64, device="cuda")
    xp, yp = C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr())
    sh = L.Shift(1.1, 1.0, 0.0)
    arr = (C.c_void_p * 1)(x.data_ptr())
    out = (C.c_double * (27 * N))()
    v = (C.c_longlong * 21)()
    calls = {
        "apply": L.lib.helm_apply(b.ctx, 0, 0, xp, yp, None),
        "vcycle": L.lib.helm_vcycle(b.ctx, 0, xp, yp, None),
        "coarse_solve": L.lib.helm_coarse_solve(b.ctx, 0, xp, yp, None),
        "solve": L.lib.helm_solve(b.ctx, 0, xp, yp, 1e-6, 10, None, None),
        "grad_m": L.lib.helm_grad_m(b.ctx, 1, arr, arr, C.c_void_p(g.data_ptr()), 0, None),
        "refactor": L.lib.helm_refactor(b.ctx, C.c_void_p(kap.data_ptr()), 10.0, C.byref(sh), None),
        "refactor_m": L.lib.helm_refactor_m(b.ctx, C.c_void_p(kap.data_ptr()), 10.0, C.byref(sh), None),
        "get_coefficients": L.lib.helm_get_coefficients(b.ctx, 2, out),
        "get_info": L.lib.helm_get_info(b.ctx, v, 21),
    }
    assert all(st == L.HELM_EINVAL for st in calls.values()), calls
    torch.cuda.synchronize()
    assert torch.count_nonzero(y).item() == 0 and torch.count_nonzero(g).item() == 0
    # the batch itself still works
    xs, infos = b.solve([probs[0].rhs(0), probs[1].rhs(0)], [0, 1], tol=1e-6, max_iter=400)
    assert all(i["status"] == 0 for i in infos)
    b.close()
