"""Batched form: uneven grid sizes, several frequencies and right-hand sides per instance,
solved concurrently; every result equals the single-instance solve bit for bit and meets
the residual bound checked with the oracle's operator."""
import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu

pytest.importorskip("paper_2604_19501_amd._lib")
from paper_2604_19501_amd import from_problem  # noqa: E402
from paper_2604_19501_amd.batched import BatchedSolver, instance_dict  # noqa: E402
from oracle import operators as ops  # noqa: E402
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
