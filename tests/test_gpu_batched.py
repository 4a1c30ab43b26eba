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
