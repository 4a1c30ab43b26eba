"""helm_vcycle_noalloc: the cycle with its per-call scratch in the library's static device
array.  Through the C ABI, its result equals helm_vcycle's bit for bit (same kernels, same
launch shapes, only the scratch addresses differ), on two calls in a row, the second on a
smaller grid, and again after the first grid is used once more; a grid whose scratch
exceeds the array is refused before any device work."""
import ctypes as C

import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu

L = pytest.importorskip("paper_2604_19501_amd._lib")
from paper_2604_19501_amd import from_problem  # noqa: E402


def _cycle_both(s, r, op):
    rt = torch.from_numpy(r).cuda()
    z_ref = torch.empty_like(rt)
    z_na = torch.full_like(rt, float("nan"))
    st = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert L.lib.helm_vcycle(s.ctx, op, C.c_void_p(rt.data_ptr()), C.c_void_p(z_ref.data_ptr()), st) == 0
    assert L.lib.helm_vcycle_noalloc(s.ctx, op, C.c_void_p(rt.data_ptr()), C.c_void_p(z_na.data_ptr()), st) == 0, \
        L.lib.helm_last_error()
    torch.cuda.synchronize()
    return z_ref, z_na


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_noalloc_cycle_equals_workspace_cycle(prec):
    big = synth.config2(256)
    small = synth.config3(32)
    sb = from_problem(big, nu=(1, 1), cycle_prec=prec)
    ss = from_problem(small, nu=(1, 1), cycle_prec=prec)
    for k, (s, p) in enumerate(((sb, big), (ss, small), (sb, big))):
        r = synth.random_vector(p.N, 100 + k)
        for op in (L.HELM_OP_N, L.HELM_OP_C):
            z_ref, z_na = _cycle_both(s, r, op)
            print("call %d %s %s op %d: |z| %.3e" % (k, p.name, prec, op, float(torch.linalg.norm(z_ref))), flush=True)
            assert torch.isfinite(z_ref).all()
            assert torch.equal(z_ref, z_na), (k, op)
    sb.close()
    ss.close()


def test_noalloc_refuses_a_grid_beyond_the_array():
    p = synth.config2(1536)
    s = from_problem(p, nu=(1, 1), cycle_prec="f64")
    r = torch.zeros(p.N, dtype=torch.complex128, device="cuda")
    z = torch.zeros_like(r)
    st = L.lib.helm_vcycle_noalloc(s.ctx, 0, C.c_void_p(r.data_ptr()), C.c_void_p(z.data_ptr()), None)
    assert st == L.HELM_EINVAL
    assert b"bytes of scratch" in L.lib.helm_last_error()
    s.close()
