"""Batched form: many media / frequencies / grid sizes and many right-hand sides.

    b = BatchedSolver([dict(n=(256, 256), h=1/256, slowness=k0, omega=w0, layer=..., sigma_max=2.0,
                            alpha=1.117, alpha2=1.0, beta=0.0), ...], nu=(1, 1), cycle_prec="f32")
    xs, infos = b.solve(rhs_list, inst_of_rhs)

All instances share one workspace; helm_solve_batched runs the instances
concurrently on library streams with their captured per-iteration graphs.
"""
from __future__ import annotations

import ctypes as C
from typing import List, Sequence

import numpy as np
import torch

from . import _lib as L
from .solver import INFO_LEN, _dev_tensor, _stream_ptr, kernel_times, make_grid, make_mg, parse_info


class BatchedSolver:
    def __init__(self, instances: Sequence[dict], cycle=2, nu=(1, 1), jacobi=0.8, cycle_prec="f32", restart=20,
                 max_rhs=8, device="cuda:0"):
        self.device = torch.device(device)
        self.ninst = len(instances)
        self.grids = (L.Grid * self.ninst)(*[make_grid(d["n"], d["h"], d["layer"], d["sigma_max"]) for d in instances])
        self.mg = make_mg(cycle, nu, jacobi, cycle_prec, restart)
        self.N = [int(np.prod([k + 1 for k in d["n"]])) for d in instances]
        b = C.c_size_t()
        L.check(L.lib.helm_workspace_bytes_batched(self.ninst, self.grids, C.byref(self.mg), int(max_rhs), C.byref(b)),
                "helm_workspace_bytes_batched")
        self.ws_bytes = int(b.value)
        self.ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
        self._ws_ptr = (self.ws.data_ptr() + 255) // 256 * 256
        kaps = [_dev_tensor(d["slowness"], torch.float64, self.device) for d in instances]
        self._kaps = kaps
        kp = (C.c_void_p * self.ninst)(*[k.data_ptr() for k in kaps])
        om = (C.c_double * self.ninst)(*[float(d["omega"]) for d in instances])
        sh = (L.Shift * self.ninst)(*[L.Shift(float(d.get("alpha", 1.0)), float(d.get("alpha2", 1.0)),
                                                float(d.get("beta", 0.0))) for d in instances])
        ctx = C.c_void_p()
        L.check(L.lib.helm_setup_batched(self.ninst, self.grids, kp, om, sh, C.byref(self.mg), int(max_rhs),
                                         C.c_void_p(self._ws_ptr), self.ws_bytes,
                                         C.c_void_p(_stream_ptr(self.device)), C.byref(ctx)), "helm_setup_batched")
        self.ctx = ctx

    def solve(self, rhs: Sequence, inst_of_rhs: Sequence[int], tol=1e-6, max_iter=1000, op=L.HELM_OP_N):
        n = len(rhs)
        bs = [_dev_tensor(r, torch.complex128, self.device) for r in rhs]
        xs = [torch.zeros_like(b) for b in bs]
        rp = (C.c_void_p * n)(*[b.data_ptr() for b in bs])
        xp = (C.c_void_p * n)(*[x.data_ptr() for x in xs])
        ii = (C.c_int * n)(*[int(i) for i in inst_of_rhs])
        infos = (L.SolveInfo * n)()
        st = L.lib.helm_solve_batched(self.ctx, op, n, ii, rp, xp, float(tol), int(max_iter), infos,
                                      C.c_void_p(_stream_ptr(self.device)))
        L.check(st, "helm_solve_batched")
        out = [dict(status=infos[k].status, iterations=infos[k].iterations,
                    true_rel_residual=infos[k].true_rel_residual) for k in range(n)]
        return xs, out

    def instance_info(self, inst: int) -> dict:
        """sizes of instance inst (helm_get_info's fields)"""
        v = (C.c_longlong * INFO_LEN)()
        L.check(L.lib.helm_get_instance_info(self.ctx, int(inst), v, INFO_LEN), "helm_get_instance_info")
        return parse_info(v)

    def set_timing(self, on: bool = True):
        """per-kernel-class HIP-event timing on every instance (graphs are bypassed meanwhile)"""
        L.check(L.lib.helm_set_timing(self.ctx, 1 if on else 0), "helm_set_timing")

    def kernel_times(self) -> dict:
        """{class: (ms, launches)} summed over the instances since set_timing(True)"""
        return kernel_times(self.ctx)

    def close(self):
        if getattr(self, "ctx", None):
            L.lib.helm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def instance_dict(prob) -> dict:
    return dict(n=prob.n, h=prob.h, slowness=prob.slowness, omega=prob.omega, layer=prob.layer,
                sigma_max=prob.sigma_max, alpha=prob.alpha, alpha2=getattr(prob, "alpha2", 1.0), beta=prob.beta)
