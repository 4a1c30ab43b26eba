"""Python face of libhelm: device memory and streams from PyTorch, every step in the HIP library.

    s = Solver(n=(1024, 1024), h=1/1024, slowness=kappa, omega=w, layer=((20, 20), (20, 20)),
               sigma_max=2.0, alpha=1.1445, alpha2=1.036, beta=0.03, nu=(1, 1), jacobi=0.8,
               cycle_prec="f32", restart=20)
    x, info = s.solve(q)          # q: complex128 tensor (or numpy) of N1 entries, x: complex128 cuda tensor

The solve is FGMRES(restart) on H = -Lap_h - omega^2 kappa^2 (1 - i sigma) (eq. (1.1)
with an absorbing layer), right-preconditioned by a 3-level cycle whose coarsest
operator is the real-shifted Galerkin operator of eq. (3.6).
"""
from __future__ import annotations

import ctypes as C
from typing import Optional, Sequence, Tuple

import numpy as np
import torch

from . import _lib as L


INFO_KEYS = ("N1", "N2", "N3", "fronts", "L_entries", "W_entries", "upd_entries", "sep_entries",
             "fwd_launches", "bwd_launches", "workspace_bytes", "max_front", "cycle_complex_bytes",
             "nd_leaf", "nd_root", "nd_tuned", "nd_tree_launches")
INFO_LEN = 29
KERNEL_CLASSES = ("l1_sweep", "l1_restrict", "l2_sweep", "l2_restrict", "nd_fwd", "nd_bwd", "arnoldi", "l2_chain",
                  "cycle_tail")
# their indices among the library's timing classes (helm_get_timing)
_CLASS_INDEX = {"l1_sweep": 0, "l1_restrict": 1, "l2_sweep": 2, "l2_restrict": 3, "nd_fwd": 4, "nd_bwd": 5,
                "arnoldi": 6, "l2_chain": 10, "cycle_tail": 11}


def parse_info(v) -> dict:
    """the INFO_LEN integers of helm_get_info as a dict"""
    out = {k: int(v[i]) for i, k in enumerate(INFO_KEYS)}
    out["nd_cuts"] = [int(v[17 + i]) for i in range(min(4, out["nd_tree_launches"]))]
    out["nd_merge"] = [h for h in range(63) if (int(v[21]) >> h) & 1]
    out["planes2"], out["planes3"] = int(v[22]), int(v[23])
    out["coarse_complex_bytes"] = int(v[24])
    out["boxes"] = [int(v[25 + i]) for i in range(4)]
    return out


def kernel_times(ctx) -> dict:
    """{class: (ms, launches)} accumulated since helm_set_timing(ctx, 1)"""
    t = (C.c_double * 29)()
    L.lib.helm_get_timing(ctx, t, 29)
    return {k: (t[5 + 2 * _CLASS_INDEX[k]], int(t[6 + 2 * _CLASS_INDEX[k]])) for k in KERNEL_CLASSES}


def _stream_ptr(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _dev_tensor(a, dtype, device) -> torch.Tensor:
    if isinstance(a, torch.Tensor):
        t = a.to(device=device, dtype=dtype)
    else:
        t = torch.from_numpy(np.ascontiguousarray(np.asarray(a).ravel())).to(device=device, dtype=dtype)
    return t.contiguous().reshape(-1)


def make_grid(n: Sequence[int], h: float, layer, sigma_max: float) -> L.Grid:
    g = L.Grid()
    g.dim = len(n)
    for a in range(3):
        g.n[a] = int(n[a]) if a < len(n) else 0
        for s in range(2):
            g.layer[a][s] = int(layer[a][s]) if a < len(n) else 0
    g.h = float(h)
    g.sigma_max = float(sigma_max)
    return g


STACKS = {"p5": L.HELM_STACK_P5, "compact": L.HELM_STACK_COMPACT}
TRANSFERS = {None: 0, "fw": 0, "cubic": L.HELM_TRANSFER_CUBIC, "levdep": L.HELM_TRANSFER_LEVDEP}


def make_mg(cycle: int = 2, nu=(1, 1), jacobi=0.8, cycle_prec: str = "f32", restart: int = 20,
            stack: str = "p5", transfer=None) -> L.MG:
    """stack 'p5' (5/7-point operator, full weighting, linear interpolation) or 'compact'
    (the compact fourth-order operator of eqs. (3.1)/(3.2) with transfer 'cubic', eq. (3.3),
    or 'levdep', eq. (3.4))"""
    m = L.MG()
    m.cycle = int(cycle)
    m.nu_pre, m.nu_post = int(nu[0]), int(nu[1])
    jw = (jacobi, jacobi) if np.ndim(jacobi) == 0 else tuple(jacobi)
    m.jacobi[0], m.jacobi[1] = float(jw[0]), float(jw[1])
    m.cycle_prec = L.HELM_F32 if cycle_prec in ("f32", "fp32", L.HELM_F32) else L.HELM_F64
    m.restart = int(restart)
    m.stack = STACKS[stack]
    m.transfer = TRANSFERS[transfer if stack == "compact" else None]
    return m


def workspace_bytes(n, h, layer, sigma_max, **mg_kw) -> int:
    b = C.c_size_t()
    g = make_grid(n, h, layer, sigma_max)
    m = make_mg(**mg_kw)
    L.check(L.lib.helm_workspace_bytes(C.byref(g), C.byref(m), C.byref(b)), "helm_workspace_bytes")
    return int(b.value)


class Solver:
    """one medium / frequency: owns the workspace tensor and the library context.  With
    max_rhs > 1 the context can also solve up to max_rhs right-hand sides in lock-step
    (solve_many)."""

    def __init__(self, n, h, slowness, omega, layer, sigma_max, alpha=1.0, alpha2=1.0, beta=0.0, cycle=2,
                 nu=(1, 1), jacobi=0.8, cycle_prec="f32", restart=20, device="cuda:0", max_rhs=1, stack="p5",
                 transfer=None):
        self.device = torch.device(device)
        self.n = tuple(int(k) for k in n)
        self.dim = len(self.n)
        self.N = int(np.prod([k + 1 for k in self.n]))
        self.grid = make_grid(n, h, layer, sigma_max)
        self.mg = make_mg(cycle, nu, jacobi, cycle_prec, restart, stack, transfer)
        self.stack = stack
        self.shift = L.Shift(float(alpha), float(alpha2), float(beta))
        self.omega = float(omega)
        self.max_rhs = int(max_rhs)
        b = C.c_size_t()
        if self.max_rhs > 1:
            L.check(L.lib.helm_workspace_bytes_multi(C.byref(self.grid), C.byref(self.mg), self.max_rhs, C.byref(b)),
                    "helm_workspace_bytes_multi")
        else:
            L.check(L.lib.helm_workspace_bytes(C.byref(self.grid), C.byref(self.mg), C.byref(b)),
                    "helm_workspace_bytes")
        self.ws_bytes = int(b.value)
        self.ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
        base = self.ws.data_ptr()
        self._ws_ptr = (base + 255) // 256 * 256
        kap = _dev_tensor(slowness, torch.float64, self.device)
        if kap.numel() != self.N:
            raise ValueError("slowness has %d entries, grid has %d nodes" % (kap.numel(), self.N))
        self._kap = kap
        self._medium = (kap, False)     # the medium the context was factored for: (tensor, is_m)
        self.medium_version = 0         # incremented by every refactor
        ctx = C.c_void_p()
        if self.max_rhs > 1:
            L.check(L.lib.helm_setup_multi(C.byref(self.grid), C.c_void_p(kap.data_ptr()), self.omega,
                                           C.byref(self.shift), C.byref(self.mg), self.max_rhs,
                                           C.c_void_p(self._ws_ptr), self.ws_bytes,
                                           C.c_void_p(_stream_ptr(self.device)), C.byref(ctx)), "helm_setup_multi")
        else:
            L.check(L.lib.helm_setup(C.byref(self.grid), C.c_void_p(kap.data_ptr()), self.omega,
                                     C.byref(self.shift), C.byref(self.mg), C.c_void_p(self._ws_ptr), self.ws_bytes,
                                     C.c_void_p(_stream_ptr(self.device)), C.byref(ctx)), "helm_setup")
        self.ctx = ctx

    def refactor(self, slowness=None, omega=None, alpha=None, alpha2=None, beta=None, m=None):
        """numerical setup again (coefficients, Galerkin operators, coarsest factorisation) for a
        new medium / frequency / shift on the same grid.  The medium is given as the slowness
        or as its square m (helm_refactor_m); without either the current one is kept."""
        if slowness is not None and m is not None:
            raise ValueError("give the slowness or m, not both")
        if slowness is not None:
            self._medium = (_dev_tensor(slowness, torch.float64, self.device), False)
        elif m is not None:
            self._medium = (_dev_tensor(m, torch.float64, self.device), True)
        if omega is not None:
            self.omega = float(omega)
        for name, v in (("alpha", alpha), ("alpha2", alpha2), ("beta", beta)):
            if v is not None:
                setattr(self.shift, name, float(v))
        t, is_m = self._medium
        f = L.lib.helm_refactor_m if is_m else L.lib.helm_refactor
        L.check(f(self.ctx, C.c_void_p(t.data_ptr()), self.omega, C.byref(self.shift), self._s()),
                "helm_refactor_m" if is_m else "helm_refactor")
        self.medium_version += 1

    KERNEL_CLASSES = KERNEL_CLASSES

    def kernel_times(self):
        """{class: (ms, launches)} accumulated since set_timing(True)."""
        return kernel_times(self.ctx)

    # -- lifetime
    def close(self):
        if getattr(self, "ctx", None):
            L.lib.helm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def cdtype(self):
        return torch.complex64 if self.mg.cycle_prec == L.HELM_F32 else torch.complex128

    def level_size(self, lev: int) -> int:
        return int(L.lib.helm_level_size(self.ctx, 0, lev))

    def _s(self):
        return C.c_void_p(_stream_ptr(self.device))

    # -- operations
    def apply(self, x, op: int = L.HELM_OP_N, prec: str = "f64") -> torch.Tensor:
        dt = torch.complex128 if prec == "f64" else torch.complex64
        xt = _dev_tensor(x, dt, self.device)
        y = torch.empty_like(xt)
        L.check(L.lib.helm_apply(self.ctx, op, L.HELM_F64 if prec == "f64" else L.HELM_F32,
                                 C.c_void_p(xt.data_ptr()), C.c_void_p(y.data_ptr()), self._s()), "helm_apply")
        return y

    def vcycle(self, r, op: int = L.HELM_OP_N) -> torch.Tensor:
        rt = _dev_tensor(r, torch.complex128, self.device)
        z = torch.empty_like(rt)
        L.check(L.lib.helm_vcycle(self.ctx, op, C.c_void_p(rt.data_ptr()), C.c_void_p(z.data_ptr()), self._s()),
                "helm_vcycle")
        return z

    def coarse_solve(self, r, op: int = L.HELM_OP_N) -> torch.Tensor:
        rt = _dev_tensor(r, torch.complex128, self.device)
        e = torch.empty_like(rt)
        L.check(L.lib.helm_coarse_solve(self.ctx, op, C.c_void_p(rt.data_ptr()), C.c_void_p(e.data_ptr()),
                                        self._s()), "helm_coarse_solve")
        return e

    def solve(self, rhs, x0=None, tol: float = 1e-6, max_iter: int = 500, op: int = L.HELM_OP_N,
              history: bool = False) -> Tuple[torch.Tensor, dict]:
        b = _dev_tensor(rhs, torch.complex128, self.device)
        x = torch.zeros_like(b) if x0 is None else _dev_tensor(x0, torch.complex128, self.device).clone()
        info = L.SolveInfo()
        hist = None
        if history:
            hist = (C.c_double * max_iter)()
            info.history = C.cast(hist, C.POINTER(C.c_double))
            info.history_cap = max_iter
        st = L.lib.helm_solve(self.ctx, op, C.c_void_p(b.data_ptr()), C.c_void_p(x.data_ptr()), float(tol),
                              int(max_iter), C.byref(info), self._s())
        L.check(st, "helm_solve")
        out = dict(status=st, iterations=info.iterations, restarts=info.restarts,
                   est_rel_residual=info.est_rel_residual, true_rel_residual=info.true_rel_residual)
        if history:
            out["history"] = [hist[i] for i in range(min(info.iterations, max_iter))]
        return x, out

    def iterate(self, rhs, x0=None, tol: float = 1e-6, max_iter: int = 500, op: int = L.HELM_OP_N,
                history: bool = False) -> Tuple[torch.Tensor, dict]:
        """the cycle as a stand-alone solver, x <- x + M^{-1}(b - op(H) x) (helm_iterate)"""
        b = _dev_tensor(rhs, torch.complex128, self.device)
        x = torch.zeros_like(b) if x0 is None else _dev_tensor(x0, torch.complex128, self.device).clone()
        info = L.SolveInfo()
        hist = None
        if history:
            hist = (C.c_double * max_iter)()
            info.history = C.cast(hist, C.POINTER(C.c_double))
            info.history_cap = max_iter
        st = L.lib.helm_iterate(self.ctx, op, C.c_void_p(b.data_ptr()), C.c_void_p(x.data_ptr()), float(tol),
                                int(max_iter), C.byref(info), self._s())
        L.check(st, "helm_iterate")
        out = dict(status=st, iterations=info.iterations, true_rel_residual=info.true_rel_residual)
        if history:
            out["history"] = [hist[i] for i in range(min(info.iterations, max_iter))]
        return x, out

    def solve_many(self, rhs: Sequence, tol: float = 1e-6, max_iter: int = 500, op: int = L.HELM_OP_N):
        """solve for every right-hand side from a zero guess, in lock-step groups of up to
        max_rhs; each result equals solve()'s.  Returns (solutions, infos)."""
        n = len(rhs)
        bs = [_dev_tensor(r, torch.complex128, self.device) for r in rhs]
        xs = [torch.zeros_like(b) for b in bs]
        rp = (C.c_void_p * n)(*[b.data_ptr() for b in bs])
        xp = (C.c_void_p * n)(*[x.data_ptr() for x in xs])
        ii = (C.c_int * n)(*([0] * n))
        infos = (L.SolveInfo * n)()
        st = L.lib.helm_solve_batched(self.ctx, op, n, ii, rp, xp, float(tol), int(max_iter), infos, self._s())
        L.check(st, "helm_solve_batched")
        return xs, [dict(status=infos[k].status, iterations=infos[k].iterations,
                         true_rel_residual=infos[k].true_rel_residual) for k in range(n)]

    def coefficients(self, lev: int) -> np.ndarray:
        """stored Galerkin coefficients of level 2 or 3: array (planes, N_lev) complex128; plane
        k holds A(i, i + d) for the offset d with k = sum_a (d_a + r) (2r + 1)^a (r: the
        level's stencil radius, 1 for the 5/7-point stack)."""
        K = self.info()["planes2" if lev == 2 else "planes3"]
        Nl = self.level_size(lev)
        out = np.empty(K * Nl, np.complex128)
        L.check(L.lib.helm_get_coefficients(self.ctx, lev, C.c_void_p(out.ctypes.data)), "helm_get_coefficients")
        return out.reshape(K, Nl)

    def grad_m(self, us, lams, g: Optional[torch.Tensor] = None, accumulate: bool = False) -> torch.Tensor:
        """sum_s omega^2 Re(conj(lam_s) (1 - i sigma) u_s) over the given fields."""
        ut = [_dev_tensor(u, torch.complex128, self.device) for u in us]
        lt = [_dev_tensor(l, torch.complex128, self.device) for l in lams]
        if g is None:
            g = torch.zeros(self.N, dtype=torch.float64, device=self.device)
        up = (C.c_void_p * len(ut))(*[t.data_ptr() for t in ut])
        lp = (C.c_void_p * len(lt))(*[t.data_ptr() for t in lt])
        L.check(L.lib.helm_grad_m(self.ctx, len(ut), up, lp, C.c_void_p(g.data_ptr()), 1 if accumulate else 0,
                                  self._s()), "helm_grad_m")
        return g


    def info(self) -> dict:
        v = (C.c_longlong * INFO_LEN)()
        L.check(L.lib.helm_get_info(self.ctx, v, INFO_LEN), "helm_get_info")
        return parse_info(v)

    def set_timing(self, on: bool = True):
        L.lib.helm_set_timing(self.ctx, 1 if on else 0)

    def timing(self):
        t = (C.c_double * 5)()
        L.lib.helm_get_timing(self.ctx, t, 5)
        return dict(total_ms=t[0], cycle_ms=t[1], outer_ms=t[2], coarse_ms=t[3], setup_ms=t[4])


def from_problem(prob, **kw) -> Solver:
    """Solver for an object with the attributes of a workload description (n, h, slowness,
    omega, layer, sigma_max, alpha, beta, cycle, nu_pre, nu_post, jacobi, restart; stack and
    transfer if it has them)."""
    args = dict(alpha=prob.alpha, alpha2=getattr(prob, "alpha2", 1.0), beta=prob.beta, cycle=prob.cycle,
                nu=(prob.nu_pre, prob.nu_post), jacobi=prob.jacobi, restart=prob.restart,
                stack=getattr(prob, "stack", "p5"), transfer=getattr(prob, "transfer", None))
    args.update(kw)
    return Solver(prob.n, prob.h, prob.slowness, prob.omega, prob.layer, prob.sigma_max, **args)
