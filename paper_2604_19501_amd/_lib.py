"""ctypes binding of libhelm.so (include/helm.h).  Argument marshalling only.

Importing this module loads the in-tree library and raises ImportError if it has
not been built (``python -m paper_2604_19501_amd.build``); there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
import re

# PyTorch supplies device memory and streams and bundles its own HIP runtime
# (soname libamdhip64.so.7).  Importing it first makes libhelm bind to that same
# runtime instance; loading the system copy first would leave two HIP/HSA runtimes
# in the process and the second one finds no device.
import torch  # noqa: F401

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "libhelm.so")
# schedules picked by the autotuner (paper_2604_19501_amd/tune.py); the library reads the
# file named by HELM_TUNE_CACHE when it plans a context
TUNE_CACHE = os.path.join(HERE, "tune_cache.json")
os.environ.setdefault("HELM_TUNE_CACHE", TUNE_CACHE)
HEADER = os.path.join(os.path.dirname(HERE), "include", "helm.h")

if not os.path.exists(LIBPATH):
    raise ImportError("libhelm.so is not built: run `python -m paper_2604_19501_amd.build` (%s)" % LIBPATH)

lib = C.CDLL(LIBPATH)

HELM_OK, HELM_EINVAL, HELM_EWORKSPACE, HELM_EDEVICE, HELM_ENONFINITE, HELM_ESINGULAR = 0, -1, -2, -3, -4, -5
HELM_ENOCONV, HELM_ESTAGNATE = 1, 2
HELM_OP_N, HELM_OP_C = 0, 1
HELM_F64, HELM_F32 = 0, 1
HELM_STACK_P5, HELM_STACK_COMPACT = 0, 1
HELM_TRANSFER_CUBIC, HELM_TRANSFER_LEVDEP = 1, 2


class Grid(C.Structure):
    _fields_ = [("dim", C.c_int), ("n", C.c_int * 3), ("h", C.c_double), ("layer", (C.c_int * 2) * 3),
                ("sigma_max", C.c_double)]


class Shift(C.Structure):
    _fields_ = [("alpha", C.c_double), ("alpha2", C.c_double), ("beta", C.c_double)]


class MG(C.Structure):
    _fields_ = [("cycle", C.c_int), ("nu_pre", C.c_int), ("nu_post", C.c_int), ("jacobi", C.c_double * 2),
                ("cycle_prec", C.c_int), ("restart", C.c_int), ("stack", C.c_int), ("transfer", C.c_int)]


class SolveInfo(C.Structure):
    _fields_ = [("iterations", C.c_int), ("restarts", C.c_int), ("status", C.c_int),
                ("est_rel_residual", C.c_double), ("true_rel_residual", C.c_double),
                ("history", C.POINTER(C.c_double)), ("history_cap", C.c_int)]


P = C.c_void_p
PP = C.POINTER(C.c_void_p)
_SIG = {
    "helm_workspace_bytes": (C.c_int, [C.POINTER(Grid), C.POINTER(MG), C.POINTER(C.c_size_t)]),
    "helm_setup": (C.c_int, [C.POINTER(Grid), P, C.c_double, C.POINTER(Shift), C.POINTER(MG), P, C.c_size_t, P,
                             C.POINTER(P)]),
    "helm_refactor": (C.c_int, [P, P, C.c_double, C.POINTER(Shift), P]),
    "helm_refactor_m": (C.c_int, [P, P, C.c_double, C.POINTER(Shift), P]),
    "helm_apply": (C.c_int, [P, C.c_int, C.c_int, P, P, P]),
    "helm_vcycle": (C.c_int, [P, C.c_int, P, P, P]),
    "helm_vcycle_noalloc": (C.c_int, [P, C.c_int, P, P, P]),
    "helm_solve": (C.c_int, [P, C.c_int, P, P, C.c_double, C.c_int, C.POINTER(SolveInfo), P]),
    "helm_coarse_solve": (C.c_int, [P, C.c_int, P, P, P]),
    "helm_iterate": (C.c_int, [P, C.c_int, P, P, C.c_double, C.c_int, C.POINTER(SolveInfo), P]),
    "helm_destroy": (C.c_int, [P]),
    "helm_workspace_bytes_batched": (C.c_int, [C.c_int, C.POINTER(Grid), C.POINTER(MG), C.c_int,
                                               C.POINTER(C.c_size_t)]),
    "helm_setup_batched": (C.c_int, [C.c_int, C.POINTER(Grid), PP, C.POINTER(C.c_double), C.POINTER(Shift),
                                     C.POINTER(MG), C.c_int, P, C.c_size_t, P, C.POINTER(P)]),
    "helm_solve_batched": (C.c_int, [P, C.c_int, C.c_int, C.POINTER(C.c_int), PP, PP, C.c_double, C.c_int,
                                     C.POINTER(SolveInfo), P]),
    "helm_grad_m": (C.c_int, [P, C.c_int, PP, PP, P, C.c_int, P]),
    "helm_status_str": (C.c_char_p, [C.c_int]),
    "helm_last_error": (C.c_char_p, []),
    "helm_set_timing": (C.c_int, [P, C.c_int]),
    "helm_get_timing": (C.c_int, [P, C.POINTER(C.c_double), C.c_int]),
    "helm_level_size": (C.c_longlong, [P, C.c_int, C.c_int]),
    "helm_get_info": (C.c_int, [P, C.POINTER(C.c_longlong), C.c_int]),
    "helm_get_instance_info": (C.c_int, [P, C.c_int, C.POINTER(C.c_longlong), C.c_int]),
    "helm_workspace_bytes_multi": (C.c_int, [C.POINTER(Grid), C.POINTER(MG), C.c_int, C.POINTER(C.c_size_t)]),
    "helm_setup_multi": (C.c_int, [C.POINTER(Grid), P, C.c_double, C.POINTER(Shift), C.POINTER(MG), C.c_int, P,
                                   C.c_size_t, P, C.POINTER(P)]),
    "helm_get_coefficients": (C.c_int, [P, C.c_int, P]),
}
for _name, (_res, _args) in _SIG.items():
    _f = getattr(lib, _name)
    _f.restype = _res
    _f.argtypes = _args


def declared_symbols():
    """function names declared in include/helm.h"""
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char\*|long long)\s+(helm_\w+)\s*\(", txt, re.M)))


class HelmError(RuntimeError):
    def __init__(self, code, where):
        msg = lib.helm_last_error().decode() if code in (HELM_EINVAL, HELM_EDEVICE, HELM_EWORKSPACE) else ""
        super().__init__("%s: %s (%d) %s" % (where, lib.helm_status_str(code).decode(), code, msg))
        self.code = code


def check(code, where):
    if code < 0:
        raise HelmError(code, where)
    return code
