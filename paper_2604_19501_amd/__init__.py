"""MI355X-native real-shifted multigrid Helmholtz solver (libhelm, gfx950 HIP).

The compute path lives in libhelm.so (C ABI in include/helm.h); this package only
marshals arguments.  Importing it fails loudly if the library is not built.
"""
from ._lib import (HELM_F32, HELM_F64, HELM_OP_C, HELM_OP_N, HELM_OK, HELM_ENOCONV, HELM_ESTAGNATE,  # noqa: F401
                   HELM_EINVAL, HELM_EDEVICE, HELM_ENONFINITE, HELM_ESINGULAR, HELM_EWORKSPACE, HelmError)
from .solver import Solver, from_problem, workspace_bytes  # noqa: F401

__all__ = ["Solver", "from_problem", "workspace_bytes", "HelmError"]
