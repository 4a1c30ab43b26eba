"""FP64 CPU oracle for the real-shifted multigrid Helmholtz solver.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, complex128 NumPy/SciPy
restatement of what the method computes, written from the paper (Yovel & Treister,
"Scalable Multigrid Solver for the Helmholtz Equation: Real-Shifted Coarse Grid
Correction"): the discretised Helmholtz operator of eq. (1.1) with an absorbing
layer, the two-grid cycle of the paper's Algorithm (Sec. 2) applied recursively
as a 3-level V/W cycle, Galerkin coarsening eq. (2.2), the real-shifted coarsest
operator eq. (3.5)-(3.6), FGMRES, the grid-to-grid dispersion analysis of Sec. 4,
and the adjoint gradient of a least-squares misfit.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import it.  It shares no code with the GPU library and the GPU
library never calls it; both read their inputs from ``synth``.

Modules
-------
operators   grid, Laplacian, absorbing layer, Helmholtz matrix, transfers, Galerkin
multigrid   3-level cycle with real-shifted exact coarsest solve
fgmres      right-preconditioned flexible GMRES (restarted)
alpha       grid-to-grid dispersion analysis and alpha* search (Sec. 4)
gradient    adjoint solve and the misfit gradient w.r.t. squared slowness
"""
