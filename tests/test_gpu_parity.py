"""GPU parity of every step of the hot path against the FP64 CPU oracle, through the C ABI.

Tolerances: FP64 kernels agree with the oracle to 1e-12 relative (rounding order
only); FP32 kernels to a few 1e-6 per stencil application (single precision
rounding of O(10) terms) and to 1e-4 for the coarsest solve and the cycle, whose
conditioning amplifies FP32 rounding; solves must meet the 1e-6 relative-residual
stopping rule in FP64 with iteration counts equal to the oracle's +-1.  Beside the
2-norm comparison every cycle result is also compared element by element
(max_i |z_i - ref_i| <= tol_inf max_i |ref_i|, tol_inf = 1e-10 in FP64 and 3e-4 in
FP32): the FP32 error of a cycle is dominated by the coarsest solve's, which the
prolongation spreads smoothly, so the largest element error stays within a small
factor of the 2-norm one, while a single wrong node would exceed it.
"""

TOL_INF = {"f64": 1e-10, "f32": 3e-4}
import numpy as np
import pytest
import scipy.sparse.linalg as spla
import torch

import synth
from tests.gpu_helpers import maxabs_rel, oracle_hierarchy, rect_problem, rel, small_problem, stencil_arrays

pytestmark = pytest.mark.gpu

L = pytest.importorskip("paper_2604_19501_amd._lib")
from paper_2604_19501_amd import HELM_OP_C, HELM_OP_N, from_problem  # noqa: E402
from oracle import fgmres  # noqa: E402
from paper_2604_19501_amd.tune import MERGES  # noqa: E402


def _rand(N, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(N) + 1j * rng.standard_normal(N)


@pytest.fixture(scope="module", params=[2, 3])
def case(request):
    dim = request.param
    p = small_problem(dim, alpha2=1.03)
    H = oracle_hierarchy(p, nu_pre=1, nu_post=1)
    return dim, p, H


def test_apply(case):
    dim, p, H = case
    print("apply dim", dim, flush=True)
    s = from_problem(p, nu=(1, 1), cycle_prec="f64")
    x = _rand(p.N, 1)
    y = s.apply(x).cpu().numpy()
    assert rel(y, H.H @ x) < 1e-13
    yc = s.apply(x, op=HELM_OP_C).cpu().numpy()
    assert rel(yc, H.H.conjugate() @ x) < 1e-13
    y32 = s.apply(x, prec="f32").cpu().numpy()
    assert rel(y32, H.H @ x) < 1e-5


def test_galerkin_coefficients(case):
    dim, p, H = case
    print("galerkin dim", dim, flush=True)
    s = from_problem(p, nu=(1, 1), cycle_prec="f64")
    A2 = stencil_arrays(H.A[1], H.n2)
    A3 = stencil_arrays(H.A[2], H.n3)
    assert rel(s.coefficients(2), A2) < 1e-13
    assert rel(s.coefficients(3), A3) < 1e-13


@pytest.mark.parametrize("prec,tol", [("f64", 1e-10), ("f32", 1e-4)])
def test_coarse_solve(case, prec, tol):
    dim, p, H = case
    print("coarse dim", dim, prec, flush=True)
    s = from_problem(p, nu=(1, 1), cycle_prec=prec)
    r = _rand(s.level_size(3), 3)
    e = s.coarse_solve(r).cpu().numpy()
    assert rel(e, H.lu3.solve(r)) < tol
    ec = s.coarse_solve(r, op=HELM_OP_C).cpu().numpy()
    assert rel(ec, np.conj(H.lu3.solve(np.conj(r)))) < tol


@pytest.mark.parametrize("dim,n", [(2, 256), (3, 64)])
@pytest.mark.parametrize("cuts,panel,splitk", [("none", "lds", None), ("", "lds", None), ("1", "lds", None),
                                               ("0,1,2,3", "lds", None), ("", "multi", None), ("none", "lds", 0),
                                               ("1", "multi", 0), ("", "multi64", None), ("", "multi_unblocked", None),
                                               ("", "lds_waves4", None), ("", "lds_blocked", None),
                                               ("", "lds_merge_odd", None), ("1", "lds_merge_even", 0),
                                               ("none", "multi_merge_two_of_three", None)])
def test_coarse_solve_schedules(monkeypatch, dim, n, cuts, panel, splitk):
    """the exact coarsest solve under every kind of substitution schedule (row-chunk
    launches only, the planner's choice, one tree-block launch, one per level, split-K
    launches for every height above the tree blocks), with both factorisation panel
    paths (LDS-resident; multi-work-group panels of 64 or 32 columns in blocks of 128 with
    one trailing update per block, or one trailing update per 64-column panel) and with
    dissection levels merged into their parents (every second level, two of every three)."""
    monkeypatch.setenv("HELM_ND_CUTS", cuts)
    for name, heights in MERGES.items():
        if panel.endswith("_merge_" + name):
            monkeypatch.setenv("HELM_ND_MERGE", heights)
    if panel.startswith("multi"):
        monkeypatch.setenv("HELM_ND_LDS_PANEL", "0")
    if panel == "multi64":
        monkeypatch.setenv("HELM_ND_KB_MULTI", "64")
    if panel == "multi_unblocked":
        monkeypatch.setenv("HELM_ND_KB_OUTER", "64")
    if panel == "lds_waves4":          # tree-block work-groups of 4 wavefronts
        monkeypatch.setenv("HELM_ND_TREE_WAVES", "4")
    if panel == "lds_blocked":         # register panels grouped into 128-column blocks at every height
        monkeypatch.setenv("HELM_ND_REG_BLOCK_MB", "0")
    if splitk is not None:
        monkeypatch.setenv("HELM_ND_SPLITK_KB", str(splitk))
    p = synth.config2(n) if dim == 2 else synth.config3(n)
    print("coarse schedule", dim, n, repr(cuts), panel, splitk, flush=True)
    H = oracle_hierarchy(p, nu_pre=1, nu_post=1)
    for prec, tol in (("f64", 1e-10), ("f32", 1e-4)):
        s = from_problem(p, nu=(1, 1), cycle_prec=prec)
        r = _rand(s.level_size(3), 4)
        e = s.coarse_solve(r).cpu().numpy()
        assert rel(e, H.lu3.solve(r)) < tol, (prec, rel(e, H.lu3.solve(r)))
        ec = s.coarse_solve(r, op=HELM_OP_C).cpu().numpy()
        assert rel(ec, np.conj(H.lu3.solve(np.conj(r)))) < tol
        s.close()


def test_coarse_solve_full_size_2d():
    """the coarsest level of the 1024^2 layered workload (66049 unknowns)."""
    p = synth.config2(1024)
    H = oracle_hierarchy(p)
    r = _rand(H.lu3.shape[0], 12)
    ref = H.lu3.solve(r)
    for prec, tol in (("f64", 1e-10), ("f32", 1e-4)):
        s = from_problem(p, nu=(1, 1), cycle_prec=prec)
        e = s.coarse_solve(r).cpu().numpy()
        assert rel(e, ref) < tol, (prec, rel(e, ref))
        s.close()


@pytest.mark.parametrize("cycle,nu", [(2, (1, 1)), (2, (2, 2)), (1, (1, 1)), (2, (0, 1)), (2, (1, 0))])
def test_cycle(case, cycle, nu):
    dim, p, H0 = case
    print("cycle dim", dim, cycle, nu, flush=True)
    H = oracle_hierarchy(p, cycle=cycle, nu_pre=nu[0], nu_post=nu[1])
    r = _rand(p.N, 5)
    ref = H.precond(r)
    Hc = oracle_hierarchy(p, cycle=cycle, nu_pre=nu[0], nu_post=nu[1], conj=True)
    refc = Hc.precond(r)
    for prec, tol in (("f64", 1e-10), ("f32", 1e-4)):
        s = from_problem(p, cycle=cycle, nu=nu, cycle_prec=prec)
        z = s.vcycle(r).cpu().numpy()
        assert rel(z, ref) < tol, (prec, rel(z, ref))
        assert maxabs_rel(z, ref) < TOL_INF[prec], (prec, maxabs_rel(z, ref))
        zc = s.vcycle(r, op=HELM_OP_C).cpu().numpy()       # the adjoint solves' preconditioner
        assert rel(zc, refc) < tol, (prec, rel(zc, refc))
        assert maxabs_rel(zc, refc) < TOL_INF[prec], (prec, maxabs_rel(zc, refc))
        s.close()


@pytest.mark.parametrize("n", [(136, 72), (40, 24, 32)])
@pytest.mark.parametrize("nu", [(1, 1), (2, 2)])
def test_cycle_rectangular_multi_tile(n, nu):
    """non-square grids: several stencil tiles per axis with ragged last tiles on every level."""
    p = rect_problem(n)
    print("cycle rect", n, nu, flush=True)
    H = oracle_hierarchy(p, cycle=2, nu_pre=nu[0], nu_post=nu[1])
    r = _rand(p.N, 6)
    ref = H.precond(r)
    refc = oracle_hierarchy(p, cycle=2, nu_pre=nu[0], nu_post=nu[1], conj=True).precond(r)
    for prec, tol in (("f64", 1e-10), ("f32", 1e-4)):
        s = from_problem(p, cycle=2, nu=nu, cycle_prec=prec)
        z = s.vcycle(r).cpu().numpy()
        assert rel(z, ref) < tol, (prec, rel(z, ref))
        assert maxabs_rel(z, ref) < TOL_INF[prec], (prec, maxabs_rel(z, ref))
        zc = s.vcycle(r, op=HELM_OP_C).cpu().numpy()
        assert rel(zc, refc) < tol, (prec, rel(zc, refc))
        assert maxabs_rel(zc, refc) < TOL_INF[prec], (prec, maxabs_rel(zc, refc))
        s.close()


@pytest.mark.parametrize("n", [(136, 72), (40, 24, 32), (200, 136)])
@pytest.mark.parametrize("boxes", ["1,1,1,1", "2,2,2,2", "3,0,3,0", "4,3,4,3", "5,4,5,4"])
def test_cycle_box_variants(monkeypatch, n, boxes):
    """every box-shape variant of the tiled cycle kernels (level-1/level-2 sweeps and
    restrictions; 4/5 and 3/4 the 3D z-marching tiles, several z-chunks with a ragged last
    one), on grids with several tiles per axis and ragged last tiles, against the oracle
    element by element (the FP64 3D kernels keep the default boxes)"""
    monkeypatch.setenv("HELM_BOXES", boxes)
    p = rect_problem(n)
    print("cycle boxes", n, boxes, flush=True)
    H = oracle_hierarchy(p, cycle=2, nu_pre=1, nu_post=1)
    r = _rand(p.N, 7)
    ref = H.precond(r)
    for prec, tol in (("f64", 1e-10), ("f32", 1e-4)):
        s = from_problem(p, cycle=2, nu=(1, 1), cycle_prec=prec)
        z = s.vcycle(r).cpu().numpy()
        assert rel(z, ref) < tol, (prec, rel(z, ref))
        assert maxabs_rel(z, ref) < TOL_INF[prec], (prec, maxabs_rel(z, ref))
        s.close()


@pytest.mark.parametrize("n", [(136, 72), (200, 136)])
def test_level2_chain_matches_separate_kernels(monkeypatch, n):
    """2D W-cycle with one pre- and one post-sweep: the fused level-2 chain (the first
    visit's post-sweep, the second visit's pre-sweep and restriction in one kernel) takes
    the separate kernels' sums in their order: the cycle equals theirs to rounding in both
    precisions, for the operator and its conjugate, and the oracle's"""
    cycle = 2
    p = rect_problem(n)
    r = _rand(p.N, 9)
    H = oracle_hierarchy(p, cycle=cycle, nu_pre=1, nu_post=1)
    ref = H.precond(r)
    for prec, tol in (("f64", 1e-14), ("f32", 1e-6)):
        out = {}
        for on in ("0", "1"):
            monkeypatch.setenv("HELM_L2_CHAIN", on)
            print("l2 chain", n, cycle, prec, on, flush=True)
            s = from_problem(p, cycle=cycle, nu=(1, 1), cycle_prec=prec)
            out[on] = (s.vcycle(r).cpu().numpy(), s.vcycle(r, op=HELM_OP_C).cpu().numpy())
            s.close()
        for o in (0, 1):
            d = np.abs(out["1"][o] - out["0"][o]).max() / np.abs(out["0"][o]).max()
            print("  %s op %d: max difference %.3e of the largest entry" % (prec, o, d), flush=True)
            assert d < tol, (prec, o, d)
        assert maxabs_rel(out["1"][0], ref) < TOL_INF[prec]


@pytest.mark.parametrize("n", [(40, 24, 32), (64, 64, 64)])
def test_z_marching_tiles_match_box_tiles(monkeypatch, n):
    """the 3D z-marching sweep and restriction tiles take the box kernels' sums in the same
    order: the FP32 cycle through them equals the default boxes' to rounding, for the
    operator and its conjugate (the adjoint solves' cycle; printed: the largest difference
    relative to the largest entry)"""
    p = rect_problem(n)
    r = _rand(p.N, 8)
    out = {}
    for boxes in ("0,0,0,0", "4,3,4,3", "5,4,5,4"):
        monkeypatch.setenv("HELM_BOXES", boxes)
        print("z tiles", n, boxes, flush=True)
        s = from_problem(p, cycle=2, nu=(1, 1), cycle_prec="f32")
        out[boxes] = (s.vcycle(r).cpu().numpy(), s.vcycle(r, op=HELM_OP_C).cpu().numpy())
        s.close()
    for o, name in ((0, "H"), (1, "conj(H)")):
        ref = out["0,0,0,0"][o]
        for boxes in ("4,3,4,3", "5,4,5,4"):
            d = np.abs(out[boxes][o] - ref).max() / np.abs(ref).max()
            print("  %s %s: max difference %.3e of the largest entry" % (name, boxes, d), flush=True)
            assert d < 1e-6, (name, boxes, d)


@pytest.mark.parametrize("restart", [20, 4])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_solve_small(case, prec, restart):
    """whole solves against the oracle's FGMRES: iterations +-1, the true residual, and the
    solution error against the exact solution (sparse LU of H) within 3x the oracle's own;
    restart 4 takes the solves through several restart cycles."""
    dim, p, H = case
    print("solve dim", dim, prec, "restart", restart, flush=True)
    q = p.rhs()
    ref = fgmres.solve(H, q, tol=1e-6, restart=restart, max_iter=400)
    ustar = spla.splu(H.H.tocsc()).solve(q)
    s = from_problem(p, nu=(1, 1), cycle_prec=prec, restart=restart)
    x, info = s.solve(q, tol=1e-6, max_iter=400)
    xg = x.cpu().numpy()
    res = np.linalg.norm(q - H.H @ xg) / np.linalg.norm(q)
    assert info["status"] == 0
    assert res <= 1e-6
    assert abs(info["true_rel_residual"] - res) <= 1e-9
    assert abs(info["iterations"] - ref.iterations) <= 1, (info["iterations"], ref.iterations)
    if restart == 4:
        assert ref.restarts >= 2 and info["restarts"] >= 2
    e_gpu, e_orc = rel(xg, ustar), rel(ref.x, ustar)
    print("  its gpu %d oracle %d, restarts %d/%d, error %.2e (oracle %.2e), diff to oracle %.2e"
          % (info["iterations"], ref.iterations, info["restarts"], ref.restarts, e_gpu, e_orc, rel(xg, ref.x)))
    assert e_gpu <= max(3.0 * e_orc, 1e-7), (e_gpu, e_orc)
    # the oracle's iterate up to rounding (FP64 cycle) or up to the FP32 cycle's
    # perturbation of the directions (same bounds as the full-size tests)
    lim = 1e-10 if prec == "f64" else 1e-6
    assert rel(xg, ref.x) <= lim and maxabs_rel(xg, ref.x) <= lim


def test_adjoint_solve_and_dot(case):
    dim, p, H = case
    s = from_problem(p, nu=(1, 1), cycle_prec="f64")
    x, y = _rand(p.N, 8), _rand(p.N, 9)
    Hx = s.apply(x).cpu().numpy()
    Hty = s.apply(y, op=HELM_OP_C).cpu().numpy()
    assert abs(np.vdot(Hx, y) - np.vdot(x, Hty)) <= 1e-12 * abs(np.vdot(Hx, y))
    q = p.rhs()
    xa, info = s.solve(q, op=HELM_OP_C, tol=1e-8, max_iter=300)
    xa = xa.cpu().numpy()
    assert np.linalg.norm(q - H.H.conjugate() @ xa) / np.linalg.norm(q) <= 1e-8


def test_edge_cases():
    p = small_problem(2)
    s = from_problem(p, nu=(1, 1), cycle_prec="f32")
    x, info = s.solve(np.zeros(p.N, np.complex128))
    assert info["status"] == 0 and info["iterations"] == 0 and torch.count_nonzero(x).item() == 0
    x, info = s.solve(p.rhs(), max_iter=1)
    assert info["status"] == L.HELM_ENOCONV and info["iterations"] == 1
    bad = p.rhs()
    bad[3] = np.nan
    with pytest.raises(L.HelmError) as ei:
        s.solve(bad)
    assert ei.value.code == L.HELM_ENONFINITE
    # resume: maxit k then a second call from the returned x converges
    x1, i1 = s.solve(p.rhs(), max_iter=3)
    x2, i2 = s.solve(p.rhs(), x0=x1, max_iter=200)
    assert i2["status"] == 0 and i2["true_rel_residual"] <= 1e-6


def test_graph_replays_match_eager(monkeypatch):
    """the per-iteration hipGraphs, replayed over several solves with eager work and host
    synchronisation in between, give exactly the eager (uncaptured) result."""
    p = small_problem(2, n=64, alpha2=1.03)
    q = p.rhs()
    monkeypatch.setenv("HELM_GRAPHS", "0")
    se = from_problem(p, nu=(1, 1), cycle_prec="f32")
    xe, ie = se.solve(q, tol=1e-6, max_iter=200)
    monkeypatch.setenv("HELM_GRAPHS", "1")
    sg = from_problem(p, nu=(1, 1), cycle_prec="f32")
    for rep in range(3):
        xg, ig = sg.solve(q, tol=1e-6, max_iter=200)
        torch.cuda.synchronize()
        _ = se.apply(xg)                       # eager work between replays
        assert ig["iterations"] == ie["iterations"]
        assert torch.equal(xg, xe), rep


def test_arnoldi_cancellation_guard_ends_the_cycle(monkeypatch):
    """when ||w - V c||^2 from the Gram formula falls below guard * ||w||^2 the column ends its
    restart cycle and the true residual is recomputed.  With the guard forced to 1 every column
    takes that branch, so the solve is FGMRES(1): its iteration count equals the oracle's
    FGMRES with restart 1 (+-1), every cycle holds one column, and it converges."""
    p = small_problem(2, alpha2=1.03)
    H = oracle_hierarchy(p, nu_pre=1, nu_post=1)
    q = p.rhs()
    ref = fgmres.solve(H, q, tol=1e-6, restart=1, max_iter=400)
    monkeypatch.setenv("HELM_ARNOLDI_GUARD", "1.0")
    for prec in ("f64", "f32"):
        s = from_problem(p, nu=(1, 1), cycle_prec=prec)
        x, info = s.solve(q, tol=1e-6, max_iter=400)
        res = np.linalg.norm(q - H.H @ x.cpu().numpy()) / np.linalg.norm(q)
        print("guard forced %s: %d iterations (oracle FGMRES(1) %d), %d restarts, residual %.2e"
              % (prec, info["iterations"], ref.iterations, info["restarts"], res), flush=True)
        assert info["status"] == 0 and res <= 1e-6
        assert abs(info["iterations"] - ref.iterations) <= 1
        assert info["restarts"] == info["iterations"] - 1
        s.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_iterate_cycle_as_solver(case, prec):
    """the cycle as a stand-alone solver (helm_iterate) against the oracle's stationary
    iteration: the same number of cycles (+-1), the residual history cycle by cycle (FP64
    cycle 1e-9, FP32 cycle 1e-4 relative), the final true residual."""
    dim, p, H = case
    from oracle import multigrid
    q = p.rhs()
    xo, its_o, hist_o = multigrid.stationary(H, q, tol=1e-6, max_iter=300)
    s = from_problem(p, nu=(1, 1), cycle_prec=prec)
    x, info = s.iterate(q, tol=1e-6, max_iter=300, history=True)
    xg = x.cpu().numpy()
    res = np.linalg.norm(q - H.H @ xg) / np.linalg.norm(q)
    print("iterate dim %d %s: %d cycles (oracle %d), residual %.2e" % (dim, prec, info["iterations"], its_o, res))
    assert info["status"] == 0 and res <= 1e-6
    assert abs(info["iterations"] - its_o) <= 1
    k = min(len(hist_o), len(info["history"]))
    hg, ho = np.array(info["history"][:k]), np.array(hist_o[:k])
    assert np.max(np.abs(hg - ho) / ho) <= (1e-9 if prec == "f64" else 1e-4)
    assert rel(xg, xo) <= (1e-9 if prec == "f64" else 1e-4)
    s.close()


def test_alpha_sweep_matches_oracle_factors():
    """convergence factors of the cycle as a solver at several real shifts (the Fig. 3
    analogue) equal the oracle's stationary iteration's within 2 %."""
    from oracle import multigrid
    from paper_2604_19501_amd import sweep as sw
    n, G = (64, 64), 12.0
    alphas = [1.0, 1.08, 1.117, 1.16]
    gpu = sw.sweep(n, G, alphas, nu=2, cycles=40, prec="f64")
    dim, h, kappa, omega, layer = sw.homogeneous(n, G)
    q = np.zeros(int(np.prod([k + 1 for k in n])), np.complex128)
    q[q.size // 2] = 1.0
    for a, r in zip(alphas, gpu):
        H = multigrid.Hierarchy(n, h, kappa.ravel() ** 2, omega, layer, 2.0, alpha=a, beta=0.0, cycle=2,
                                nu_pre=2, nu_post=2, jacobi=(0.8, 0.8))
        _, its, hist = multigrid.stationary(H, q, tol=1e-300, max_iter=40)
        fo = sw.factor(hist)
        print("alpha %.3f: factor gpu %.4f oracle %.4f" % (a, r["factor"], fo))
        assert abs(r["factor"] - fo) <= 0.02 * fo
