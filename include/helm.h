/*
 * helm.h - C ABI of libhelm, a gfx950 (MI355X) solver for the discretised
 * heterogeneous Helmholtz equation preconditioned by a 3-level multigrid cycle
 * with a real-shifted coarsest-grid Galerkin operator.
 *
 * Method (Yovel & Treister, "Scalable Multigrid Solver for the Helmholtz
 * Equation: Real-Shifted Coarse Grid Correction"):
 *   problem   -Lap p - k^2 p = q, k = omega * slowness            (eq. 1.1)
 *             discretised on a regular node grid with an absorbing layer
 *   level 1   H_beta = -Lap_h - (1 - i beta) omega^2 m (1 - i sigma),  m = slowness^2
 *   level 2   A2 = R1 H_beta P1                                     (eq. 2.2)
 *   level 3   A3 = R2 (R1 H_beta^alpha P1) P2, k -> alpha k          (eq. 3.5, 3.6)
 *             solved exactly (nested-dissection block elimination)
 *   cycle     two-grid algorithm of Sec. 2 applied recursively (V or W),
 *             damped Jacobi relaxation
 *   outer     right-preconditioned restarted FGMRES on the unshifted H
 *             (stopping rule: relative residual, Sec. 5)
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Grid: n[a] cells and n[a]+1 nodes along axis a (a < dim); every node is an
 * unknown and values one node beyond each end are zero.  n[a] must be a
 * multiple of 4 (three levels) and at least 4.  Node arrays are x-fastest:
 * flat index i0 + (n0+1)*(i1 + (n1+1)*i2).  N1 = prod(n[a]+1).
 * Complex arrays are interleaved (re, im): "c128" = 2 x double per entry,
 * "c64" = 2 x float per entry.
 * Absorbing layer: layer[a][0] / layer[a][1] cells on the low / high face of
 * axis a; sigma = sigma_max * sum_a (depth_a / width_a)^2 where depth_a is the
 * distance in cells into that layer (quadratic profile, zero outside).
 *
 * Memory: every pointer argument named as "device" is a device pointer owned
 * by the caller; the library never allocates device memory.  helm_setup
 * carves all persistent device state out of the caller's workspace (size from
 * helm_workspace_bytes), which must stay allocated and untouched until
 * helm_destroy.  The context itself is host memory owned by the library.
 * Work is enqueued on the given stream (a hipStream_t, NULL = default stream);
 * helm_solve synchronises that stream to read convergence scalars.
 *
 * Errors: every call returns an int status.  0 = success, negative = error
 * (nothing was computed or the outputs are undefined), positive = warning
 * (outputs valid, see the code).  No exception crosses the ABI.  Argument
 * validation happens before any device call.  The calls that work on one hierarchy
 * (helm_refactor, helm_refactor_m, helm_apply, helm_vcycle, helm_coarse_solve,
 * helm_solve, helm_iterate, helm_grad_m, helm_get_coefficients, helm_get_info) return
 * HELM_EINVAL for the parent context of helm_setup_batched.
 */
#ifndef HELM_H
#define HELM_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HELM_OK            0
#define HELM_EINVAL       -1   /* invalid argument (message: helm_last_error) */
#define HELM_EWORKSPACE   -2   /* workspace NULL, misaligned or too small */
#define HELM_EDEVICE      -3   /* HIP runtime error */
#define HELM_ENONFINITE   -4   /* NaN/Inf met in an input or a Krylov scalar */
#define HELM_ESINGULAR    -5   /* zero pivot in the coarsest-grid elimination */
#define HELM_ENOCONV       1   /* max_iter reached before the tolerance */
#define HELM_ESTAGNATE     2   /* no residual decrease over a full restart cycle */

#define HELM_OP_N 0            /* the operator H */
#define HELM_OP_C 1            /* its conjugate transpose H^H (= conj(H): the 5/7-point H is
                                  complex symmetric; not available for the compact stack) */

#define HELM_F64 0
#define HELM_F32 1

/* discretisation stacks (helm_mg.stack) and transfers of the compact stack (helm_mg.transfer) */
#define HELM_STACK_P5        0 /* 5-point (2D) / 7-point (3D) operator, full weighting, linear
                                  interpolation; 9/27-point Galerkin operators */
#define HELM_STACK_COMPACT   1 /* compact fourth-order 9-point / 19-point operator with its
                                  mass term (eqs. 3.1, 3.2) */
#define HELM_TRANSFER_CUBIC  1 /* R = [1 4 6 4 1]/16 per axis on both levels, P = 2^d R^T
                                  (eq. 3.3): level-2 operator 25 points, level-3 49 (2D only) */
#define HELM_TRANSFER_LEVDEP 2 /* level-dependent (eq. 3.4): the restriction from level 2 to 3
                                  is [1 2 1]/4 per axis, the rest cubic: level-2 operator 25 /
                                  125 points, level-3 25 / 125 (2D / 3D) */

typedef struct helm_ctx helm_ctx;

typedef struct {
  int dim;             /* 2 or 3 */
  int n[3];            /* cells per axis (entries >= dim ignored) */
  double h;            /* grid spacing (> 0) */
  int layer[3][2];     /* absorbing-layer width in cells: [axis][low face, high face] */
  double sigma_max;    /* layer damping at the outermost node (>= 0) */
} helm_grid;

typedef struct {
  double alpha;        /* real shift of the coarsest Galerkin operator, eq. (3.5)-(3.6) */
  double alpha2;       /* real shift of the level-2 Galerkin operator (1 = none) */
  double beta;         /* complex shift of the preconditioner: c -> (1 - i beta) c (0 = none) */
} helm_shift;

typedef struct {
  int cycle;           /* 1 = V cycle, 2 = W cycle (level 2 visited twice) */
  int nu_pre;          /* damped-Jacobi sweeps before the coarse correction, 0..4 */
  int nu_post;         /* sweeps after it, 0..4 */
  double jacobi[2];    /* damping weight on level 1 and level 2 */
  int cycle_prec;      /* HELM_F32: cycle in complex FP32 (FGMRES stays FP64); HELM_F64 */
  int restart;         /* FGMRES restart length m, 1..64 */
  int stack;           /* HELM_STACK_P5 (0) or HELM_STACK_COMPACT (Sec. 3.1) */
  int transfer;        /* HELM_STACK_COMPACT: HELM_TRANSFER_CUBIC (2D) or HELM_TRANSFER_LEVDEP;
                          ignored for HELM_STACK_P5.  The compact operator is not complex
                          symmetric: with it every call refuses HELM_OP_C (HELM_EINVAL), and
                          helm_grad_m refuses the context */
} helm_mg;

typedef struct {
  int iterations;            /* preconditioner applications */
  int restarts;              /* completed restart cycles before the last one */
  int status;                /* same code the call returned */
  double est_rel_residual;   /* Givens estimate |g_{j+1}| / ||b|| at exit */
  double true_rel_residual;  /* ||b - H x|| / ||b|| recomputed in FP64 at exit */
  double* history;           /* optional host buffer: estimate after every iteration */
  int history_cap;           /* its capacity (entries written: min(iterations, cap)) */
} helm_solve_info;

/* Device bytes of workspace helm_setup needs for this grid and cycle (pure host
 * computation, no device call).  Returns HELM_EINVAL for an invalid grid/mg. */
int helm_workspace_bytes(const helm_grid* grid, const helm_mg* mg, size_t* bytes);

/* Build the operator hierarchy for one medium (Sec. 3): coefficients, level-2
 * Galerkin operator (eq. 2.2), real-shifted level-3 operator (eq. 3.6) and its
 * exact factorisation.
 *   slowness: device, N1 doubles (kappa at every node; m = kappa^2 is formed
 *             internally; may be freed after the call returns)
 *   omega:    angular frequency (> 0)
 *   ws:       device workspace of ws_bytes >= helm_workspace_bytes(), 256-byte aligned
 *   stream:   hipStream_t
 *   out:      receives the context (host)
 * Returns HELM_ESINGULAR if the coarsest elimination meets a zero pivot. */
int helm_setup(const helm_grid* grid, const double* slowness, double omega,
               const helm_shift* shift, const helm_mg* mg, void* ws, size_t ws_bytes,
               void* stream, helm_ctx** out);

/* Redo the numerical setup of helm_setup (coefficients, Galerkin operators, coarsest
 * factorisation) for a new medium / frequency / shift on the same grid, reusing the
 * context's symbolic structure and workspace.  Arguments as in helm_setup. */
int helm_refactor(helm_ctx* ctx, const double* slowness, double omega, const helm_shift* shift, void* stream);

/* helm_refactor for a medium given as its squared slowness m = kappa^2 (device, N1 doubles,
 * m > 0), the variable of eq. (1.1)'s coefficient k^2 = omega^2 m.  Callers that
 * differentiate with respect to m (helm_grad_m) pass it here unchanged instead of forming
 * sqrt(m) for helm_refactor to square again. */
int helm_refactor_m(helm_ctx* ctx, const double* m, double omega, const helm_shift* shift, void* stream);

/* y = H x (op HELM_OP_N) or y = H^H x (HELM_OP_C), the unshifted operator of eq. (1.1).
 * prec HELM_F64: x, y device c128[N1]; HELM_F32: x, y device c64[N1].  x != y. */
int helm_apply(helm_ctx* ctx, int op, int prec, const void* x, void* y, void* stream);

/* z = M^{-1} r: one multigrid cycle from a zero initial guess (Sec. 2 algorithm, 3 levels)
 * on the preconditioner of op.  r, z: device c128[N1] (the cycle runs in the setup's
 * cycle precision).  r != z. */
int helm_vcycle(helm_ctx* ctx, int op, const void* r, void* z, void* stream);

/* Size of the static device array helm_vcycle_noalloc takes its scratch from (64 MiB on
 * every device the library runs on, held until the process ends). */
#define HELM_NOALLOC_SCRATCH_BYTES (64ull << 20)

/* helm_vcycle for callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): the same cycle and kernels,
 * with its per-call scratch (level iterates, coarsest-solve update pool, gather and
 * partial-product buffers) taken from a static device array of HELM_NOALLOC_SCRATCH_BYTES
 * instead of the context's workspace.  It calls no hipMalloc, hipFree or other allocating
 * routine (per-kernel timing is skipped for the call).  The operator data stay in the
 * context's workspace; r and z as in helm_vcycle.
 * Limit: returns HELM_EINVAL, before any device work, when the grid's scratch exceeds the
 * array (2D up to 1024^2 in either cycle precision, 3D up to 128^3 with the FP32 cycle fit;
 * the message gives the size needed).
 * Sharing: every call on one device uses that device's one array; calls that overlap in
 * time on one device (another stream, another thread) race and give undefined results.
 * Nothing in the array needs to start at zero (every entry is written before it is read),
 * so it keeps the last call's contents without harm. */
int helm_vcycle_noalloc(helm_ctx* ctx, int op, const void* r, void* z, void* stream);

/* Solve op(H) x = rhs by FGMRES(restart) preconditioned by one cycle per iteration.
 *   rhs: device c128[N1];  x: device c128[N1], initial guess on entry, solution on exit
 *   tol: relative-residual tolerance (> 0);  max_iter >= 1
 *   info: host struct filled on return (may be NULL)
 * Returns 0 when ||rhs - op(H) x|| <= tol ||rhs|| (recomputed in FP64), HELM_ENOCONV
 * or HELM_ESTAGNATE otherwise.  A zero rhs returns x = 0 after 0 iterations. */
int helm_solve(helm_ctx* ctx, int op, const void* rhs, void* x, double tol, int max_iter,
               helm_solve_info* info, void* stream);

/* The cycle as a stand-alone solver (Sec. 5.1: the method "as a solver", the counts in
 * parentheses of Table 3): the stationary iteration x <- x + M^{-1} (rhs - op(H) x) with one
 * cycle per iteration, the residual recomputed in FP64 after each, until
 * ||rhs - op(H) x|| <= tol ||rhs||.  Arguments and info as in helm_solve: iterations = cycles
 * applied, restarts = 0, est_rel_residual = true_rel_residual = the last relative residual,
 * history = the relative residual after every cycle.  Returns HELM_ENOCONV when max_iter is
 * reached or the residual grows beyond 1e8 ||rhs|| (divergence), HELM_ENONFINITE on a NaN. */
int helm_iterate(helm_ctx* ctx, int op, const void* rhs, void* x, double tol, int max_iter,
                 helm_solve_info* info, void* stream);

/* e = A3^{-1} r on the coarsest level (op HELM_OP_C: conj(A3)^{-1} r) with the factors the
 * cycle uses.  r, e: device c128[N3], N3 = helm_level_size(ctx, 0, 3).  For checking. */
int helm_coarse_solve(helm_ctx* ctx, int op, const void* r, void* e, void* stream);

/* Release the host context (the workspace stays the caller's).  NULL is accepted. */
int helm_destroy(helm_ctx* ctx);

/* ---- batched form: many media / frequencies / grid sizes, many right-hand sides ---- */

/* Workspace for n_inst instances (grids[i]), each solving up to min(max_rhs, 16) right-hand
 * sides in lock-step (every vector buffer of an instance is carved that many times). */
int helm_workspace_bytes_batched(int n_inst, const helm_grid* grids, const helm_mg* mg,
                                 int max_rhs, size_t* bytes);

/* Set up n_inst independent instances in one workspace.
 *   slowness: host array of n_inst device pointers (each N1(i) doubles)
 *   omega, shift: host arrays of n_inst entries */
int helm_setup_batched(int n_inst, const helm_grid* grids, const double* const* slowness,
                       const double* omega, const helm_shift* shift, const helm_mg* mg,
                       int max_rhs, void* ws, size_t ws_bytes, void* stream, helm_ctx** out);

/* One instance (as helm_workspace_bytes / helm_setup) that can also solve up to
 * min(max_rhs, 16) right-hand sides in lock-step through helm_solve_batched with every
 * inst_of_rhs[k] = 0, e.g. the sources of one medium (Sec. 5).  helm_refactor, helm_solve,
 * helm_grad_m and the other single-instance calls work on it as on a helm_setup context. */
int helm_workspace_bytes_multi(const helm_grid* grid, const helm_mg* mg, int max_rhs, size_t* bytes);
int helm_setup_multi(const helm_grid* grid, const double* slowness, double omega, const helm_shift* shift,
                     const helm_mg* mg, int max_rhs, void* ws, size_t ws_bytes, void* stream, helm_ctx** out);

/* Solve n_rhs systems; rhs k belongs to instance inst_of_rhs[k].
 *   rhs, x: host arrays of n_rhs device pointers (c128[N1(inst)] each; x holds the initial
 *           guess and receives the solution; rhs[k] != x[k])
 *   info:   host array of n_rhs structs (may be NULL)
 * An instance's right-hand sides are taken in order, in groups of up to its lock-step
 * capacity: a group runs every kernel once for all its right-hand sides (grid y), each
 * with its own FGMRES state; one that has converged or stopped does no more Krylov work
 * while the others continue.  Instances run concurrently on library-owned streams
 * (HELM_BATCH_STREAMS, default 8).  Each result, status and iteration count equals that
 * of helm_solve on the instance.  Returns the worst status over the right-hand sides
 * (the most severe error, else the largest warning). */
int helm_solve_batched(helm_ctx* ctx, int op, int n_rhs, const int* inst_of_rhs,
                       const void* const* rhs, void* const* x, double tol, int max_iter,
                       helm_solve_info* info, void* stream);

/* ---- gradient of a least-squares misfit w.r.t. squared slowness ---- */

/* g[j] (+)= sum_s omega^2 Re( conj(lambda_s[j]) (1 - i sigma_j) u_s[j] ), the derivative of
 * 1/2 sum_s ||P u_s - d_s||^2 when H u_s = q_s and H^H lambda_s = P^T (P u_s - d_s)
 * (dH/dm_j = -omega^2 (1 - i sigma_j) e_j e_j^T).
 *   u, lambda: host arrays of n_src device pointers (c128[N1]);  g: device double[N1]
 *   accumulate: 0 overwrites g, 1 adds to it.  Single-instance contexts only. */
int helm_grad_m(helm_ctx* ctx, int n_src, const void* const* u, const void* const* lambda,
                double* g, int accumulate, void* stream);

/* ---- introspection ---- */

/* Human-readable name of a status code (static string). */
const char* helm_status_str(int status);

/* Message of the last HELM_EINVAL / HELM_EDEVICE raised on this thread (static buffer). */
const char* helm_last_error(void);

/* Device timing (HIP events), recorded while enabled by helm_set_timing(ctx, 1), which also
 * clears the accumulators (on every instance of a batched context; its class sums are then
 * summed over the instances).  helm_get_timing fills host array t[0..n): [0] last solve total ms,
 * [1..3] reserved (0), [4] last setup ms, then for kernel class k = 0..11 (level-1 sweep,
 * level-1 residual+restriction, level-2 sweep, level-2 residual+restriction, coarsest
 * forward substitution, coarsest backward substitution, Arnoldi step (apply, two
 * orthogonalisation passes, Givens, normalisation), -, -, -, level-2 chain (2D, one pre-
 * and one post-sweep: the post-sweep of a level-2 visit, the pre-sweep of the next and its
 * residual+restriction in one launch), cycle tail (2D, one post-sweep per level: the last
 * level-2 post-sweep and the level-1 post-sweep in one launch)) the pair t[5+2k] =
 * accumulated ms, t[6+2k] = launches.  Returns the number of entries written. */
int helm_set_timing(helm_ctx* ctx, int on);
int helm_get_timing(helm_ctx* ctx, double* t, int n);

/* Sizes of a single-instance context (host integers), for bytes models and checks:
 * [0] N1, [1] N2, [2] N3 unknowns per level, [3] fronts of the coarsest elimination,
 * [4] entries of the forward factor blocks sum(nF*nS), [5] entries of the backward blocks
 * sum(nS*nB), [6] update entries sum(nB), [7] separator entries sum(nS) (= N3),
 * [8] forward and [9] backward substitution kernel launches per coarsest solve, [10] workspace
 * bytes, [11] largest front size nF, [12] bytes per complex of the cycle (8 or 16),
 * [13] leaf box size and [14] root merge limit of the nested dissection, [15] 1 if the
 * schedule came from the autotuner cache (HELM_TUNE_CACHE), [16] number of tree-block
 * launches per direction, [17..20] the heights closing them (-1 beyond), [21] bit mask of
 * the dissection-tree heights whose fronts were merged into their parents, [22] and [23]
 * coefficient planes of the stored level-2 and level-3 operators ((2r+1)^dim for stencil
 * radius r: 9 / 27 for the 5/7-point stack), [24] bytes per complex of the coarsest solve's
 * factors and vectors (the cycle's precision; 16 for the compact stack), [25..28] box-shape
 * variants of the tiled level-1 sweep, level-1 restriction, level-2 sweep and level-2
 * restriction kernels (5/7-point stack; HELM_BOXES or the autotuner's cache).
 * Returns the number of entries written (at most n). */
int helm_get_info(helm_ctx* ctx, long long* out, int n);

/* The same sizes for instance inst of a batched context (inst 0 of a single-instance
 * context).  HELM_EINVAL for an instance that does not exist. */
int helm_get_instance_info(helm_ctx* ctx, int inst, long long* out, int n);

/* Number of unknowns on level lev (1..3) of instance inst. */
long long helm_level_size(helm_ctx* ctx, int inst, int lev);

/* Copy the stored Galerkin coefficients of level lev (2 or 3) of a single-instance
 * context to host memory: out receives 3^dim * N_lev complex doubles, coefficient k of
 * node i at out[k*N_lev + i], offset k = (d0+1) + 3 (d1+1) [+ 9 (d2+1)].  For checking. */
int helm_get_coefficients(helm_ctx* ctx, int lev, double* out);

#ifdef __cplusplus
}
#endif
#endif /* HELM_H */
