/*
 * srj.h - C ABI of an MI355X (gfx950) solver for A x = b by Scheduled
 * Relaxation Jacobi (SRJ) with a data-driven choice of scheme per cycle.
 *
 * Method: Islam & Wang, "A data driven heuristic for rapid convergence of
 * Scheduled Relaxation Jacobi schemes", arXiv 2011.06636.
 *   - matrix splitting A = D + L + U: section 2, Eq. 1;
 *   - relaxed Jacobi sweep x <- x + w D^-1 (b - A x): section 2, Eq. 3
 *     (residual form of the same update);
 *   - SRJ cycle = M sweeps with the factors of one scheme: section 2, Eq. 7;
 *   - scheme family w_j = (l* + 1) / (2 (l* - x_j)), x_j the roots of the
 *     Chebyshev polynomial T_M and T_M(l*) = 3: section 2, Eq. (17);
 *   - scheme level -> M: Appendix B (25 levels, M = 1 ... 2362);
 *   - next level from the ratio of the residual norms after and before a
 *     cycle: section 3, Algorithm 1 (ratio > 0.4: up one level; 0.2 < ratio
 *     < 0.4: down one level; otherwise keep);
 *   - stopping: L2 residual norm (section 4.1) or relative L2 residual
 *     (section 4.2.3, Eq. (27)), tested at the end of each cycle.
 *
 * Problems are symmetric stencil matrices on a structured n0 x n1 x n2
 * interior grid (unused axes have size 1) with homogeneous Dirichlet ghosts:
 *   A[p][p]       = diag ? diag[p] : dconst              (> 0)
 *   A[p][p + e_d] = A[p + e_d][p] = -(face[d] ? face[d][p] : cconst[d])
 * Every field is a dense array of n0*n1*n2 binary64 values with axis 0
 * contiguous: point (i0, i1, i2) is element i0 + n0*(i1 + n1*i2).  A
 * non-zero Dirichlet boundary is folded into b by the caller.
 *
 * Arithmetic: binary64, round to nearest even, with no contraction into
 * fused multiply-add, in the fixed per-point order
 *   s = D_p x_p;  for d = 0..ndim-1: s -= c_lo * x[p - e_d]; s -= c_hi * x[p + e_d];
 *   x'_p = x_p + w * ((1 / D_p) * (b_p - s))
 * (ghost neighbours contribute nothing, whatever face[d] holds on the last
 * layer along axis d), so iterates do not depend on tiling
 * or on the number of sweeps fused into one kernel.  The refinement modes
 * run the inner cycles on the correction equation in binary32 arithmetic.
 *
 * Memory and streams.  All array pointers passed to setup/solve calls are
 * DEVICE pointers owned by the caller and borrowed by the library: they must
 * stay valid, and b/faces/diag unchanged, until the context is destroyed.
 * The library owns its workspaces (ping-pong buffers, reduction scratch,
 * scheme tables).  All device work is enqueued on the hipStream_t given at
 * setup (NULL = the null stream).  Calls that return host values block until
 * those values are valid.  A context must not be used by two threads at once.
 *
 * Errors.  Every call returns an srj_status; no exception crosses the ABI.
 * Arguments are validated before any device work (SRJ_ERR_INVALID), device
 * arrays included: each must lie, whole, inside one allocation of device (or
 * managed) memory of the device that was current at setup; host memory,
 * pinned or not, is refused.
 * srj_last_error() returns a thread-local description of the last non-OK
 * status.
 */
#ifndef SRJ_H
#define SRJ_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct srj_ctx srj_ctx;
typedef struct srj_batch srj_batch;

typedef enum {
    SRJ_OK = 0,
    SRJ_ERR_INVALID = 1,       /* bad argument; nothing was run */
    SRJ_ERR_NOMEM = 2,         /* device or host allocation failed */
    SRJ_ERR_HIP = 3,           /* a HIP runtime call failed */
    SRJ_ERR_NOT_CONVERGED = 4, /* a cap was reached; results are filled */
    SRJ_ERR_NONFINITE = 5,     /* a residual norm was NaN/Inf; x holds the last iterate */
    SRJ_ERR_UNSUPPORTED = 6    /* valid request the library does not implement */
} srj_status;

typedef enum {
    SRJ_PREC_F64 = 0,        /* plain binary64 SRJ */
    SRJ_PREC_F32_REFINE = 1, /* binary32 inner cycles, binary64 outer refinement */
    SRJ_PREC_F16_REFINE = 2, /* binary16 storage of the correction, binary32 math */
    SRJ_PREC_BF16_REFINE = 3 /* bfloat16 storage of the correction, binary32 math */
} srj_precision;

typedef enum {
    SRJ_RULE_HEURISTIC = 0,  /* Algorithm 1 */
    SRJ_RULE_INCREASING = 1, /* level + 1 every cycle (comparison rule of section 4) */
    SRJ_RULE_FIXED = 2       /* fixed_level every cycle */
} srj_rule;

/* Stopping tests.  RELATIVE: cycle-end ||b - A x||_2 < tol * r0 (section
 * 4.2.3, Eq. (27)).  ABSOLUTE: cycle-end ||b - A x||_2 < tol (section 4.1).
 * UPDATE_INF: after every sweep, max_p |x'_p - x_p| < tol, the update norm
 * of the 2D Laplace test with Neumann boundaries (section 4.2.2, Eq. (25));
 * the selector still runs on cycle-end residual ratios.  UPDATE_INF needs
 * precision SRJ_PREC_F64; the update's maximum is reduced in the sweep
 * kernels (one sweep per launch, the fused per-face blocks of plan kind 10,
 * where the stop sweep's iterate is formed again from its launch's input, or
 * the one-workgroup solve of grids of at most 4000 points); the solve stops
 * at the exact sweep, with the same iterate for every plan. */
typedef enum { SRJ_TOL_RELATIVE = 0, SRJ_TOL_ABSOLUTE = 1, SRJ_TOL_UPDATE_INF = 2 } srj_tol_mode;

#define SRJ_NUM_LEVELS 25
#define SRJ_MAX_M 2362

typedef struct {
    int32_t ndim;          /* 1, 2 or 3 */
    int64_t n[3];          /* interior sizes, >= 1; n[d] == 1 for d >= ndim; n[1], n[2]
                              <= 65535 (srj_setup); n[0] n[1] n[2] <= 2^38 */
    double cconst[3];      /* coupling on axis d when face[d] == NULL, finite, >= 0 */
    const double *face[3]; /* optional device array: coupling between p and p + e_d */
    double dconst;         /* diagonal when diag == NULL; must be > 0 */
    const double *diag;    /* optional device array: diagonal D (> 0) */
    const double *b;       /* device array: right-hand side (required) */
} srj_problem;

typedef struct {
    srj_rule rule;
    int32_t fixed_level;      /* SRJ_RULE_FIXED only, 0..24 */
    srj_tol_mode tol_mode;
    double tol;               /* > 0 */
    int32_t max_cycles;       /* >= 1 */
    int64_t max_sweeps;       /* >= 1 */
    srj_precision precision;
    int32_t start_level;      /* first cycle's level, 0..max_level */
    int32_t max_level;        /* highest level the rules may choose, 0..24 */
    double scale_target;      /* refinement: target RMS of the scaled residual (0 = default) */
    double r0;                /* resume: reference norm for SRJ_TOL_RELATIVE (<= 0: computed) */
} srj_solve_opts;

typedef struct {
    int32_t converged;
    int32_t cycles;
    int32_t final_level;      /* level of the last cycle run */
    int32_t reserved;
    int64_t sweeps;           /* relaxation sweeps run (sum of M over cycles) */
    double r0;                /* initial (or resumed reference) residual norm */
    double r_final;           /* residual norm after the last cycle */
    double min_margin;        /* min |ratio - 0.2|, |ratio - 0.4| over selector calls */
} srj_solve_result;

/* Fill opts with defaults: heuristic rule, relative tolerance 1e-10,
 * max_cycles 10000, max_sweeps 5e7, binary64, start level 0, max level 24. */
void srj_default_opts(srj_solve_opts *opts);

/* Relaxation factors of scheme `level` (Appendix B level, Eq. (17)
 * factors) in the order a cycle applies them: Leja order of the roots
 * 1 - 1/w_j of the amplification polynomial, largest factor first (section 2,
 * last paragraph, which cycles the factors for robustness to round-off).
 * Writes min(M, cap) values to omega_out (host memory) and M to *M_out.
 * SRJ_ERR_INVALID if level is outside 0..24 or a pointer is NULL. */
srj_status srj_scheme(int32_t level, double *omega_out, int32_t cap, int32_t *M_out);

/* Create a solver context for problem *p (section 2, Eq. 1).  Validates
 * the description (ndim, sizes, dconst > 0 when diag is NULL, b != NULL),
 * allocates workspaces and precomputes 1/D on the device.  hip_stream is a
 * hipStream_t (NULL: null stream).  On success *out owns the workspaces. */
srj_status srj_setup(const srj_problem *p, void *hip_stream, srj_ctx **out);

/* General sparse matrices (the random tridiagonal matrices of section
 * 4.2.1 and the finite element systems of section 4.2.4): A in CSR form, all
 * DEVICE arrays.  Every row holds its diagonal exactly once, with a value >
 * 0; the other entries may have any sign.  One sweep evaluates, per row,
 *   s = A_pp x_p;  for the row's other entries in storage order: s += A_pq x_q;
 *   x'_p = x_p + w * ((1 / A_pp) * (b_p - s))
 * in binary64 without contraction (a stencil written this way, entries
 * A_pq = -c in the stencil's neighbour order, gives the stencil's bits).  The
 * library copies the matrix and b at setup (the caller may free them after).
 * Such a context runs one sweep per launch (or the whole solve in one
 * workgroup for at most 4000 rows), binary64 only, with the residual tests;
 * srj_collect accepts it too. */
typedef struct {
    int64_t n;              /* rows = unknowns */
    const int64_t *rowptr;  /* n + 1 entries, rowptr[0] = 0, non-decreasing */
    const int32_t *col;     /* rowptr[n] column indices in 0 .. n - 1 */
    const double *val;      /* rowptr[n] finite entries */
    const double *b;        /* n right-hand side values */
} srj_csr_problem;

/* Context for a general sparse matrix.  Validates the structure on the host
 * (SRJ_ERR_INVALID: rowptr not starting at 0 or decreasing, a column out of
 * range, a row without its diagonal or with it twice, a diagonal <= 0, a
 * non-finite entry) after synchronising hip_stream. */
srj_status srj_setup_csr(const srj_csr_problem *p, void *hip_stream, srj_ctx **out);

/* Replaces the context's scheme family (host arrays, copied): level l has
 * M[l] factors, omegas holds the factors of level 0, then level 1, ... each
 * in the order a cycle applies them.  nlevels = 0 restores the paper's family
 * (Appendix B levels, Eq. (17) factors in the library's execution order, as
 * srj_scheme returns them).  Later solves clamp max_level to nlevels - 1;
 * a start or fixed level beyond it, or a run_cycle level beyond it, is
 * SRJ_ERR_INVALID.  Batched solves always use the paper's family.
 * Synchronises the context's stream.  SRJ_ERR_INVALID for nlevels outside
 * 0..25, M[l] outside 1..2^20, more than 2^24 factors or a non-finite
 * factor. */
srj_status srj_set_scheme_family(srj_ctx *ctx, int32_t nlevels, const int32_t *M,
                                 const double *omegas);

/* One SRJ cycle (section 2, Eq. 7) of scheme `level` on the device array x
 * (in/out, n0*n1*n2 binary64), followed by the L2 norm of b - A x written to
 * *resnorm_out (host).  Blocks until *resnorm_out is valid. */
srj_status srj_run_cycle(srj_ctx *ctx, double *x, int32_t level, double *resnorm_out);

/* L2 norm of b - A x for the device array x (host result, blocking). */
srj_status srj_residual_norm(srj_ctx *ctx, const double *x, double *norm_out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the L2 norm
 * of b - A x, as srj_residual_norm computes it, without a context and
 * without any allocation.  *p is a stencil problem as for srj_setup (its
 * device arrays are only read during the call's kernels); x (n0*n1*n2
 * binary64) and norm_out (one binary64) are DEVICE pointers of the current
 * device.  The norm is written to *norm_out on the device by work enqueued on
 * hip_stream (a hipStream_t, NULL: null stream); the call does not
 * synchronise, so *norm_out is valid once that stream has reached it.
 * Partial sums go to a fixed 2 MiB device array that each GPU holds from the
 * first call until the process ends: grids needing more than 2^18 partial
 * sums return SRJ_ERR_UNSUPPORTED: one partial per 256 columns x 4 rows of
 * a plane, 8 * ceil(n0 / 256) * ceil(ceil(n1 / 8) / 4) * n2 of them when
 * n1 >= 64, else ceil(n0 / 256) * ceil(n1 / 4) * n2 (16384^2 and 512^3
 * fit).  Every call
 * on one GPU shares that array, so calls whose work overlaps on one GPU (two
 * streams, two threads) race: order them on one stream.  Validation as
 * srj_setup, plus x and norm_out (SRJ_ERR_INVALID). */
srj_status srj_residual_norm_noalloc(const srj_problem *p, const double *x, void *hip_stream,
                                     double *norm_out);

/* Solve A x = b from the initial guess in x (device, in/out) with cycles
 * whose schemes the rule picks (Algorithm 1 by default), until the stopping
 * test of opts->tol_mode holds (see srj_tol_mode) or a cap is reached; with
 * SRJ_TOL_UPDATE_INF, res->sweeps counts the sweeps up to the one that met
 * the test and x holds that sweep's iterate.  levels_out (host, max_cycles entries) receives the level of each
 * cycle and norms_out (host, max_cycles + 1 entries) the initial norm and
 * each cycle-end norm; either may be NULL.  Returns SRJ_OK when converged,
 * SRJ_ERR_NOT_CONVERGED at a cap and SRJ_ERR_NONFINITE on a NaN/Inf norm,
 * with *res filled in every one of these cases.
 * With the environment variable SRJ_LOG set (1 or "stderr": standard error;
 * any other value except 0: a file appended to), a solve that ends with one
 * of those statuses writes one line per cycle (level, its sweeps M, norm,
 * ratio to the previous norm, -log(ratio) / M) and a summary line, formed
 * from the histories after the solve (srj_mg_solve does the same per
 * V-cycle). */
srj_status srj_solve(srj_ctx *ctx, double *x, const srj_solve_opts *opts, srj_solve_result *res,
                     int32_t *levels_out, double *norms_out);

/* Kernel plans of a context (tuning only: every plan gives bit-identical
 * iterates).  which = 0 selects the plan of the binary64 sweeps, which = 1
 * the plan of the inner sweeps of the refinement modes.  kind 0: one sweep
 * per launch, any problem.  kind 1: 2D constant-coefficient register tiles of
 * 64 columns x tile_rows rows fusing up to sweeps_per_launch sweeps per launch
 * (right-hand side in registers); kind 2 (binary64 only): the same with the
 * right-hand side in LDS; kind 3: 3D, one sweep per launch, each thread
 * streaming tile_rows planes along axis 2 (any coefficients); kind 5: 2D
 * constant-coefficient wavefront strips of 64 columns x tile_rows output rows
 * that push every loaded row through up to sweeps_per_launch sweeps; kind 6:
 * 3D, one sweep per launch, register plane tiles of 64 columns x tile_rows
 * rows streamed over waves_per_simd planes along axis 2 (for kind 6 that
 * field is the plane-chunk length; all faces and a diagonal array, or all
 * constant); kind 7: 2D constant-coefficient blocks of waves_per_simd
 * cooperating waves (for kinds 7 and 8 that field is the number of waves
 * per block), each wave holding tile_rows rows of 64 columns, fusing up to
 * sweeps_per_launch sweeps per launch with the halo paid once per block;
 * kind 8: the same with two adjacent columns per lane (128-column blocks);
 * kind 10: the blocks of kind 7 for 2D grids with both per-face coupling
 * arrays and a per-point diagonal, one column per lane; kind 11: 3D with
 * constant couplings and diagonal, two sweeps per launch (sweeps_per_launch
 * 1 or 2) in plane tiles of 60 written columns x tile_rows rows streamed
 * over waves_per_simd planes (that field is the chunk length, as for kind 6);
 * kind 12: the same for 3D with all faces and a diagonal array.
 * Otherwise waves_per_simd is the register budget the kernel was compiled
 * for.  SRJ_ERR_UNSUPPORTED if the problem cannot use the plan.  Defaults at
 * setup, binary64: 2D constant-coefficient grids of at least 64 x 64 take
 * kind 8 (8 rows, 10 sweeps, 8 waves) when they hold at least 512 blocks of
 * 108 x 44 written points, else kind 7 (8 rows, 8 sweeps, 8 waves); 2D
 * per-face grids of at least 64 x 64 take kind 10, (8 rows, 8 sweeps, 8
 * waves) when they hold at least 1024 blocks of 48 x 48 written points, else
 * (4 rows, 12 sweeps, 16 waves); 3D with constant coefficients takes kind
 * 11 (4 rows, 2 sweeps, 8-plane chunks), 3D with all faces and a diagonal
 * array kind 12 (4 rows, 2 sweeps, 16-plane chunks where that still gives
 * 4096 tiles of 60 columns x 4 rows x 16 planes, else 8), other 3D layouts kind
 * 3; anything else kind 0.  Inner sweeps: the same with kind 7 in place of
 * kind 8, kind 10 always (8 rows, 8 sweeps, 8 waves) and kind 11 with 8
 * rows. */
srj_status srj_set_plan(srj_ctx *ctx, int32_t which, int32_t kind, int32_t tile_rows,
                        int32_t sweeps_per_launch, int32_t waves_per_simd);
srj_status srj_get_plan(srj_ctx *ctx, int32_t which, int32_t *kind, int32_t *tile_rows,
                        int32_t *sweeps_per_launch, int32_t *waves_per_simd);
/* Small grids (at most 4000 points): with resident mode on (the default
 * when the grid fits), a binary64 srj_solve runs entirely inside one
 * workgroup of one kernel launch: sweeps in LDS, the residual norm, Algorithm
 * 1 and the stop test on the device, no host round trip per cycle.  Iterates
 * are bit-identical to the multi-kernel path; norms may differ in the last
 * bits (summation order).  SRJ_ERR_UNSUPPORTED to enable it on a larger grid. */
srj_status srj_set_resident(srj_ctx *ctx, int32_t enable);

/* Lists the fused variants for `which` as 4 int32 each (kind, tile_rows, most
 * sweeps per launch, waves_per_simd): writes up to cap of them to out (host)
 * and their number to *count. */
srj_status srj_plan_variants(int32_t which, int32_t *out, int32_t cap, int32_t *count);

/* Autotuner: times every plan for `which` (0: binary64 sweeps, 1: inner
 * sweeps of the refinement modes) that fits this problem, `sweeps` sweeps
 * each on library scratch buffers (x is not touched), with HIP events on the
 * context's stream; sets the fastest and writes its time per sweep (us) to
 * *best_us_per_sweep.  With use_cache != 0 and the environment variable
 * SRJ_TUNE_CACHE naming a file, a plan cached for the same GPU architecture,
 * CU count and problem shape class is reused without timing, and new choices
 * are stored there.  Results never depend on the plan. */
srj_status srj_autotune(srj_ctx *ctx, int32_t which, int32_t sweeps, int32_t use_cache,
                        double *best_us_per_sweep);

/* Profiling aid.  While enabled, the relaxation launches of every cycle
 * are bracketed by HIP events recorded on the context's stream; the elapsed
 * times (ms), the number of sweep launches and of sweeps are accumulated.
 * Enabling (or re-enabling) clears the totals. */
srj_status srj_set_profiling(srj_ctx *ctx, int32_t enable);
srj_status srj_get_profile(srj_ctx *ctx, double *sweep_ms, int64_t *launches, int64_t *sweeps);

/* Release a context and its workspaces (NULL is accepted). */
srj_status srj_destroy(srj_ctx *ctx);

/* Batched solves: `count` independent problems (each described as for
 * srj_setup, constant couplings and diagonal only; 1D, 2D and 3D may be
 * mixed), advanced together with per-instance scheme choice (Algorithm 1),
 * stopping and caps.  The b arrays are copied into packed device storage at
 * setup (the caller may free them afterwards).  The batch runs on its own
 * stream; calls synchronise with hip_stream before reading caller memory.
 * SRJ_ERR_UNSUPPORTED for per-face couplings or a per-point diagonal. */
srj_status srj_batch_setup(int32_t count, const srj_problem *probs, void *hip_stream,
                           srj_batch **out);

/* Kernel plan of a batch.  With waves_per_block = 1, 2D/1D instances use
 * single-wave register tiles of 64 columns x tile_rows rows (16, 24, 32 or
 * 48) fusing up to sweeps_per_launch sweeps per step (at most 2, 4, 4/6 or
 * 8); with waves_per_block > 1 they use blocks of that many cooperating waves
 * of tile_rows rows each (the shapes of plan kind 7: (8, 8 waves, up to 4 or
 * 8 sweeps), (12, 8 waves, 8), (16, 4 waves, 8)).  3D instances advance one
 * plane-tile sweep per step.  steps_per_graph steps are captured in one
 * hipGraph (use_graph = 1) or enqueued directly (use_graph = 0).  Iterates do
 * not depend on the plan. */
srj_status srj_batch_set_plan(srj_batch *batch, int32_t tile_rows, int32_t sweeps_per_launch,
                              int32_t waves_per_block, int32_t steps_per_graph, int32_t use_graph);
srj_status srj_batch_get_plan(srj_batch *batch, int32_t *tile_rows, int32_t *sweeps_per_launch,
                              int32_t *waves_per_block, int32_t *steps_per_graph,
                              int32_t *use_graph);

/* Solve every instance from its initial guess xs[i] (device, in/out, the
 * instance's n0*n1*n2 binary64 values).  opts applies to every instance
 * (relative tolerances use each instance's own r0).  res[count] (host)
 * receives each instance's counters; levels_out (host, count * max_cycles,
 * may be NULL) the level of each of its cycles.  Returns SRJ_OK if every
 * instance converged, else the first non-OK status among the instances (all
 * results filled).  Blocks until done. */
srj_status srj_batch_solve(srj_batch *batch, double *const *xs, const srj_solve_opts *opts,
                           srj_solve_result *res, int32_t *levels_out);

/* ---- Training data for the scheme selector (section 3) ----------------
 *
 * Data collection as in section 3: a trial starts from x = 0 and applies one
 * level-0 cycle; then, at every step, the cycles of the levels one up, the
 * same and one down (those within 0..max_level) are each applied to a copy
 * of the current iterate, and one of them is taken at random.  Every branch
 * is recorded with the state it started from (the current level and the
 * residual ratio of the previous cycle) and the L2 residual norms before and
 * after its cycle; the average convergence rate of the branch is
 * -log(r_after / r_before) / M.  A trial ends once the residual norm of the
 * iterate falls below tol (the paper uses 1e-8), or after max_steps steps. */
typedef struct {
    int32_t trial;       /* trial index */
    int32_t step;        /* step within the trial (0 = the first step after the level-0 start) */
    int32_t level;       /* state: scheme level before the step */
    int32_t action;      /* +1 (level up), 0 (same level), -1 (level down) */
    int32_t M;           /* factors of the branch's level; 0: action not available (no data) */
    int32_t chosen;      /* 1 for the branch the trial continued with */
    double prev_ratio;   /* state: residual ratio (after / before) of the previous cycle */
    double r_before;     /* L2 residual norm of the iterate before the cycle */
    double r_after;      /* L2 residual norm after the branch's cycle */
} srj_sample;

/* Runs `trials` independent trials on the context's problem (at most 1024
 * grid points; x0 = 0; one workgroup per trial with the grid in LDS) and
 * writes their samples to DEVICE memory: samples[(t * max_steps + s) * 3 + j]
 * holds trial t, step s, action 1 - j (slots of actions that are not
 * available have M = 0); steps[t] (DEVICE) receives the number of steps
 * trial t took, and slots of later steps are left untouched.  u (DEVICE,
 * trials * max_steps binary64 values in [0, 1)) supplies the random draws:
 * step s of trial t takes available action floor(u[t * max_steps + s] * k)
 * of the k available ones, in the order up, same, down.  Samples are
 * bit-identical to a sequential reference (the library's sweep expression;
 * every norm sums its squares in index order).  Synchronises the context's
 * stream before returning.  SRJ_ERR_UNSUPPORTED for more than 1024 points;
 * SRJ_ERR_INVALID for bad counts, tol <= 0 or max_level outside 0..24. */
srj_status srj_collect(srj_ctx *ctx, int32_t trials, int32_t max_steps, const double *u, double tol,
                       int32_t max_level, srj_sample *samples, int32_t *steps);

#define SRJ_ACTION_NONE 2 /* srj_cluster.best when no action is confidently best */

typedef struct {
    int32_t level;        /* scheme level (state) of the cluster's samples */
    int32_t count;        /* samples in the cluster (= n_set) */
    double mean_ratio;    /* mean previous residual ratio of the cluster */
    int32_t best;         /* best action (+1, 0, -1), or SRJ_ACTION_NONE */
    int32_t n[3];         /* samples per action; index 0: up, 1: same, 2: down */
    double mean_rate[3];  /* mean average convergence rate per action */
    double half_width[3]; /* confidence half-width z * s / sqrt(n) (infinite for n < 2) */
} srj_cluster;

/* Post-processing of section 3 (host memory in and out, no GPU work):
 * usable samples (M > 0, positive finite norms) are grouped by level, sorted
 * by prev_ratio (stable, so ties keep input order) and cut into consecutive
 * clusters of n_set samples (a trailing partial cluster is dropped; the
 * paper uses n_set = 10000).  Per cluster and action: the mean rate and the
 * half-width z * s / sqrt(n) of its confidence interval (z = 1.96 for 95 %).
 * The action with the largest mean rate is the cluster's best if its
 * interval lies strictly above the interval of every other action present;
 * otherwise best = SRJ_ACTION_NONE.  Writes up to cap clusters (levels
 * ascending, ratios ascending) and their total number to *n_out. */
srj_status srj_cluster_samples(const srj_sample *samples, int64_t count, int32_t n_set, double z,
                               srj_cluster *out, int32_t cap, int32_t *n_out);

/* Fits the rule of Algorithm 1 (host memory): over the clusters with a best
 * action, sorted by mean_ratio, chooses thresholds t_low <= t_high (halfway
 * between neighbouring clusters) for "ratio > t_high: up; t_low < ratio <
 * t_high: down; otherwise same" that agree with the most clusters (the
 * first such split in ascending order).  *agree: clusters the rule agrees
 * with; *decided: clusters with a best action. */
srj_status srj_fit_rule(const srj_cluster *clusters, int32_t count, double *t_low, double *t_high,
                        int32_t *agree, int32_t *decided);

/* 3D plane tile of a batch: 3D instances are swept by waves that each own
 * tile_rows rows of 62 written columns (sweeps = 1) or 60 (sweeps = 2) and
 * walk `planes` planes along axis 2; with sweeps = 2 each step applies the
 * next two sweeps of an instance's cycle in one pass (one when a single
 * sweep is left).  (tile_rows, planes) in {(2, 16), (4, 8), (4, 16), (8, 8),
 * (8, 16)}; default (4, 8) with 2 sweeps.  SRJ_ERR_UNSUPPORTED for any other
 * shape, SRJ_ERR_INVALID for sweeps other than 1 or 2.  Iterates do not
 * depend on the plan. */
srj_status srj_batch_set_plan3d(srj_batch *batch, int32_t tile_rows, int32_t planes,
                                int32_t sweeps);
srj_status srj_batch_get_plan3d(srj_batch *batch, int32_t *tile_rows, int32_t *planes,
                                int32_t *sweeps);

/* Batch autotuner: for `precision`, times every tile or block plan of the
 * batch's 2D/1D instances (when it has any; `sweeps` sweeps of them) and then
 * every 3D plane tile (when it has 3D instances; `sweeps` steps, one sweep of
 * every 3D instance each), from x0 = 0 on the batch's own buffers (no caller
 * memory is touched), and sets the fastest of each.  *best_us_per_sweep: the
 * time per sweep of the 2D/1D instances, or, when the batch has 3D instances,
 * the time per step.  Iterates do not depend on the choice. */
srj_status srj_batch_autotune(srj_batch *batch, int32_t precision, int32_t sweeps,
                              double *best_us_per_sweep);

srj_status srj_batch_destroy(srj_batch *batch);

/* SRJ as the smoother of a geometric multigrid V-cycle (section 5 names
 * SRJ as a candidate multigrid smoother; the paper gives no design, so the
 * following is this library's reading).  For constant-coefficient stencil
 * problems whose active sizes are odd: level l + 1 halves every active axis,
 * n' = (n - 1) / 2, while all active sizes are odd and >= 3, with couplings
 * and diagonal divided by 4 (rediscretisation on the doubled spacing).  One
 * V-cycle on level l: `pre` SRJ cycles of the current scheme (section 2,
 * Eq. 7), the residual restricted by full weighting (weights 1/4, 1/2, 1/4
 * per axis), the coarse correction from zero by the V-cycle on level l + 1,
 * multilinear interpolation of it added to x, `post` SRJ cycles.  The
 * coarsest level used is solved by SRJ with Algorithm 1 from zero to the
 * relative tolerance coarse_tol (at most coarse_max_cycles cycles).  After
 * each V-cycle the binary64 residual norm is tested (tol_mode relative or
 * absolute) and, with SRJ_RULE_HEURISTIC, the V-cycle's residual ratio picks
 * the next V-cycle's smoothing scheme by Algorithm 1 (section 3) within
 * start_level .. max_level; SRJ_RULE_FIXED keeps start_level.  Transfers and
 * smoothing evaluate fixed-order expressions without contraction, so x is
 * bit-identical to a CPU evaluation in the same order. */
typedef struct srj_mg srj_mg;
typedef struct {
    srj_rule rule;             /* SRJ_RULE_HEURISTIC or SRJ_RULE_FIXED */
    int32_t start_level;       /* smoothing scheme of the first V-cycle, 0..max_level */
    int32_t max_level;         /* highest smoothing scheme, 0..24 */
    int32_t pre, post;         /* SRJ cycles before / after the coarse correction, 0..1000 */
    int32_t max_levels;        /* grid levels used at most, >= 2 */
    double coarse_tol;         /* relative tolerance of the coarsest solve, > 0 */
    int32_t coarse_max_cycles; /* >= 1 */
    srj_tol_mode tol_mode;     /* SRJ_TOL_RELATIVE or SRJ_TOL_ABSOLUTE */
    double tol;                /* > 0 */
    int32_t max_vcycles;       /* >= 1 */
} srj_mg_opts;

typedef struct {
    int32_t converged;
    int32_t vcycles;
    int32_t final_level;       /* smoothing scheme of the last V-cycle */
    int32_t levels;            /* grid levels used */
    int64_t sweeps;            /* smoothing sweeps on the finest grid */
    int64_t coarse_sweeps;     /* SRJ sweeps of the coarsest solves */
    double work;               /* all sweeps in finest-grid sweep equivalents */
    double r0, r_final;        /* residual norms before the first and after the last V-cycle */
} srj_mg_result;

/* Defaults: heuristic, start level 0, max level 24, one pre- and one post-
 * cycle, up to 32 grid levels, coarsest solve to 1e-8 (1000 cycles), relative
 * tolerance 1e-10, 200 V-cycles. */
void srj_mg_default_opts(srj_mg_opts *opts);

/* Builds the level hierarchy for *p (device arrays as for srj_setup; b is
 * borrowed, the coarse levels' arrays and contexts are owned by *out).
 * SRJ_ERR_UNSUPPORTED for per-face couplings or a diagonal array, or a grid
 * that cannot be coarsened once; SRJ_ERR_INVALID as srj_setup. */
srj_status srj_mg_setup(const srj_problem *p, void *hip_stream, srj_mg **out);

/* V-cycles from the initial guess in x (device, in/out) until the residual
 * test holds or max_vcycles.  levels_out (host, max_vcycles entries): the
 * smoothing scheme of each V-cycle; norms_out (host, max_vcycles + 1): the
 * initial norm and each V-cycle's; either may be NULL.  Returns SRJ_OK,
 * SRJ_ERR_NOT_CONVERGED at the cap or SRJ_ERR_NONFINITE, with *res filled;
 * blocks until x is valid. */
srj_status srj_mg_solve(srj_mg *mg, double *x, const srj_mg_opts *opts, srj_mg_result *res,
                        int32_t *levels_out, double *norms_out);
srj_status srj_mg_destroy(srj_mg *mg);

/* Measurement aid, not a step of the method: one launch of a streaming
 * kernel of known traffic on hip_stream (no synchronisation), the ceiling
 * that sweep kernels' byte rates are quoted against and the reference
 * dispatch for hardware byte counters.  kind 0: out[i] = a[i] (8 B read and
 * 8 B written per value); kind 1: out[i] = a[i] + b[i] (16 B read, 8 B
 * written: the mix of a one-sweep launch; b unused for kind 0).  a, b, out:
 * DEVICE arrays of n binary64 values, 16-byte aligned, of the current device.
 * SRJ_ERR_INVALID for another kind, n odd, n < 2 or n > 2^36, or an array
 * that is not device memory. */
srj_status srj_stream_probe(int32_t kind, const double *a, const double *b, double *out, int64_t n,
                            void *hip_stream);

const char *srj_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* SRJ_H */
