/*
 * srj_oracle.h - CPU reference implementation of the Scheduled Relaxation
 * Jacobi (SRJ) method with the data-driven scheme selector of Islam & Wang,
 * "A data driven heuristic for rapid convergence of Scheduled Relaxation
 * Jacobi schemes" (arXiv 2011.06636).
 *
 * TEST INFRASTRUCTURE ONLY.  This header and srj_oracle.c are the slow,
 * plain reference that the GPU library is checked against.  They share no
 * code, header, table or constant with the GPU library, and the library never
 * links, loads or calls them.
 *
 * Grid convention: interior grid n[0] x n[1] x n[2] (unused axes = 1), axis 0
 * contiguous, flat index p = i0 + n0*(i1 + n1*i2).  Homogeneous Dirichlet:
 * the ghost layer is zero and not stored.
 */
#ifndef SRJ_ORACLE_H
#define SRJ_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* A = D + L + U (section 2, Eq. 1) as a symmetric stencil.
 * A[p][p] = diag ? diag[p] : dconst.
 * A[p][p+e_d] = A[p+e_d][p] = -(face[d] ? face[d][p] : c[d]). */
typedef struct {
    int32_t ndim;
    int64_t n[3];
    double c[3];
    const double *face[3];
    double dconst;
    const double *diag;
    const double *b;
    /* General sparse matrix instead of a stencil (ndim = 1, n[0] rows): CSR
     * arrays; every row holds its diagonal once.  NULL rowptr: stencil. */
    const int64_t *rowptr;
    const int32_t *col;
    const double *val;
} srjo_problem;

enum { SRJO_RULE_HEURISTIC = 0, SRJO_RULE_INCREASING = 1, SRJO_RULE_FIXED = 2,
       SRJO_RULE_JACOBI = 3 };
/* RELATIVE: cycle-end ||b - A x||_2 < tol * r0 (Eq. (27)); ABSOLUTE:
 * cycle-end ||b - A x||_2 < tol (section 4.1); UPDATE_INF: after every
 * sweep, max_p |x'_p - x_p| < tol (section 4.2.2, Eq. (25)), binary64 only. */
enum { SRJO_TOL_RELATIVE = 0, SRJO_TOL_ABSOLUTE = 1, SRJO_TOL_UPDATE_INF = 2 };
enum { SRJO_PREC_F64 = 0, SRJO_PREC_F32 = 1, SRJO_PREC_F16 = 2, SRJO_PREC_BF16 = 3 };
enum { SRJO_OK = 0, SRJO_INVALID = 1, SRJO_NOT_CONVERGED = 4, SRJO_NONFINITE = 5 };

typedef struct {
    int32_t rule;           /* SRJO_RULE_* */
    int32_t fixed_level;    /* level used by SRJO_RULE_FIXED */
    int32_t tol_mode;       /* SRJO_TOL_* */
    double tol;
    int32_t max_cycles;
    int64_t max_sweeps;
    int32_t stop_per_sweep; /* 1: test the residual after every sweep (F64 only) */
    int32_t precision;      /* SRJO_PREC_*: inner-cycle precision of the refinement */
    int32_t start_level;
    int32_t max_level;      /* highest selectable level (<= 24) */
    double scale_target;    /* refinement: target RMS of the scaled residual */
} srjo_opts;

typedef struct {
    int32_t status;
    int32_t converged;
    int32_t cycles;
    int32_t final_level;
    int64_t sweeps;
    double r0;
    double r_final;
    double min_margin;      /* min |ratio - 0.2|, |ratio - 0.4| over selector calls */
} srjo_result;

int32_t srjo_num_levels(void);
int32_t srjo_level_M(int32_t level);
/* Eq. (17): relaxation factors of the length-M scheme in natural root order. */
void srjo_omega_natural(int32_t M, double *w);
/* Execution order of a scheme: a permutation of 0..M-1 (section 2, last paragraph). */
void srjo_leja_order(int32_t M, const double *w, int32_t *order);
/* Factors of a level in execution order; returns M. */
int32_t srjo_scheme(int32_t level, double *w_out);

/* One relaxed Jacobi sweep (Eq. 3, residual form), x_out must not alias x. */
void srjo_sweep(const srjo_problem *p, const double *x, double w, double *x_out);
/* ||b - A x||_2 with the sum taken sequentially in index order. */
double srjo_residual_norm(const srjo_problem *p, const double *x);
/* y = A x */
void srjo_apply(const srjo_problem *p, const double *x, double *y);

/* Solve to tolerance.  levels_out[max_cycles] and norms_out[max_cycles+1]
 * may be NULL.  norms_out[0] is the initial residual norm. */
int32_t srjo_solve(const srjo_problem *p, double *x, const srjo_opts *o,
                   srjo_result *res, int32_t *levels_out, double *norms_out);

/* Section 3, data collection for the scheme selector.  One record per
 * branch; field meanings as in the paper's tuples (state: level and the
 * residual ratio of the previous cycle; action; residual norms before and
 * after the branch's cycle, from which the average convergence rate
 * -log(r_after / r_before) / M follows). */
typedef struct {
    int32_t trial;
    int32_t step;
    int32_t level;
    int32_t action;      /* +1, 0, -1 */
    int32_t M;           /* 0: action not available at this level */
    int32_t chosen;
    double prev_ratio;
    double r_before;
    double r_after;
} srjo_sample;

/* trials independent trials from x = 0 (one level-0 cycle first), at most
 * max_steps steps each, until the residual norm falls below tol; step s of
 * trial t takes available action floor(u[t * max_steps + s] * k) of the k
 * available ones (order: up, same, down).  out[(t * max_steps + s) * 3 + j]
 * receives the branch of action 1 - j; steps[t] the steps taken. */
void srjo_collect(const srjo_problem *p, int32_t trials, int32_t max_steps, const double *u,
                  double tol, int32_t max_level, srjo_sample *out, int32_t *steps);

/* SRJ as the smoother of a geometric multigrid V-cycle (srj_mg.c; section 5
 * names the use, the design is this library's reading).  Constant-coefficient
 * stencils only; every active axis of the fine grid is halved, n' = (n-1)/2,
 * while all active sizes are odd and >= 3 (at least two levels needed). */
typedef struct {
    int32_t rule;              /* SRJO_RULE_HEURISTIC or SRJO_RULE_FIXED: smoothing scheme */
    int32_t start_level;       /* smoothing scheme of the first V-cycle */
    int32_t max_level;         /* highest smoothing level the selector may choose */
    int32_t pre, post;         /* SRJ cycles before and after the coarse-grid correction */
    int32_t max_levels;        /* grid levels at most (>= 2) */
    double coarse_tol;         /* coarsest grid: SRJ with the selector from 0 to this relative tol */
    int32_t coarse_max_cycles;
    int32_t tol_mode;          /* SRJO_TOL_RELATIVE or SRJO_TOL_ABSOLUTE, after each V-cycle */
    double tol;
    int32_t max_vcycles;
} srjo_mg_opts;

typedef struct {
    int32_t status, converged, vcycles, final_level, levels;
    int64_t sweeps;          /* fine-grid smoothing sweeps */
    int64_t coarse_sweeps;   /* coarsest-grid SRJ sweeps */
    double work;             /* all sweeps in fine-sweep equivalents (points / fine points) */
    double r0, r_final;
} srjo_mg_result;

int32_t srjo_mg_hierarchy(const srjo_problem *p, int32_t max_levels, int64_t *dims_out);
/* bc = R (b - A x), full weighting, coarse grid of the hierarchy's next level */
void srjo_restrict_residual(const srjo_problem *p, const double *x, double *bc);
/* x += P ec, multilinear interpolation from the next level's grid */
void srjo_prolong_add(const srjo_problem *p, const double *ec, double *x);
/* V-cycles until the residual test holds; levels_out[max_vcycles] receives
 * the smoothing level of each V-cycle, norms_out[max_vcycles + 1] the
 * initial norm and each V-cycle's. */
int32_t srjo_mg_solve(const srjo_problem *p, double *x, const srjo_mg_opts *o,
                      srjo_mg_result *res, int32_t *levels_out, double *norms_out);

/* Storage roundings used by the 16-bit refinement modes. */
float srjo_round_f16(float v);
float srjo_round_bf16(float v);
int32_t srjo_num_threads(void);
void srjo_set_num_threads(int32_t n);

#ifdef __cplusplus
}
#endif
#endif
