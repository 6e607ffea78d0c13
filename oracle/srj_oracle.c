/*
 * srj_oracle.c - CPU reference of the SRJ method with the data-driven scheme
 * selector (Islam & Wang, arXiv 2011.06636).
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the CPU
 * baseline of the benchmark.  The GPU library never links or calls it, and
 * it shares no code with the library.
 *
 * Everything here is written to be checked by eye against the paper:
 *   - scheme family: section 2, Eq. (13)-(17) and Appendix B;
 *   - execution order of a scheme's factors: section 2, last paragraph
 *     (reading: Leja order of the roots, largest factor first);
 *   - one relaxed Jacobi sweep: section 2, Eq. 3 (written in residual form,
 *     x + w D^-1 (b - A x), which is the same update);
 *   - one SRJ cycle: M sweeps with the scheme's factors (section 2, Eq. 7);
 *   - residual: L2 norm of b - A x after each cycle (section 3) and the
 *     relative residual of section 4.2.3, Eq. (27);
 *   - selector: section 3, Algorithm 1;
 *   - training data for the selector: section 3, data collection (three
 *     branches per step from the same iterate, one taken at random).
 * Arithmetic: IEEE binary64 (binary32 for the inner cycles of the
 * refinement modes, which are not in the paper), round to nearest even, no
 * contraction into fused multiply-add (-ffp-contract=off), no fast-math.
 * The only parallelism is an OpenMP loop over independent grid points inside
 * a sweep, and one over independent trials of the data collection; sums are
 * always taken sequentially in index order.
 */
#include "srj_oracle.h"

#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Sweeps over fewer points than this run on one thread. */
#define PAR_MIN_POINTS 65536

/* Appendix B: scheme level -> number of factors M. */
static const int32_t LEVEL_M[25] = {1,   2,   3,   5,   7,   10,  14,   19,   26,
                                    35,  47,  63,  84,  111, 147, 194,  256,  338,
                                    446, 589, 778, 1027, 1356, 1790, 2362};

int32_t srjo_num_levels(void) { return 25; }

int32_t srjo_level_M(int32_t level)
{
    if (level < 0 || level > 24) return -1;
    return LEVEL_M[level];
}

int32_t srjo_num_threads(void)
{
#ifdef _OPENMP
    return (int32_t)omp_get_max_threads();
#else
    return 1;
#endif
}

/* Thread count of later parallel loops (timing only: the sums that the
 * results depend on are sequential, so results do not depend on it). */
void srjo_set_num_threads(int32_t n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads((int)n);
#else
    (void)n;
#endif
}

/* Eq. (17): omega_j = (l* + 1) / (2 (l* - x_j)), j = 0..M-1, where
 * x_j = cos((2j+1) pi / (2M)) are the roots of the Chebyshev polynomial T_M
 * and l* is the real root > 1 of T_M(l*) = 3, i.e. cosh(arccosh(3) / M)
 * (section 2 after Eq. (13); T_M(cosh t) = cosh(M t) for t >= 0). */
void srjo_omega_natural(int32_t M, double *w)
{
    double lstar = cosh(acosh(3.0) / (double)M);
    for (int32_t j = 0; j < M; j++) {
        double xj = cos((2.0 * j + 1.0) * M_PI / (2.0 * M));
        w[j] = (lstar + 1.0) / (2.0 * (lstar - xj));
    }
}

/* Order in which a cycle applies its factors.  The paper cycles through the
 * factors so that each step gives the largest error reduction, to stay
 * robust against round-off and overflow (section 2, last paragraph).  Reading
 * used here: Leja order of the amplification-polynomial roots
 * l_j = 1 - 1/omega_j (Eq. (15)): start with the largest factor (j = 0),
 * then repeatedly take the unused root that maximises the sum of log
 * distances to the roots already taken.  The sums are accumulated in the
 * order the roots were taken; on equal scores the lowest index wins.  This
 * reproduces the printed orders of Table 2 for M = 3, 5 and 7. */
void srjo_leja_order(int32_t M, const double *w, int32_t *order)
{
    double *root = (double *)malloc(sizeof(double) * (size_t)M);
    double *score = (double *)malloc(sizeof(double) * (size_t)M);
    char *used = (char *)calloc((size_t)M, 1);
    for (int32_t j = 0; j < M; j++) {
        root[j] = 1.0 - 1.0 / w[j];
        score[j] = 0.0;
    }
    order[0] = 0;
    used[0] = 1;
    for (int32_t step = 1; step < M; step++) {
        int32_t last = order[step - 1];
        int32_t best = -1;
        for (int32_t j = 0; j < M; j++) {
            if (used[j]) continue;
            score[j] = score[j] + log(fabs(root[j] - root[last]));
            if (best < 0 || score[j] > score[best]) best = j;
        }
        order[step] = best;
        used[best] = 1;
    }
    free(root);
    free(score);
    free(used);
}

int32_t srjo_scheme(int32_t level, double *w_out)
{
    int32_t M = srjo_level_M(level);
    if (M < 0) return -1;
    double *w = (double *)malloc(sizeof(double) * (size_t)M);
    int32_t *order = (int32_t *)malloc(sizeof(int32_t) * (size_t)M);
    srjo_omega_natural(M, w);
    srjo_leja_order(M, w, order);
    for (int32_t k = 0; k < M; k++) w_out[k] = w[order[k]];
    free(w);
    free(order);
    return M;
}

/* ---------------------------------------------------------------------- */
/* Matrix-free stencil, binary64                                            */
/* ---------------------------------------------------------------------- */

static int64_t npoints(const srjo_problem *p) { return p->n[0] * p->n[1] * p->n[2]; }

static void strides(const srjo_problem *p, int64_t st[3])
{
    st[0] = 1;
    st[1] = p->n[0];
    st[2] = p->n[0] * p->n[1];
}

static double diag_at(const srjo_problem *p, int64_t idx)
{
    if (p->rowptr) { /* the stored diagonal of the row */
        for (int64_t k = p->rowptr[idx]; k < p->rowptr[idx + 1]; k++)
            if (p->col[k] == idx) return p->val[k];
        return NAN;
    }
    return p->diag ? p->diag[idx] : p->dconst;
}

/* (A x)_p, evaluated in one fixed order: D_p x_p first, then for each axis
 * the lower neighbour and the upper neighbour.  Neighbours in the Dirichlet
 * ghost layer hold zero, so their terms are omitted. */
static double row_product(const srjo_problem *p, const double *x, int64_t idx,
                          const int64_t ii[3], const int64_t st[3])
{
    if (p->rowptr) { /* sparse row: the diagonal first, then the row in storage order */
        double s = diag_at(p, idx) * x[idx];
        for (int64_t k = p->rowptr[idx]; k < p->rowptr[idx + 1]; k++)
            if (p->col[k] != idx) s = s + p->val[k] * x[p->col[k]];
        return s;
    }
    double s = diag_at(p, idx) * x[idx];
    for (int d = 0; d < p->ndim; d++) {
        if (ii[d] > 0) {
            double cl = p->face[d] ? p->face[d][idx - st[d]] : p->c[d];
            s = s - cl * x[idx - st[d]];
        }
        if (ii[d] < p->n[d] - 1) {
            double cr = p->face[d] ? p->face[d][idx] : p->c[d];
            s = s - cr * x[idx + st[d]];
        }
    }
    return s;
}

void srjo_apply(const srjo_problem *p, const double *x, double *y)
{
    int64_t st[3];
    strides(p, st);
    for (int64_t i2 = 0; i2 < p->n[2]; i2++)
        for (int64_t i1 = 0; i1 < p->n[1]; i1++)
            for (int64_t i0 = 0; i0 < p->n[0]; i0++) {
                int64_t ii[3] = {i0, i1, i2};
                int64_t idx = i0 + p->n[0] * (i1 + p->n[1] * i2);
                y[idx] = row_product(p, x, idx, ii, st);
            }
}

/* Eq. 3 in residual form: x' = x + w D^-1 (b - A x). */
void srjo_sweep(const srjo_problem *p, const double *x, double w, double *x_out)
{
    int64_t st[3];
    strides(p, st);
    int64_t n0 = p->n[0], n1 = p->n[1], n2 = p->n[2];
#pragma omp parallel for collapse(2) schedule(static) if (n0 * n1 * n2 >= PAR_MIN_POINTS)
    for (int64_t i2 = 0; i2 < n2; i2++)
        for (int64_t i1 = 0; i1 < n1; i1++)
            for (int64_t i0 = 0; i0 < n0; i0++) {
                int64_t ii[3] = {i0, i1, i2};
                int64_t idx = i0 + n0 * (i1 + n1 * i2);
                double s = row_product(p, x, idx, ii, st);
                double r = p->b[idx] - s;
                double dinv = 1.0 / diag_at(p, idx);
                double t = dinv * r;
                x_out[idx] = x[idx] + w * t;
            }
}

/* L2 norm of b - A x, sum of squares taken sequentially in index order. */
double srjo_residual_norm(const srjo_problem *p, const double *x)
{
    int64_t st[3];
    strides(p, st);
    double sum = 0.0;
    for (int64_t i2 = 0; i2 < p->n[2]; i2++)
        for (int64_t i1 = 0; i1 < p->n[1]; i1++)
            for (int64_t i0 = 0; i0 < p->n[0]; i0++) {
                int64_t ii[3] = {i0, i1, i2};
                int64_t idx = i0 + p->n[0] * (i1 + p->n[1] * i2);
                double r = p->b[idx] - row_product(p, x, idx, ii, st);
                sum = sum + r * r;
            }
    return sqrt(sum);
}

/* Section 3, Algorithm 1 (and the comparison rules of section 4): next
 * level from the ratio of the residual norms after and before the cycle.
 * The level is kept inside the table of Appendix B. */
static int32_t next_level(int32_t rule, int32_t level, double ratio, int32_t max_level)
{
    int32_t nl = level;
    if (rule == SRJO_RULE_HEURISTIC) {
        if (ratio > 0.4)
            nl = level + 1;
        else if (ratio < 0.4 && ratio > 0.2)
            nl = level - 1;
        else
            nl = level;
    } else if (rule == SRJO_RULE_INCREASING) {
        nl = level + 1;
    }
    if (nl < 0) nl = 0;
    if (nl > max_level) nl = max_level;
    return nl;
}

static int32_t validate(const srjo_problem *p, const srjo_opts *o)
{
    if (!p || !o || !p->b) return SRJO_INVALID;
    if (p->ndim < 1 || p->ndim > 3) return SRJO_INVALID;
    for (int d = 0; d < 3; d++) {
        if (p->n[d] < 1) return SRJO_INVALID;
        if (d >= p->ndim && p->n[d] != 1) return SRJO_INVALID;
    }
    if (p->rowptr) {
        if (p->ndim != 1 || !p->col || !p->val) return SRJO_INVALID;
        for (int64_t i = 0; i < p->n[0]; i++)
            if (!(diag_at(p, i) > 0.0)) return SRJO_INVALID;
    } else if (!p->diag && !(p->dconst > 0.0)) {
        return SRJO_INVALID;
    }
    if (!(o->tol > 0.0)) return SRJO_INVALID;
    if (o->rule < 0 || o->rule > 3) return SRJO_INVALID;
    if (o->max_level < 0 || o->max_level > 24) return SRJO_INVALID;
    if (o->start_level < 0 || o->start_level > o->max_level) return SRJO_INVALID;
    if (o->rule == SRJO_RULE_FIXED && (o->fixed_level < 0 || o->fixed_level > 24))
        return SRJO_INVALID;
    if (o->precision < 0 || o->precision > 3) return SRJO_INVALID;
    if (o->tol_mode < 0 || o->tol_mode > 2) return SRJO_INVALID;
    if (o->precision != SRJO_PREC_F64 &&
        (o->stop_per_sweep || o->rule == SRJO_RULE_JACOBI || o->tol_mode == SRJO_TOL_UPDATE_INF))
        return SRJO_INVALID;
    return SRJO_OK;
}

static int32_t solve_f64(const srjo_problem *p, double *x, const srjo_opts *o,
                         srjo_result *res, int32_t *levels_out, double *norms_out);
static int32_t solve_refine(const srjo_problem *p, double *x, const srjo_opts *o,
                            srjo_result *res, int32_t *levels_out, double *norms_out);

int32_t srjo_solve(const srjo_problem *p, double *x, const srjo_opts *o, srjo_result *res,
                   int32_t *levels_out, double *norms_out)
{
    memset(res, 0, sizeof(*res));
    res->min_margin = INFINITY;
    int32_t st = validate(p, o);
    if (st != SRJO_OK) {
        res->status = st;
        return st;
    }
    if (o->precision == SRJO_PREC_F64) return solve_f64(p, x, o, res, levels_out, norms_out);
    return solve_refine(p, x, o, res, levels_out, norms_out);
}

static void track_margin(srjo_result *res, double ratio)
{
    double m = fmin(fabs(ratio - 0.2), fabs(ratio - 0.4));
    if (m < res->min_margin) res->min_margin = m;
}

static int32_t solve_f64(const srjo_problem *p, double *x, const srjo_opts *o,
                         srjo_result *res, int32_t *levels_out, double *norms_out)
{
    int64_t N = npoints(p);
    double *buf = (double *)malloc(sizeof(double) * (size_t)N);
    double *w = (double *)malloc(sizeof(double) * 2362);
    double *cur = x, *nxt = buf;

    double r0 = srjo_residual_norm(p, x);
    res->r0 = r0;
    res->r_final = r0;
    if (norms_out) norms_out[0] = r0;
    double target = (o->tol_mode == SRJO_TOL_RELATIVE) ? o->tol * r0 : o->tol;
    /* section 4.2.2, Eq. (25): stop after the first sweep whose largest
     * update max_p |x'_p - x_p| is below tol (a NaN update never passes) */
    int update_test = o->tol_mode == SRJO_TOL_UPDATE_INF;
    int32_t status = SRJO_NOT_CONVERGED;
    int32_t level = o->start_level;
    double prev = r0;

    if (!isfinite(r0)) {
        status = SRJO_NONFINITE;
        goto done;
    }
    if (r0 == 0.0 || (!update_test && r0 < target)) {
        res->converged = 1;
        status = SRJO_OK;
        goto done;
    }
    for (int32_t cycle = 0; cycle < o->max_cycles; cycle++) {
        int32_t M;
        if (o->rule == SRJO_RULE_JACOBI) {
            M = 1;
            w[0] = 1.0; /* unweighted Jacobi, Eq. 2 */
        } else {
            M = srjo_scheme(o->rule == SRJO_RULE_FIXED ? o->fixed_level : level, w);
        }
        if (res->sweeps + M > o->max_sweeps) break;
        int stopped_mid_cycle = 0, update_met = 0;
        double norm = 0.0;
        for (int32_t k = 0; k < M; k++) {
            srjo_sweep(p, cur, w[k], nxt);
            double umax = 0.0;
            if (update_test) {
                int nan_seen = 0;
                for (int64_t i = 0; i < N; i++) {
                    double d = fabs(nxt[i] - cur[i]);
                    if (isnan(d)) nan_seen = 1;
                    else if (d > umax) umax = d;
                }
                if (nan_seen) umax = NAN;
            }
            double *t = cur;
            cur = nxt;
            nxt = t;
            res->sweeps += 1;
            if (update_test && umax < o->tol) {
                update_met = 1;
                break;
            }
            if (o->stop_per_sweep && k + 1 < M) {
                double nk = srjo_residual_norm(p, cur);
                if (nk < target) {
                    norm = nk;
                    stopped_mid_cycle = 1;
                    break;
                }
            }
        }
        if (!stopped_mid_cycle) norm = srjo_residual_norm(p, cur);
        res->cycles = cycle + 1;
        res->r_final = norm;
        res->final_level = (o->rule == SRJO_RULE_FIXED) ? o->fixed_level : level;
        if (levels_out) levels_out[cycle] = (o->rule == SRJO_RULE_JACOBI) ? -1 : res->final_level;
        if (norms_out) norms_out[cycle + 1] = norm;
        if (update_met) {
            res->converged = 1;
            status = SRJO_OK;
            break;
        }
        if (!isfinite(norm)) {
            status = SRJO_NONFINITE;
            break;
        }
        if (!update_test && norm < target) {
            res->converged = 1;
            status = SRJO_OK;
            break;
        }
        double ratio = norm / prev;
        prev = norm;
        if (o->rule == SRJO_RULE_HEURISTIC) track_margin(res, ratio);
        level = next_level(o->rule, level, ratio, o->max_level);
    }
done:
    if (cur != x) memcpy(x, cur, sizeof(double) * (size_t)N);
    res->status = status;
    free(buf);
    free(w);
    return status;
}

/* ---------------------------------------------------------------------- */
/* Mixed-precision iterative refinement (not in the paper).               */
/* One outer step = one SRJ cycle on the correction equation A d = r:     */
/*   r = b - A x (binary64), rhat = storage(s * r) with s a power of two,  */
/*   d = 0, M inner sweeps on A d = rhat in binary32 arithmetic with the    */
/*   iterate rounded to the storage format after every sweep,              */
/*   x = x + d / s (binary64).                                             */
/* In exact arithmetic the error obeys e' = B_SRJ e exactly as in Eq. 7.   */
/* ---------------------------------------------------------------------- */

/* Round a binary32 value to the nearest (ties to even) value with 'mant'
 * explicit mantissa bits and minimum normal exponent 'emin', saturating to
 * infinity above 'maxval'.  Written from the definition: the spacing of
 * representable numbers near |v| is 2^(floor(log2|v|) - mant) for normal
 * numbers and 2^(emin - mant) below the normal range. */
static float round_format(float v, int mant, int emin, double maxval)
{
    if (!isfinite(v) || v == 0.0f) return v;
    double a = fabs((double)v);
    int e2;
    frexp(a, &e2);          /* a = m 2^e2, m in [0.5, 1) => floor(log2 a) = e2 - 1 */
    int e = e2 - 1;
    if (e < emin) e = emin; /* subnormal spacing */
    double q = ldexp(1.0, e - mant);
    double r = rint(a / q) * q; /* a/q is exact: q is a power of two */
    if (r > maxval) r = INFINITY;
    return (float)(v < 0.0f ? -r : r);
}

float srjo_round_f16(float v) { return round_format(v, 10, -14, 65504.0); }

float srjo_round_bf16(float v)
{
    return round_format(v, 7, -126, ldexp(255.0, 120)); /* (2 - 2^-7) * 2^127 */
}

static float store(float v, int32_t precision)
{
    if (precision == SRJO_PREC_F16) return srjo_round_f16(v);
    if (precision == SRJO_PREC_BF16) return srjo_round_bf16(v);
    return v;
}

/* Binary32 copy of the operator used by the inner cycles: every coefficient
 * is the binary64 one rounded to binary32, and D^-1 is 1/D computed in
 * binary64 and then rounded. */
typedef struct {
    float c[3];
    float *face[3];
    float *d32;
    float *dinv32;
    float dconst32, dinvconst32;
} op32;

static void op32_init(const srjo_problem *p, op32 *op)
{
    int64_t N = npoints(p);
    memset(op, 0, sizeof(*op));
    for (int d = 0; d < 3; d++) {
        op->c[d] = (float)p->c[d];
        if (p->face[d]) {
            op->face[d] = (float *)malloc(sizeof(float) * (size_t)N);
            for (int64_t i = 0; i < N; i++) op->face[d][i] = (float)p->face[d][i];
        }
    }
    if (p->diag) {
        op->d32 = (float *)malloc(sizeof(float) * (size_t)N);
        op->dinv32 = (float *)malloc(sizeof(float) * (size_t)N);
        for (int64_t i = 0; i < N; i++) {
            op->d32[i] = (float)p->diag[i];
            op->dinv32[i] = (float)(1.0 / p->diag[i]);
        }
    } else {
        op->dconst32 = (float)p->dconst;
        op->dinvconst32 = (float)(1.0 / p->dconst);
    }
}

static void op32_free(op32 *op)
{
    for (int d = 0; d < 3; d++) free(op->face[d]);
    free(op->d32);
    free(op->dinv32);
}

/* One inner sweep on A d = rhat in binary32, same expression order as the
 * binary64 sweep, result rounded to the storage format. */
static void sweep32(const srjo_problem *p, const op32 *op, const float *d, const float *rhat,
                    float w, int32_t precision, float *d_out)
{
    int64_t st[3];
    strides(p, st);
    int64_t n0 = p->n[0], n1 = p->n[1], n2 = p->n[2];
#pragma omp parallel for collapse(2) schedule(static) if (n0 * n1 * n2 >= PAR_MIN_POINTS)
    for (int64_t i2 = 0; i2 < n2; i2++)
        for (int64_t i1 = 0; i1 < n1; i1++)
            for (int64_t i0 = 0; i0 < n0; i0++) {
                int64_t ii[3] = {i0, i1, i2};
                int64_t idx = i0 + n0 * (i1 + n1 * i2);
                float dd = op->d32 ? op->d32[idx] : op->dconst32;
                float s = dd * d[idx];
                for (int k = 0; k < p->ndim; k++) {
                    if (ii[k] > 0) {
                        float cl = op->face[k] ? op->face[k][idx - st[k]] : op->c[k];
                        s = s - cl * d[idx - st[k]];
                    }
                    if (ii[k] < p->n[k] - 1) {
                        float cr = op->face[k] ? op->face[k][idx] : op->c[k];
                        s = s - cr * d[idx + st[k]];
                    }
                }
                float r = rhat[idx] - s;
                float dinv = op->dinv32 ? op->dinv32[idx] : op->dinvconst32;
                float t = dinv * r;
                d_out[idx] = store(d[idx] + w * t, precision);
            }
}

/* Largest power of two not above target_rms * sqrt(N) / norm (1 if the norm
 * is zero): scales the residual so that its RMS sits near target_rms. */
static double pow2_scale(double norm, int64_t N, double target_rms)
{
    if (!(norm > 0.0) || !isfinite(norm)) return 1.0;
    double q = target_rms * sqrt((double)N) / norm;
    int e;
    frexp(q, &e);
    return ldexp(1.0, e - 1);
}

static double default_target(int32_t precision)
{
    return precision == SRJO_PREC_F16 ? ldexp(1.0, -8) : 1.0;
}

static void scaled_residual(const srjo_problem *p, const double *x, double s, int32_t precision,
                            float *rhat, double *sumsq)
{
    int64_t st[3];
    strides(p, st);
    double sum = 0.0;
    for (int64_t i2 = 0; i2 < p->n[2]; i2++)
        for (int64_t i1 = 0; i1 < p->n[1]; i1++)
            for (int64_t i0 = 0; i0 < p->n[0]; i0++) {
                int64_t ii[3] = {i0, i1, i2};
                int64_t idx = i0 + p->n[0] * (i1 + p->n[1] * i2);
                double r = p->b[idx] - row_product(p, x, idx, ii, st);
                sum = sum + r * r;
                rhat[idx] = store((float)(s * r), precision);
            }
    *sumsq = sum;
}

static int32_t solve_refine(const srjo_problem *p, double *x, const srjo_opts *o,
                            srjo_result *res, int32_t *levels_out, double *norms_out)
{
    int64_t N = npoints(p);
    int32_t prec = o->precision;
    double tgt_rms = o->scale_target > 0.0 ? o->scale_target : default_target(prec);
    float *d = (float *)malloc(sizeof(float) * (size_t)N);
    float *d2 = (float *)malloc(sizeof(float) * (size_t)N);
    float *rhat = (float *)malloc(sizeof(float) * (size_t)N);
    double *w = (double *)malloc(sizeof(double) * 2362);
    op32 op;
    op32_init(p, &op);

    double r0 = srjo_residual_norm(p, x);
    res->r0 = r0;
    res->r_final = r0;
    if (norms_out) norms_out[0] = r0;
    double target = (o->tol_mode == SRJO_TOL_RELATIVE) ? o->tol * r0 : o->tol;
    int32_t status = SRJO_NOT_CONVERGED;
    int32_t level = o->start_level;
    double prev = r0;
    if (!isfinite(r0)) {
        status = SRJO_NONFINITE;
        goto done;
    }
    if (r0 == 0.0 || r0 < target) {
        res->converged = 1;
        status = SRJO_OK;
        goto done;
    }
    /* The scale applied to the residual of a pass is computed from the last
     * norm known before that pass: r0 for the first two passes, then the
     * norm of the cycle before the previous one. */
    double s = pow2_scale(r0, N, tgt_rms);
    double sumsq;
    scaled_residual(p, x, s, prec, rhat, &sumsq);
    for (int32_t cycle = 0; cycle < o->max_cycles; cycle++) {
        int32_t lv = (o->rule == SRJO_RULE_FIXED) ? o->fixed_level : level;
        int32_t M = srjo_scheme(lv, w);
        if (res->sweeps + M > o->max_sweeps) break;
        for (int64_t i = 0; i < N; i++) d[i] = 0.0f;
        for (int32_t k = 0; k < M; k++) {
            sweep32(p, &op, d, rhat, (float)w[k], prec, d2);
            float *t = d;
            d = d2;
            d2 = t;
        }
        res->sweeps += M;
        for (int64_t i = 0; i < N; i++) x[i] = x[i] + (double)d[i] / s;
        double s_next = pow2_scale(prev, N, tgt_rms);
        scaled_residual(p, x, s_next, prec, rhat, &sumsq);
        double norm = sqrt(sumsq);
        s = s_next;
        res->cycles = cycle + 1;
        res->r_final = norm;
        res->final_level = lv;
        if (levels_out) levels_out[cycle] = lv;
        if (norms_out) norms_out[cycle + 1] = norm;
        if (!isfinite(norm)) {
            status = SRJO_NONFINITE;
            break;
        }
        if (norm < target) {
            res->converged = 1;
            status = SRJO_OK;
            break;
        }
        double ratio = norm / prev;
        prev = norm;
        if (o->rule == SRJO_RULE_HEURISTIC) track_margin(res, ratio);
        level = next_level(o->rule, level, ratio, o->max_level);
    }
done:
    res->status = status;
    op32_free(&op);
    free(d);
    free(d2);
    free(rhat);
    free(w);
    return status;
}

/* ---- Section 3: data collection for the scheme selector ---------------- */

/* One SRJ cycle of the given level applied to x in place (tmp: scratch). */
static void apply_cycle(const srjo_problem *p, int32_t level, double *x, double *tmp)
{
    double w[2400];
    int32_t M = srjo_scheme(level, w);
    int64_t N = npoints(p);
    for (int32_t j = 0; j < M; j++) {
        srjo_sweep(p, x, w[j], tmp);
        memcpy(x, tmp, sizeof(double) * (size_t)N);
    }
}

void srjo_collect(const srjo_problem *p, int32_t trials, int32_t max_steps, const double *u,
                  double tol, int32_t max_level, srjo_sample *out, int32_t *steps)
{
    int64_t N = npoints(p);
#pragma omp parallel for schedule(dynamic)
    for (int32_t t = 0; t < trials; t++) {
        double *x = calloc((size_t)N, sizeof(double));
        double *z = malloc(sizeof(double) * (size_t)N);
        double *tmp = malloc(sizeof(double) * (size_t)N);
        double *next = malloc(sizeof(double) * (size_t)N);
        /* start: x = 0, one cycle of level 0; its residual ratio is the first state */
        double r_init = srjo_residual_norm(p, x);
        apply_cycle(p, 0, x, tmp);
        double rcur = srjo_residual_norm(p, x);
        double rho = rcur / r_init;
        int32_t level = 0, taken = 0;
        if (rcur >= tol && isfinite(rcur)) {
            for (int32_t s = 0; s < max_steps; s++) {
                /* the actions available from this level, in the order up, same, down */
                int32_t acts[3], k = 0;
                if (level + 1 <= max_level) acts[k++] = 1;
                acts[k++] = 0;
                if (level >= 1) acts[k++] = -1;
                int32_t idx = (int32_t)(u[(int64_t)t * max_steps + s] * (double)k);
                if (idx < 0) idx = 0;
                if (idx > k - 1) idx = k - 1;
                int32_t chosen = acts[idx];
                double r_chosen = 0.0;
                /* every available branch runs one cycle from the same iterate */
                for (int32_t j = 0; j < 3; j++) {
                    int32_t act = 1 - j;
                    int avail = act == 0 || (act == 1 && level + 1 <= max_level) ||
                                (act == -1 && level >= 1);
                    srjo_sample *o = &out[((int64_t)t * max_steps + s) * 3 + j];
                    o->trial = t;
                    o->step = s;
                    o->level = level;
                    o->action = act;
                    o->M = 0;
                    o->chosen = act == chosen;
                    o->prev_ratio = rho;
                    o->r_before = rcur;
                    o->r_after = 0.0;
                    if (!avail) continue;
                    memcpy(z, x, sizeof(double) * (size_t)N);
                    apply_cycle(p, level + act, z, tmp);
                    o->M = srjo_level_M(level + act);
                    o->r_after = srjo_residual_norm(p, z);
                    if (act == chosen) {
                        memcpy(next, z, sizeof(double) * (size_t)N);
                        r_chosen = o->r_after;
                    }
                }
                /* continue with the branch taken */
                memcpy(x, next, sizeof(double) * (size_t)N);
                rho = r_chosen / rcur;
                rcur = r_chosen;
                level += chosen;
                taken = s + 1;
                if (!(rcur >= tol) || !isfinite(rcur)) break;
            }
        }
        steps[t] = taken;
        free(x);
        free(z);
        free(tmp);
        free(next);
    }
}
