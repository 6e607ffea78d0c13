/*
 * srj_mg.c - CPU reference of SRJ cycles used as the smoother of a geometric
 * multigrid V-cycle (Islam & Wang, arXiv 2011.06636, section 5 names SRJ as a
 * multigrid smoother; the paper gives no design, so every choice below is a
 * stated reading: vertex-centred coarsening of odd grids, full-weighting
 * restriction, multilinear prolongation, coarse operators rediscretised with
 * the couplings and diagonal divided by 4, and the paper's scheme selector
 * choosing the smoothing scheme from one V-cycle to the next).
 *
 * TEST INFRASTRUCTURE ONLY, like srj_oracle.c: plain binary64 loops in a
 * fixed order, no fused multiply-add (built with -ffp-contract=off), and no
 * code shared with the GPU library.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "srj_oracle.h"

/* Grid hierarchy: level l + 1 halves every active axis of level l,
 * n' = (n - 1) / 2, while every active n is odd and at least 3 and fewer
 * than max_levels levels exist.  Returns the number of levels. */
int32_t srjo_mg_hierarchy(const srjo_problem *p, int32_t max_levels, int64_t *dims_out)
{
    int64_t n[3] = {p->n[0], p->n[1], p->n[2]};
    int32_t L = 0;
    for (;;) {
        for (int d = 0; d < 3; d++) dims_out[3 * L + d] = n[d];
        L++;
        if (L >= max_levels) break;
        int can = 1;
        for (int d = 0; d < p->ndim; d++)
            if (n[d] < 3 || n[d] % 2 == 0) can = 0;
        if (!can) break;
        for (int d = 0; d < p->ndim; d++) n[d] = (n[d] - 1) / 2;
    }
    return L;
}

/* Weight of a fine point at offset a in {-1, 0, 1} from the fine image of a
 * coarse point, per axis (full weighting: 1/4, 1/2, 1/4). */
static double fw(int a) { return a == 0 ? 0.5 : 0.25; }

/* Residual of the fine problem at point idx (same expression as a sweep). */
static double residual_at(const srjo_problem *p, const double *x, int64_t i0, int64_t i1,
                          int64_t i2)
{
    const int64_t n0 = p->n[0], n1 = p->n[1], n2 = p->n[2];
    const int64_t idx = i0 + n0 * (i1 + n1 * i2);
    double s = p->dconst * x[idx];
    const int64_t ii[3] = {i0, i1, i2};
    const int64_t st[3] = {1, n0, n0 * n1};
    const int64_t nn[3] = {n0, n1, n2};
    for (int d = 0; d < p->ndim; d++) {
        if (ii[d] > 0) s = s - p->c[d] * x[idx - st[d]];
        if (ii[d] < nn[d] - 1) s = s - p->c[d] * x[idx + st[d]];
    }
    return p->b[idx] - s;
}

/* Coarse right-hand side bc = R (b - A x): coarse point I gathers the
 * residuals of fine points 2 I + 1 + a, a in {-1, 0, 1} per active axis,
 * with weight (product of the per-axis full weights), summed with axis 2
 * outermost and axis 0 innermost, offsets in increasing order. */
void srjo_restrict_residual(const srjo_problem *p, const double *x, double *bc)
{
    const int nd = p->ndim;
    int64_t m[3] = {1, 1, 1};
    for (int d = 0; d < nd; d++) m[d] = (p->n[d] - 1) / 2;
    for (int64_t I2 = 0; I2 < m[2]; I2++)
        for (int64_t I1 = 0; I1 < m[1]; I1++)
            for (int64_t I0 = 0; I0 < m[0]; I0++) {
                double s = 0.0;
                for (int a2 = (nd > 2 ? -1 : 0); a2 <= (nd > 2 ? 1 : 0); a2++)
                    for (int a1 = (nd > 1 ? -1 : 0); a1 <= (nd > 1 ? 1 : 0); a1++)
                        for (int a0 = -1; a0 <= 1; a0++) {
                            double wt = fw(a0);
                            if (nd > 1) wt = wt * fw(a1);
                            if (nd > 2) wt = wt * fw(a2);
                            const int64_t i0 = 2 * I0 + 1 + a0;
                            const int64_t i1 = nd > 1 ? 2 * I1 + 1 + a1 : 0;
                            const int64_t i2 = nd > 2 ? 2 * I2 + 1 + a2 : 0;
                            s = s + wt * residual_at(p, x, i0, i1, i2);
                        }
                bc[I0 + m[0] * (I1 + m[1] * I2)] = s;
            }
}

/* x += P ec: per axis, a fine point 2 J + 1 takes coarse point J with
 * weight 1; a fine point 2 J takes coarse points J - 1 and J with weight 1/2
 * each (points beyond the coarse grid are the zero boundary).  The terms of a
 * fine point are summed with axis 2 outermost, axis 0 innermost, candidates
 * in increasing order, then added to x. */
void srjo_prolong_add(const srjo_problem *p, const double *ec, double *x)
{
    const int nd = p->ndim;
    const int64_t n0 = p->n[0], n1 = p->n[1], n2 = p->n[2];
    int64_t m[3] = {1, 1, 1};
    for (int d = 0; d < nd; d++) m[d] = (p->n[d] - 1) / 2;
    for (int64_t i2 = 0; i2 < n2; i2++)
        for (int64_t i1 = 0; i1 < n1; i1++)
            for (int64_t i0 = 0; i0 < n0; i0++) {
                const int64_t ii[3] = {i0, i1, i2};
                int64_t cj[3][2];
                double cw[3][2];
                int cnt[3];
                for (int d = 0; d < 3; d++) {
                    if (d >= nd) {
                        cnt[d] = 1;
                        cj[d][0] = 0;
                        cw[d][0] = 1.0;
                    } else if (ii[d] % 2 == 1) {
                        cnt[d] = 1;
                        cj[d][0] = (ii[d] - 1) / 2;
                        cw[d][0] = 1.0;
                    } else {
                        cnt[d] = 0;
                        const int64_t J = ii[d] / 2;
                        if (J - 1 >= 0) {
                            cj[d][cnt[d]] = J - 1;
                            cw[d][cnt[d]] = 0.5;
                            cnt[d]++;
                        }
                        if (J < m[d]) {
                            cj[d][cnt[d]] = J;
                            cw[d][cnt[d]] = 0.5;
                            cnt[d]++;
                        }
                    }
                }
                double v = 0.0;
                for (int k2 = 0; k2 < cnt[2]; k2++)
                    for (int k1 = 0; k1 < cnt[1]; k1++)
                        for (int k0 = 0; k0 < cnt[0]; k0++) {
                            double wt = cw[0][k0];
                            if (nd > 1) wt = wt * cw[1][k1];
                            if (nd > 2) wt = wt * cw[2][k2];
                            v = v + wt * ec[cj[0][k0] + m[0] * (cj[1][k1] + m[1] * cj[2][k2])];
                        }
                const int64_t idx = i0 + n0 * (i1 + n1 * i2);
                x[idx] = x[idx] + v;
            }
}

typedef struct {
    int32_t L;
    srjo_problem *prob;  /* per level; prob[0] is the caller's */
    double **x, **b;     /* per level >= 1 (x[0] unused) */
    double *work;        /* ping-pong buffer of the finest size */
    double *w;           /* scheme factors */
} mg_state;

/* nu SRJ cycles of `level` on level l's problem, x in place. */
static int64_t smooth(mg_state *g, int l, double *x, int32_t level, int32_t nu)
{
    const srjo_problem *p = &g->prob[l];
    const int64_t N = p->n[0] * p->n[1] * p->n[2];
    const int32_t M = srjo_scheme(level, g->w);
    double *cur = x, *nxt = g->work;
    for (int32_t c = 0; c < nu; c++)
        for (int32_t k = 0; k < M; k++) {
            srjo_sweep(p, cur, g->w[k], nxt);
            double *t = cur;
            cur = nxt;
            nxt = t;
        }
    if (cur != x) memcpy(x, cur, sizeof(double) * (size_t)N);
    return (int64_t)nu * M;
}

static void vcycle(mg_state *g, int l, double *x, const srjo_mg_opts *o, int32_t level,
                   srjo_mg_result *res)
{
    const srjo_problem *p = &g->prob[l];
    const int64_t N = p->n[0] * p->n[1] * p->n[2];
    const double frac = (double)N / (double)(g->prob[0].n[0] * g->prob[0].n[1] * g->prob[0].n[2]);
    if (l == g->L - 1) {
        /* coarsest grid: SRJ with the selector from x = 0 to a relative
         * tolerance (Algorithm 1, cycle-end test) */
        memset(x, 0, sizeof(double) * (size_t)N);
        srjo_opts so;
        memset(&so, 0, sizeof(so));
        so.rule = SRJO_RULE_HEURISTIC;
        so.tol_mode = SRJO_TOL_RELATIVE;
        so.tol = o->coarse_tol;
        so.max_cycles = o->coarse_max_cycles;
        so.max_sweeps = 50000000;
        so.precision = SRJO_PREC_F64;
        so.max_level = 24;
        srjo_result r;
        srjo_solve(p, x, &so, &r, NULL, NULL);
        res->coarse_sweeps += r.sweeps;
        res->work += (double)r.sweeps * frac;
        return;
    }
    int64_t sw = smooth(g, l, x, level, o->pre);
    srjo_restrict_residual(p, x, g->b[l + 1]);
    /* the coarse correction starts from zero */
    const srjo_problem *pc = &g->prob[l + 1];
    memset(g->x[l + 1], 0, sizeof(double) * (size_t)(pc->n[0] * pc->n[1] * pc->n[2]));
    vcycle(g, l + 1, g->x[l + 1], o, level, res);
    srjo_prolong_add(p, g->x[l + 1], x);
    sw += smooth(g, l, x, level, o->post);
    if (l == 0) res->sweeps += sw;
    res->work += (double)sw * frac;
}

int32_t srjo_mg_solve(const srjo_problem *p, double *x, const srjo_mg_opts *o,
                      srjo_mg_result *res, int32_t *levels_out, double *norms_out)
{
    memset(res, 0, sizeof(*res));
    if (!p || !o || !p->b || p->rowptr || p->diag || p->ndim < 1 || p->ndim > 3)
        return res->status = SRJO_INVALID;
    for (int d = 0; d < 3; d++)
        if (p->face[d] || p->n[d] < 1 || (d >= p->ndim && p->n[d] != 1))
            return res->status = SRJO_INVALID;
    if (!(p->dconst > 0.0) || !(o->tol > 0.0) || o->pre < 0 || o->post < 0 ||
        o->max_levels < 1 || o->max_vcycles < 1 || o->start_level < 0 ||
        o->start_level > o->max_level || o->max_level > 24 ||
        (o->rule != SRJO_RULE_HEURISTIC && o->rule != SRJO_RULE_FIXED) ||
        !(o->coarse_tol > 0.0) || o->coarse_max_cycles < 1 ||
        (o->tol_mode != SRJO_TOL_RELATIVE && o->tol_mode != SRJO_TOL_ABSOLUTE))
        return res->status = SRJO_INVALID;

    int64_t dims[3 * 32];
    mg_state g;
    memset(&g, 0, sizeof(g));
    g.L = srjo_mg_hierarchy(p, o->max_levels < 32 ? o->max_levels : 32, dims);
    if (g.L < 2) return res->status = SRJO_INVALID;
    g.prob = (srjo_problem *)calloc((size_t)g.L, sizeof(srjo_problem));
    g.x = (double **)calloc((size_t)g.L, sizeof(double *));
    g.b = (double **)calloc((size_t)g.L, sizeof(double *));
    g.prob[0] = *p;
    for (int l = 1; l < g.L; l++) {
        srjo_problem q = g.prob[l - 1];
        for (int d = 0; d < 3; d++) q.n[d] = dims[3 * l + d];
        /* rediscretisation on the doubled spacing: couplings and diagonal / 4 */
        for (int d = 0; d < 3; d++) q.c[d] = q.c[d] / 4.0;
        q.dconst = q.dconst / 4.0;
        const int64_t N = q.n[0] * q.n[1] * q.n[2];
        g.x[l] = (double *)calloc((size_t)N, sizeof(double));
        g.b[l] = (double *)calloc((size_t)N, sizeof(double));
        q.b = g.b[l];
        g.prob[l] = q;
    }
    g.work = (double *)malloc(sizeof(double) * (size_t)(p->n[0] * p->n[1] * p->n[2]));
    g.w = (double *)malloc(sizeof(double) * 2362);
    res->levels = g.L;

    const double r0 = srjo_residual_norm(p, x);
    res->r0 = r0;
    res->r_final = r0;
    if (norms_out) norms_out[0] = r0;
    const double target = o->tol_mode == SRJO_TOL_RELATIVE ? o->tol * r0 : o->tol;
    int32_t status = SRJO_NOT_CONVERGED;
    int32_t level = o->start_level;
    double prev = r0;
    if (!isfinite(r0)) {
        status = SRJO_NONFINITE;
    } else if (r0 == 0.0 || r0 < target) {
        res->converged = 1;
        status = SRJO_OK;
    } else {
        for (int32_t v = 0; v < o->max_vcycles; v++) {
            const int32_t lv = o->rule == SRJO_RULE_FIXED ? o->start_level : level;
            vcycle(&g, 0, x, o, lv, res);
            const double norm = srjo_residual_norm(p, x);
            if (levels_out) levels_out[v] = lv;
            if (norms_out) norms_out[v + 1] = norm;
            res->vcycles = v + 1;
            res->final_level = lv;
            res->r_final = norm;
            if (!isfinite(norm)) {
                status = SRJO_NONFINITE;
                break;
            }
            if (norm < target) {
                res->converged = 1;
                status = SRJO_OK;
                break;
            }
            /* the selector of section 3 (Algorithm 1) on V-cycle ratios */
            const double ratio = norm / prev;
            prev = norm;
            if (o->rule == SRJO_RULE_HEURISTIC) {
                if (ratio > 0.4)
                    level = level + 1;
                else if (ratio < 0.4 && ratio > 0.2)
                    level = level - 1;
                if (level < 0) level = 0;
                if (level > o->max_level) level = o->max_level;
            }
        }
    }
    for (int l = 1; l < g.L; l++) {
        free(g.x[l]);
        free(g.b[l]);
    }
    free(g.prob);
    free(g.x);
    free(g.b);
    free(g.work);
    free(g.w);
    res->status = status;
    return status;
}
