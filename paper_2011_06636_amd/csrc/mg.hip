// SRJ cycles as the smoother of a geometric multigrid V-cycle.
//
// Islam & Wang (arXiv 2011.06636) name SRJ as a candidate multigrid smoother
// in section 5 without a design; this file's design is the library's reading:
//   * vertex-centred coarsening of odd grids: every active axis halves,
//     n' = (n - 1) / 2, while all active sizes are odd and >= 3;
//   * coarse operators rediscretised on the doubled spacing: couplings and
//     diagonal divided by 4 (constant-coefficient stencils only);
//   * full-weighting restriction of the residual and multilinear
//     interpolation of the correction, each a fixed-order sum;
//   * pre- and post-smoothing by whole SRJ cycles of one scheme (section 2,
//     Eqs. 3 and 7), the scheme chosen from one V-cycle to the next by
//     Algorithm 1 of section 3 on the V-cycle residual ratios (or fixed);
//   * the coarsest grid solved by SRJ with Algorithm 1 from zero to a
//     relative tolerance (srj_solve on that level's context).
// Every level is an ordinary context, so smoothing and the coarsest solve use
// the library's sweep, residual and resident kernels; the transfers are the
// two kernels below.  Each value is formed by the same operations in the same
// order as the CPU reference, so iterates are bit-identical to it.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <vector>

#include "internal.h"

#pragma clang fp contract(off)

namespace srj {

namespace {

constexpr int kMgBlock = 256;
constexpr int kMgMaxLevels = 32;

__device__ __forceinline__ double full_weight(int a) { return a == 0 ? 0.5 : 0.25; }

// Coarse right-hand side bc = R (b - A x): one thread per coarse point; the
// fine residuals of points 2 I + 1 + a (a in {-1, 0, 1} per active axis) are
// weighted by the product of the per-axis full weights and summed with axis 2
// outermost and axis 0 innermost.  Each residual is the sweep's expression.
template <int ND>
__global__ __launch_bounds__(kMgBlock) void k_restrict_residual(DevProblem P,
                                                                const double *__restrict__ x,
                                                                double *__restrict__ bc,
                                                                int64_t m0, int64_t m1,
                                                                int64_t m2)
{
    const int64_t t = (int64_t)blockIdx.x * kMgBlock + threadIdx.x;
    if (t >= m0 * m1 * m2) return;
    const int64_t I0 = t % m0, I1 = (t / m0) % m1, I2 = t / (m0 * m1);
    const int64_t n0 = P.n0, n1 = P.n1, n2 = P.n2;
    const int64_t s1 = n0, s2 = n0 * n1;
    double s = 0.0;
#pragma unroll
    for (int a2 = (ND > 2 ? -1 : 0); a2 <= (ND > 2 ? 1 : 0); ++a2)
#pragma unroll
        for (int a1 = (ND > 1 ? -1 : 0); a1 <= (ND > 1 ? 1 : 0); ++a1)
#pragma unroll
            for (int a0 = -1; a0 <= 1; ++a0) {
                double wt = full_weight(a0);
                if (ND > 1) wt = wt * full_weight(a1);
                if (ND > 2) wt = wt * full_weight(a2);
                const int64_t i0 = 2 * I0 + 1 + a0;
                const int64_t i1 = ND > 1 ? 2 * I1 + 1 + a1 : 0;
                const int64_t i2 = ND > 2 ? 2 * I2 + 1 + a2 : 0;
                const int64_t p = i0 + s1 * i1 + s2 * i2;
                double r = P.dconst * x[p];
                if (i0 > 0) r = r - P.c[0] * x[p - 1];
                if (i0 < n0 - 1) r = r - P.c[0] * x[p + 1];
                if (ND > 1) {
                    if (i1 > 0) r = r - P.c[1] * x[p - s1];
                    if (i1 < n1 - 1) r = r - P.c[1] * x[p + s1];
                }
                if (ND > 2) {
                    if (i2 > 0) r = r - P.c[2] * x[p - s2];
                    if (i2 < n2 - 1) r = r - P.c[2] * x[p + s2];
                }
                s = s + wt * (P.b[p] - r);
            }
    bc[t] = s;
}

// x += P ec: one thread per fine point.  Per axis a fine index 2 J + 1 takes
// coarse J with weight 1, a fine index 2 J takes coarse J - 1 and J with
// weight 1/2 (indices outside the coarse grid are the zero boundary); terms
// summed with axis 2 outermost, axis 0 innermost, candidates in increasing
// order.
template <int ND>
__global__ __launch_bounds__(kMgBlock) void k_prolong_add(const double *__restrict__ ec,
                                                          double *__restrict__ x, int64_t n0,
                                                          int64_t n1, int64_t n2, int64_t m0,
                                                          int64_t m1, int64_t m2)
{
    const int64_t t = (int64_t)blockIdx.x * kMgBlock + threadIdx.x;
    if (t >= n0 * n1 * n2) return;
    const int64_t ii[3] = {t % n0, (t / n0) % n1, t / (n0 * n1)};
    const int64_t mm[3] = {m0, m1, m2};
    int64_t cj[3][2];
    double cw[3][2];
    int cnt[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        if (d >= ND) {
            cnt[d] = 1;
            cj[d][0] = 0;
            cw[d][0] = 1.0;
            cj[d][1] = 0;
            cw[d][1] = 0.0;
        } else if (ii[d] & 1) {
            cnt[d] = 1;
            cj[d][0] = (ii[d] - 1) / 2;
            cw[d][0] = 1.0;
            cj[d][1] = 0;
            cw[d][1] = 0.0;
        } else {
            const int64_t J = ii[d] / 2;
            int c = 0;
            cj[d][0] = cj[d][1] = 0;
            cw[d][0] = cw[d][1] = 0.0;
            if (J - 1 >= 0) {
                cj[d][c] = J - 1;
                cw[d][c] = 0.5;
                ++c;
            }
            if (J < mm[d]) {
                cj[d][c] = J;
                cw[d][c] = 0.5;
                ++c;
            }
            cnt[d] = c;
        }
    }
    double v = 0.0;
    for (int k2 = 0; k2 < cnt[2]; ++k2)
        for (int k1 = 0; k1 < cnt[1]; ++k1)
            for (int k0 = 0; k0 < cnt[0]; ++k0) {
                double wt = cw[0][k0];
                if (ND > 1) wt = wt * cw[1][k1];
                if (ND > 2) wt = wt * cw[2][k2];
                v = v + wt * ec[cj[0][k0] + m0 * (cj[1][k1] + m1 * cj[2][k2])];
            }
    x[t] = x[t] + v;
}

__global__ void k_mg_zero(double *__restrict__ x, int64_t n)
{
    const int64_t t = (int64_t)blockIdx.x * kMgBlock + threadIdx.x;
    if (t < n) x[t] = 0.0;
}

unsigned blocks_for(int64_t n) { return (unsigned)((n + kMgBlock - 1) / kMgBlock); }

}  // namespace

}  // namespace srj

using namespace srj;

// Levels: contexts (level 0 borrows the caller's b), per-level correction
// and right-hand-side buffers for levels >= 1.
struct srj_mg {
    int L = 0;
    int ndim = 1;
    hipStream_t stream = nullptr;
    std::vector<srj_ctx *> ctx;
    std::vector<double *> xb, bb;   // index 0 unused
    std::vector<int64_t> npts;
};

namespace {

srj_status mg_free(srj_mg *g)
{
    if (!g) return SRJ_OK;
    if (g->stream) (void)hipStreamSynchronize(g->stream);
    else (void)hipDeviceSynchronize();
    for (srj_ctx *c : g->ctx) srj_destroy(c);
    for (double *p : g->xb) (void)hipFree(p);
    for (double *p : g->bb) (void)hipFree(p);
    delete g;
    return SRJ_OK;
}

struct MgRun {
    srj_mg *g;
    const srj_mg_opts *o;
    int Lc;                 // coarsest level used
    std::vector<double *> cur;
    srj_mg_result *res;
};

srj_status launch_restrict(const srj_ctx *c, const double *x, double *bc, hipStream_t s)
{
    const DevProblem &P = c->P;
    const int64_t m0 = P.ndim > 0 ? (P.n0 - 1) / 2 : 1, m1 = P.ndim > 1 ? (P.n1 - 1) / 2 : 1,
                  m2 = P.ndim > 2 ? (P.n2 - 1) / 2 : 1;
    const unsigned nb = blocks_for(m0 * m1 * m2);
    switch (P.ndim) {
    case 1: hipLaunchKernelGGL(k_restrict_residual<1>, dim3(nb), dim3(kMgBlock), 0, s, P, x, bc, m0, m1, m2); break;
    case 2: hipLaunchKernelGGL(k_restrict_residual<2>, dim3(nb), dim3(kMgBlock), 0, s, P, x, bc, m0, m1, m2); break;
    default: hipLaunchKernelGGL(k_restrict_residual<3>, dim3(nb), dim3(kMgBlock), 0, s, P, x, bc, m0, m1, m2); break;
    }
    SRJ_HIP_CHECK(hipGetLastError());
    return SRJ_OK;
}

srj_status launch_prolong(const srj_ctx *c, const double *ec, double *x, hipStream_t s)
{
    const DevProblem &P = c->P;
    const int64_t m0 = (P.n0 - 1) / 2, m1 = P.ndim > 1 ? (P.n1 - 1) / 2 : 1,
                  m2 = P.ndim > 2 ? (P.n2 - 1) / 2 : 1;
    const unsigned nb = blocks_for(P.n0 * P.n1 * P.n2);
    switch (P.ndim) {
    case 1: hipLaunchKernelGGL(k_prolong_add<1>, dim3(nb), dim3(kMgBlock), 0, s, ec, x, P.n0, P.n1, P.n2, m0, m1, m2); break;
    case 2: hipLaunchKernelGGL(k_prolong_add<2>, dim3(nb), dim3(kMgBlock), 0, s, ec, x, P.n0, P.n1, P.n2, m0, m1, m2); break;
    default: hipLaunchKernelGGL(k_prolong_add<3>, dim3(nb), dim3(kMgBlock), 0, s, ec, x, P.n0, P.n1, P.n2, m0, m1, m2); break;
    }
    SRJ_HIP_CHECK(hipGetLastError());
    return SRJ_OK;
}

srj_status vcycle(MgRun &run, int l, int level, double *x0)
{
    srj_mg *g = run.g;
    srj_ctx *c = g->ctx[l];
    const double frac = (double)g->npts[l] / (double)g->npts[0];
    if (l == run.Lc) {
        // coarsest grid: SRJ with Algorithm 1 from zero to coarse_tol
        double *x = g->xb[l];
        hipLaunchKernelGGL(k_mg_zero, dim3(blocks_for(g->npts[l])), dim3(kMgBlock), 0, g->stream, x,
                           g->npts[l]);
        SRJ_HIP_CHECK(hipGetLastError());
        srj_solve_opts so;
        srj_default_opts(&so);
        so.rule = SRJ_RULE_HEURISTIC;
        so.tol_mode = SRJ_TOL_RELATIVE;
        so.tol = run.o->coarse_tol;
        so.max_cycles = run.o->coarse_max_cycles;
        so.max_sweeps = 50000000;
        so.max_level = SRJ_NUM_LEVELS - 1;
        srj_solve_result r;
        srj_status st = srj_solve(c, x, &so, &r, nullptr, nullptr);
        if (st != SRJ_OK && st != SRJ_ERR_NOT_CONVERGED) return st;
        run.cur[l] = x;
        run.res->coarse_sweeps += r.sweeps;
        run.res->work += (double)r.sweeps * frac;
        return SRJ_OK;
    }
    // the level's two buffers: level 0 the caller's x and the context's
    // ping-pong buffer, other levels their correction buffer and theirs
    int64_t sw = 0;
    auto pair_smooth = [&](int nu) -> srj_status {
        double *a = l == 0 ? x0 : g->xb[l];
        double *cur = run.cur[l];
        double *nxt = cur == a ? c->ws : a;
        for (int k = 0; k < nu; ++k) {
            srj_status st = run_sweeps(c, &cur, &nxt, level);
            if (st != SRJ_OK) return st;
            sw += (int64_t)c->factors[level].size();
        }
        run.cur[l] = cur;
        return SRJ_OK;
    };
    srj_status st = pair_smooth(run.o->pre);
    if (st != SRJ_OK) return st;
    if ((st = launch_restrict(c, run.cur[l], g->bb[l + 1], g->stream)) != SRJ_OK) return st;
    // the coarse correction starts from zero
    double *xc = g->xb[l + 1];
    hipLaunchKernelGGL(k_mg_zero, dim3(blocks_for(g->npts[l + 1])), dim3(kMgBlock), 0, g->stream, xc,
                       g->npts[l + 1]);
    SRJ_HIP_CHECK(hipGetLastError());
    run.cur[l + 1] = xc;
    if ((st = vcycle(run, l + 1, level, x0)) != SRJ_OK) return st;
    if ((st = launch_prolong(c, run.cur[l + 1], run.cur[l], g->stream)) != SRJ_OK) return st;
    if ((st = pair_smooth(run.o->post)) != SRJ_OK) return st;
    if (l == 0) run.res->sweeps += sw;
    run.res->work += (double)sw * frac;
    return SRJ_OK;
}

srj_status validate_mg_opts(const srj_mg_opts *o)
{
    if (!o) return fail(SRJ_ERR_INVALID, "opts is NULL");
    if (o->rule != SRJ_RULE_HEURISTIC && o->rule != SRJ_RULE_FIXED)
        return fail(SRJ_ERR_INVALID, "rule must be SRJ_RULE_HEURISTIC or SRJ_RULE_FIXED");
    if (o->max_level < 0 || o->max_level >= SRJ_NUM_LEVELS)
        return fail(SRJ_ERR_INVALID, "max_level outside 0..24");
    if (o->start_level < 0 || o->start_level > o->max_level)
        return fail(SRJ_ERR_INVALID, "start_level outside 0..max_level");
    if (o->pre < 0 || o->post < 0 || o->pre > 1000 || o->post > 1000)
        return fail(SRJ_ERR_INVALID, "pre and post must be 0..1000");
    if (o->max_levels < 2) return fail(SRJ_ERR_INVALID, "max_levels must be >= 2");
    if (!(o->coarse_tol > 0.0)) return fail(SRJ_ERR_INVALID, "coarse_tol must be > 0");
    if (o->coarse_max_cycles < 1) return fail(SRJ_ERR_INVALID, "coarse_max_cycles must be >= 1");
    if (o->tol_mode != SRJ_TOL_RELATIVE && o->tol_mode != SRJ_TOL_ABSOLUTE)
        return fail(SRJ_ERR_INVALID, "tol_mode must be relative or absolute");
    if (!(o->tol > 0.0)) return fail(SRJ_ERR_INVALID, "tol must be > 0");
    if (o->max_vcycles < 1) return fail(SRJ_ERR_INVALID, "max_vcycles must be >= 1");
    return SRJ_OK;
}

}  // namespace

extern "C" {

void srj_mg_default_opts(srj_mg_opts *o)
{
    if (!o) return;
    memset(o, 0, sizeof(*o));
    o->rule = SRJ_RULE_HEURISTIC;
    o->start_level = 0;
    o->max_level = SRJ_NUM_LEVELS - 1;
    o->pre = 1;
    o->post = 1;
    o->max_levels = kMgMaxLevels;
    o->coarse_tol = 1e-8;
    o->coarse_max_cycles = 1000;
    o->tol_mode = SRJ_TOL_RELATIVE;
    o->tol = 1e-10;
    o->max_vcycles = 200;
}

srj_status srj_mg_setup(const srj_problem *p, void *hip_stream, srj_mg **out)
{
    if (!out) return fail(SRJ_ERR_INVALID, "out is NULL");
    *out = nullptr;
    srj_status st = validate_problem(p);
    if (st != SRJ_OK) return st;
    if (p->diag || p->face[0] || p->face[1] || p->face[2])
        return fail(SRJ_ERR_UNSUPPORTED, "multigrid takes constant-coefficient stencils");
    int64_t n[3] = {p->n[0], p->n[1], p->n[2]};
    std::vector<std::array<int64_t, 3>> dims;
    for (;;) {
        dims.push_back({n[0], n[1], n[2]});
        if ((int)dims.size() >= kMgMaxLevels) break;
        bool can = true;
        for (int d = 0; d < p->ndim; ++d)
            if (n[d] < 3 || n[d] % 2 == 0) can = false;
        if (!can) break;
        for (int d = 0; d < p->ndim; ++d) n[d] = (n[d] - 1) / 2;
    }
    if (dims.size() < 2)
        return fail(SRJ_ERR_UNSUPPORTED, "grid cannot be coarsened (every active size must be odd and >= 3)");
    srj_mg *g = new srj_mg();
    g->L = (int)dims.size();
    g->ndim = p->ndim;
    g->stream = static_cast<hipStream_t>(hip_stream);
    g->ctx.assign(g->L, nullptr);
    g->xb.assign(g->L, nullptr);
    g->bb.assign(g->L, nullptr);
    g->npts.assign(g->L, 0);
    srj_problem q = *p;
    for (int l = 0; l < g->L; ++l) {
        for (int d = 0; d < 3; ++d) q.n[d] = dims[l][d];
        g->npts[l] = q.n[0] * q.n[1] * q.n[2];
        if (l > 0) {
            // rediscretisation on the doubled spacing: couplings and diagonal / 4
            for (int d = 0; d < 3; ++d) q.cconst[d] = q.cconst[d] / 4.0;
            q.dconst = q.dconst / 4.0;
            const size_t bytes = sizeof(double) * (size_t)g->npts[l];
            if (hipMalloc(&g->xb[l], bytes) != hipSuccess || hipMalloc(&g->bb[l], bytes) != hipSuccess) {
                mg_free(g);
                return fail(SRJ_ERR_NOMEM, "hipMalloc failed for a multigrid level");
            }
            q.b = g->bb[l];
        }
        srj_ctx *c = nullptr;
        st = srj_setup(&q, hip_stream, &c);
        if (st != SRJ_OK) {
            const std::string msg = srj_last_error();
            mg_free(g);
            return fail(st, "multigrid level " + std::to_string(l) + ": " + msg);
        }
        g->ctx[l] = c;
    }
    *out = g;
    return SRJ_OK;
}

srj_status srj_mg_solve(srj_mg *g, double *x, const srj_mg_opts *o, srj_mg_result *res,
                        int32_t *levels_out, double *norms_out)
{
    if (!g || !x || !res) return fail(SRJ_ERR_INVALID, "NULL argument");
    srj_status st = validate_mg_opts(o);
    if (st != SRJ_OK) return st;
    srj_ctx *c0 = g->ctx[0];
    st = check_device_array(x, sizeof(double) * (size_t)g->npts[0], c0->device, "x");
    if (st != SRJ_OK) return st;
    memset(res, 0, sizeof(*res));
    MgRun run{g, o, std::min(g->L, o->max_levels) - 1, std::vector<double *>(g->L, nullptr), res};
    res->levels = run.Lc + 1;
    run.cur[0] = x;

    double norm0 = 0.0;
    if ((st = residual_norm(c0, x, &norm0)) != SRJ_OK) return st;
    res->r0 = norm0;
    res->r_final = norm0;
    if (norms_out) norms_out[0] = norm0;
    const double target = o->tol_mode == SRJ_TOL_RELATIVE ? o->tol * norm0 : o->tol;
    srj_status status = SRJ_ERR_NOT_CONVERGED;
    int level = o->start_level;
    double prev = norm0;
    if (!std::isfinite(norm0)) {
        status = SRJ_ERR_NONFINITE;
    } else if (norm0 == 0.0 || norm0 < target) {
        res->converged = 1;
        status = SRJ_OK;
    } else {
        for (int v = 0; v < o->max_vcycles; ++v) {
            const int lv = o->rule == SRJ_RULE_FIXED ? o->start_level : level;
            if ((st = vcycle(run, 0, lv, x)) != SRJ_OK) return st;
            double norm = 0.0;
            if ((st = residual_norm(c0, run.cur[0], &norm)) != SRJ_OK) return st;
            if (levels_out) levels_out[v] = lv;
            if (norms_out) norms_out[v + 1] = norm;
            res->vcycles = v + 1;
            res->final_level = lv;
            res->r_final = norm;
            if (!std::isfinite(norm)) {
                status = SRJ_ERR_NONFINITE;
                break;
            }
            if (norm < target) {
                res->converged = 1;
                status = SRJ_OK;
                break;
            }
            // Algorithm 1 on the V-cycle ratios picks the next smoothing scheme
            const double ratio = norm / prev;
            prev = norm;
            if (o->rule == SRJ_RULE_HEURISTIC) level = next_level(o->rule, level, ratio, o->max_level);
        }
    }
    if (run.cur[0] != x)
        SRJ_HIP_CHECK(hipMemcpyAsync(x, run.cur[0], sizeof(double) * (size_t)g->npts[0],
                                     hipMemcpyDeviceToDevice, g->stream));
    SRJ_HIP_CHECK(hipStreamSynchronize(g->stream));
    if (status == SRJ_ERR_NONFINITE) return fail(status, "non-finite residual norm");
    if (status == SRJ_ERR_NOT_CONVERGED) return fail(status, "V-cycle cap reached");
    return SRJ_OK;
}

srj_status srj_mg_destroy(srj_mg *g) { return mg_free(g); }

}  // extern "C"
