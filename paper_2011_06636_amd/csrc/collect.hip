// Training data for the scheme selector, and the rule derived from it
// (Islam & Wang, arXiv 2011.06636, section 3).
//
// Data collection: a trial starts from x = 0, applies one level-0 cycle, and
// then repeats one step: from the current iterate, the cycles of the three
// neighbouring levels (one up, the same, one down; only those inside
// 0..max_level) are each applied to a copy, the L2 residual norm before and
// after each is recorded with the state (current level and the residual
// ratio of the previous cycle), and one of the branches is taken at random.
// A trial ends when the residual norm of the iterate falls below tol (or
// after max_steps steps).  The random draws are an input, so a run is
// reproducible and can be replayed on the CPU.
//
// One workgroup runs one trial with the whole grid (at most kCollectMax
// points, one per thread) in LDS; the per-point arithmetic is the library's
// fixed binary64 expression, and every residual norm sums its squares in
// index order, so samples are bit-identical to a sequential CPU reference.
//
// Post-processing (host): samples are grouped by level, sorted by the
// previous residual ratio and cut into clusters of n_set samples; per
// cluster and action the mean average convergence rate, -log(r_after /
// r_before) / M, gets a confidence interval, and the best action counts only
// if its interval overlaps no other action's.  The rule "ratio > t_high: up;
// t_low < ratio < t_high: down; otherwise keep" is then fitted to the decided
// clusters.
#include <math.h>

#include <algorithm>
#include <numeric>
#include <string>
#include <vector>

#include "internal.h"
#include "rowsum.h"

#pragma clang fp contract(off)

namespace srj {

namespace {

constexpr int kCollectMax = 1024;  // grid points of a collection problem

struct CollectArgs {
    int32_t max_steps, max_level;
    double tol;
};

// L2 norm of b - A u: the squares are formed in parallel and summed by one
// thread in index order; every thread gets the result.
__device__ double norm_seq(const DevProblem &P, const double *u, double *sq, double *slot,
                           int64_t N, int64_t p, int64_t i0, int64_t i1, int64_t i2, double bv)
{
    if (p < N) {
        const double r = bv - row_s(P, u, p, i0, i1, i2);
        sq[p] = r * r;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int64_t q = 0; q < N; ++q) s = s + sq[q];
        *slot = sqrt(s);
    }
    __syncthreads();
    return *slot;
}

__global__ __launch_bounds__(kCollectMax) void k_collect(DevProblem P, const double *__restrict__ omega,
                                                         const int32_t *__restrict__ offsets,
                                                         const int32_t *__restrict__ levelM,
                                                         const double *__restrict__ u, CollectArgs a,
                                                         srj_sample *__restrict__ out,
                                                         int32_t *__restrict__ steps_out)
{
    extern __shared__ double lds[];
    const int64_t N = P.n0 * P.n1 * P.n2;
    double *xs = lds, *keep = lds + N, *wa = lds + 2 * N, *wb = lds + 3 * N, *sq = lds + 4 * N,
           *slot = lds + 5 * N;
    const int trial = blockIdx.x;
    const int64_t p = threadIdx.x;
    const int64_t i0 = p % P.n0, i1 = (p / P.n0) % P.n1, i2 = p / (P.n0 * P.n1);
    const double bv = p < N ? P.b[p] : 0.0;
    const double dinv = p < N ? (P.diag ? P.dinv[p] : P.dinvconst) : 0.0;
    if (p < N) xs[p] = 0.0;
    __syncthreads();
    // one cycle of level lvl applied to xs; returns the buffer holding the result
    auto cycle = [&](int lvl) -> const double * {
        const int M = levelM[lvl];
        const double *w = omega + offsets[lvl];
        const double *src = xs;
        double *dst = wa;
        for (int j = 0; j < M; ++j) {
            if (p < N) {
                const double s = row_s(P, src, p, i0, i1, i2);
                const double r = bv - s;
                const double t = dinv * r;
                dst[p] = src[p] + w[j] * t;
            }
            __syncthreads();
            src = dst;
            dst = dst == wa ? wb : wa;
        }
        return src;
    };
    auto norm = [&](const double *v) { return norm_seq(P, v, sq, slot, N, p, i0, i1, i2, bv); };

    const double r_init = norm(xs);
    {
        const double *R = cycle(0);  // the start: one cycle of level 0
        if (p < N) xs[p] = R[p];
        __syncthreads();
    }
    double rcur = norm(xs);
    double rho = rcur / r_init;
    int level = 0, steps = 0;
    if (rcur >= a.tol && isfinite(rcur)) {
        for (int step = 0; step < a.max_steps; ++step) {
            // available actions in slot order: up, keep, down
            int acts[3], k = 0;
            if (level + 1 <= a.max_level) acts[k++] = 1;
            acts[k++] = 0;
            if (level >= 1) acts[k++] = -1;
            int idx = (int)(u[(int64_t)trial * a.max_steps + step] * (double)k);
            idx = idx < 0 ? 0 : (idx >= k ? k - 1 : idx);
            const int chosen = acts[idx];
            double rchosen = 0.0;
            for (int j = 0; j < 3; ++j) {
                const int act = 1 - j;
                srj_sample *o = out + ((int64_t)trial * a.max_steps + step) * 3 + j;
                const bool avail = act == 0 || (act == 1 && level + 1 <= a.max_level) ||
                                   (act == -1 && level >= 1);
                double ra = 0.0;
                if (avail) {
                    const double *R = cycle(level + act);
                    ra = norm(R);
                    if (act == chosen && p < N) keep[p] = R[p];
                    if (act == chosen) rchosen = ra;
                    __syncthreads();  // keep is written before the next branch reuses wa / wb
                }
                if (threadIdx.x == 0) {
                    o->trial = trial;
                    o->step = step;
                    o->level = level;
                    o->action = act;
                    o->M = avail ? levelM[level + act] : 0;
                    o->chosen = act == chosen;
                    o->prev_ratio = rho;
                    o->r_before = rcur;
                    o->r_after = ra;
                }
            }
            if (p < N) xs[p] = keep[p];
            __syncthreads();
            rho = rchosen / rcur;
            rcur = rchosen;
            level += chosen;
            steps = step + 1;
            if (!(rcur >= a.tol) || !isfinite(rcur)) break;
        }
    }
    if (threadIdx.x == 0) steps_out[trial] = steps;
}

}  // namespace

}  // namespace srj

using namespace srj;

extern "C" {

srj_status srj_collect(srj_ctx *c, int32_t trials, int32_t max_steps, const double *u, double tol,
                       int32_t max_level, srj_sample *samples, int32_t *steps)
{
    if (!c || !u || !samples || !steps) return fail(SRJ_ERR_INVALID, "NULL argument");
    if (trials < 1) return fail(SRJ_ERR_INVALID, "trials must be >= 1");
    if (max_steps < 1) return fail(SRJ_ERR_INVALID, "max_steps must be >= 1");
    if ((int64_t)trials * max_steps > ((int64_t)1 << 40))
        return fail(SRJ_ERR_INVALID, "trials x max_steps too large");
    if (!(tol > 0.0)) return fail(SRJ_ERR_INVALID, "tol must be > 0");
    if (max_level < 0 || max_level >= SRJ_NUM_LEVELS)
        return fail(SRJ_ERR_INVALID, "max_level outside 0..24");
    max_level = std::min(max_level, c->nlevels - 1);  // the context's scheme family
    if (c->npoints > kCollectMax)
        return fail(SRJ_ERR_UNSUPPORTED, "collection problems hold at most 1024 points");
    srj_status chk = check_device_array(u, sizeof(double) * (size_t)trials * (size_t)max_steps,
                                        c->device, "u");
    if (chk != SRJ_OK) return chk;
    const int64_t N = c->npoints;
    std::vector<int32_t> lmh(SRJ_NUM_LEVELS);
    for (int l = 0; l < SRJ_NUM_LEVELS; ++l) lmh[l] = l < c->nlevels ? c->levelM[l] : 0;
    int32_t *lm = nullptr, *offs = nullptr;
    srj_status st = SRJ_OK;
    if (hipMalloc(&lm, sizeof(int32_t) * SRJ_NUM_LEVELS) != hipSuccess ||
        hipMalloc(&offs, sizeof(int32_t) * c->offsets.size()) != hipSuccess)
        st = fail(SRJ_ERR_NOMEM, "hipMalloc failed for the collection tables");
    if (st == SRJ_OK) {
        hipError_t e = hipMemcpyAsync(lm, lmh.data(), sizeof(int32_t) * SRJ_NUM_LEVELS,
                                      hipMemcpyHostToDevice, c->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(offs, c->offsets.data(), sizeof(int32_t) * c->offsets.size(),
                               hipMemcpyHostToDevice, c->stream);
        if (e == hipSuccess) {
            CollectArgs a{max_steps, max_level, tol};
            const int threads = (int)std::max<int64_t>(64, (N + 63) / 64 * 64);
            const size_t shmem = sizeof(double) * (size_t)(5 * N + 1);
            hipLaunchKernelGGL(k_collect, dim3((unsigned)trials), dim3(threads), shmem, c->stream,
                               c->P, c->omega_dev, offs, lm, u, a, samples, steps);
            e = hipGetLastError();
        }
        // the tables are freed below: wait for the kernel that reads them
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) st = fail(SRJ_ERR_HIP, std::string("collect: ") + hipGetErrorString(e));
    }
    (void)hipFree(lm);
    (void)hipFree(offs);
    return st;
}

srj_status srj_cluster_samples(const srj_sample *samples, int64_t count, int32_t n_set, double z,
                               srj_cluster *out, int32_t cap, int32_t *n_out)
{
    if ((!samples && count > 0) || !n_out || (!out && cap > 0))
        return fail(SRJ_ERR_INVALID, "NULL argument");
    if (count < 0 || n_set < 2 || cap < 0) return fail(SRJ_ERR_INVALID, "count, n_set or cap out of range");
    if (!(z > 0.0)) return fail(SRJ_ERR_INVALID, "z must be > 0");
    // usable samples, grouped by level in input order, as compact records
    struct Rec {
        double ratio, rate;
        int32_t slot;  // 0 up, 1 keep, 2 down
    };
    std::vector<std::vector<Rec>> by_level(SRJ_NUM_LEVELS);
    for (int64_t i = 0; i < count; ++i) {
        const srj_sample &s = samples[i];
        if (s.M <= 0 || s.level < 0 || s.level >= SRJ_NUM_LEVELS || s.action < -1 || s.action > 1)
            continue;
        if (!(s.r_before > 0.0) || !(s.r_after > 0.0) || !isfinite(s.prev_ratio)) continue;
        const double rate = -log(s.r_after / s.r_before) / (double)s.M;
        if (!isfinite(rate)) continue;
        by_level[s.level].push_back({s.prev_ratio, rate, 1 - s.action});
    }
    int32_t n = 0;
    for (int lv = 0; lv < SRJ_NUM_LEVELS; ++lv) {
        std::vector<Rec> &ix = by_level[lv];
        std::stable_sort(ix.begin(), ix.end(),
                         [](const Rec &a, const Rec &b) { return a.ratio < b.ratio; });
        // whole clusters only: a trailing partial cluster is dropped
        for (size_t c0 = 0; c0 + (size_t)n_set <= ix.size(); c0 += (size_t)n_set) {
            srj_cluster cl{};
            cl.level = lv;
            cl.count = n_set;
            double sr = 0.0;
            double sum[3] = {0.0, 0.0, 0.0};
            for (size_t k = c0; k < c0 + (size_t)n_set; ++k) {
                sr = sr + ix[k].ratio;
                cl.n[ix[k].slot] += 1;
                sum[ix[k].slot] = sum[ix[k].slot] + ix[k].rate;
            }
            cl.mean_ratio = sr / (double)n_set;
            double ss[3] = {0.0, 0.0, 0.0};
            for (int j = 0; j < 3; ++j) cl.mean_rate[j] = cl.n[j] > 0 ? sum[j] / (double)cl.n[j] : 0.0;
            for (size_t k = c0; k < c0 + (size_t)n_set; ++k) {
                const int j = ix[k].slot;
                const double d = ix[k].rate - cl.mean_rate[j];
                ss[j] = ss[j] + d * d;
            }
            for (int j = 0; j < 3; ++j)
                cl.half_width[j] = cl.n[j] >= 2 ? z * sqrt(ss[j] / (double)(cl.n[j] - 1) / (double)cl.n[j])
                                                : INFINITY;
            // best mean among the actions seen; decided only if its interval
            // lies strictly above every other seen action's interval
            int best = -1;
            for (int j = 0; j < 3; ++j)
                if (cl.n[j] > 0 && (best < 0 || cl.mean_rate[j] > cl.mean_rate[best])) best = j;
            bool decided = best >= 0 && cl.n[best] >= 2;
            for (int j = 0; j < 3 && decided; ++j)
                if (j != best && cl.n[j] > 0 &&
                    !(cl.mean_rate[best] - cl.half_width[best] > cl.mean_rate[j] + cl.half_width[j]))
                    decided = false;
            cl.best = decided ? 1 - best : SRJ_ACTION_NONE;
            if (n < cap) out[n] = cl;
            ++n;
        }
    }
    *n_out = n;
    return SRJ_OK;
}

srj_status srj_fit_rule(const srj_cluster *clusters, int32_t count, double *t_low, double *t_high,
                        int32_t *agree, int32_t *decided)
{
    if ((!clusters && count > 0) || !t_low || !t_high || !agree || !decided)
        return fail(SRJ_ERR_INVALID, "NULL argument");
    if (count < 0) return fail(SRJ_ERR_INVALID, "count must be >= 0");
    std::vector<const srj_cluster *> d;
    for (int32_t i = 0; i < count; ++i)
        if (clusters[i].best >= -1 && clusters[i].best <= 1) d.push_back(&clusters[i]);
    std::stable_sort(d.begin(), d.end(), [](const srj_cluster *a, const srj_cluster *b) {
        return a->mean_ratio < b->mean_ratio;
    });
    const int64_t m = (int64_t)d.size();
    *decided = (int32_t)m;
    if (m == 0) {
        *t_low = 0.0;
        *t_high = 0.0;
        *agree = 0;
        return SRJ_OK;
    }
    // prefix counts of keep / down / up among the first i decided clusters
    std::vector<int64_t> kp(m + 1, 0), dn(m + 1, 0), up(m + 1, 0);
    for (int64_t i = 0; i < m; ++i) {
        kp[i + 1] = kp[i] + (d[i]->best == 0);
        dn[i + 1] = dn[i] + (d[i]->best == -1);
        up[i + 1] = up[i] + (d[i]->best == 1);
    }
    // thresholds sit between consecutive clusters: clusters [0, i) keep,
    // [i, j) step down, [j, m) step up; the first best split wins
    int64_t bi = 0, bj = 0, bagree = -1;
    for (int64_t i = 0; i <= m; ++i)
        for (int64_t j = i; j <= m; ++j) {
            const int64_t ag = kp[i] + (dn[j] - dn[i]) + (up[m] - up[j]);
            if (ag > bagree) {
                bagree = ag;
                bi = i;
                bj = j;
            }
        }
    auto cut = [&](int64_t i) -> double {
        if (i <= 0) return 0.0;
        if (i >= m) return d[m - 1]->mean_ratio;
        return 0.5 * (d[i - 1]->mean_ratio + d[i]->mean_ratio);
    };
    *t_low = cut(bi);
    *t_high = cut(bj);
    *agree = (int32_t)bagree;
    return SRJ_OK;
}

}  // extern "C"
