// The one-workgroup SRJ solve on a grid held in LDS, shared by the
// resident solver (resident.hip) and the coarsest grid of the multigrid
// tail (mg.hip): the sweeps of each cycle's scheme (Islam & Wang, arXiv
// 2011.06636, section 2, Eq. 3 and Eq. 7, Eq. (17) factors in the library's
// execution order), the L2 residual norm after the cycle (a fixed-order
// workgroup reduction), the next level from Algorithm 1 (section 3) and the
// stopping test, every thread taking the same decisions from the same
// broadcast norm.
#pragma once

#include <math.h>

#include "internal.h"
#include "rowsum.h"

#pragma clang fp contract(off)

namespace srj {

constexpr int kThreads = 1024;
constexpr int kPPT = 4;  // points per thread

struct ResidentOut {
    int32_t status, converged, cycles, final_level;
    int64_t sweeps;
    double r0, r_final, min_margin;
};

struct ResidentArgs {
    int32_t rule, fixed_level, max_level, max_cycles, start_level, tol_mode;
    int64_t max_sweeps;
    double tol, r0_given;
};

// Largest of the threads' values (bit patterns of non-negative doubles, which
// order like the values; a NaN orders above everything), broadcast.
__device__ inline unsigned long long group_max_bits(unsigned long long v, double *red)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const unsigned long long o = __shfl_xor(v, off);
        v = o > v ? o : v;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wave] = __longlong_as_double((long long)v);
    __syncthreads();
    const int nw = blockDim.x / 64;
    if (threadIdx.x == 0) {
        unsigned long long t = (unsigned long long)__double_as_longlong(red[0]);
        for (int i = 1; i < nw; ++i) {
            const unsigned long long u = (unsigned long long)__double_as_longlong(red[i]);
            t = u > t ? u : t;
        }
        red[kThreads / 64] = __longlong_as_double((long long)t);
    }
    __syncthreads();
    return (unsigned long long)__double_as_longlong(red[kThreads / 64]);
}

// Fixed-order sum over the workgroup, broadcast to every thread.
__device__ inline double group_sum(double v, double *red)
{
    v = wave_sum64(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    const int nw = blockDim.x / 64;
    if (threadIdx.x == 0) {
        double t = red[0];
        for (int i = 1; i < nw; ++i) t += red[i];
        red[kThreads / 64] = t;
    }
    __syncthreads();
    return red[kThreads / 64];
}

// The whole solve on a grid held in LDS (cur: the iterate, nxt: its
// ping-pong partner, red: kThreads / 64 + 1 values of reduction space), by
// every thread of the workgroup; b is read from bsrc (global memory or LDS).
// Returns the buffer holding the final iterate and fills *out (thread 0).
// UPD: the update stopping test (a.tol_mode == SRJ_TOL_UPDATE_INF); a
// template argument so that the residual-test kernel carries none of it.
template <bool UPD>
__device__ double *resident_run(const DevProblem &P, double *cur, double *nxt, double *red,
                                const double *bsrc, const double *__restrict__ omega,
                                const int32_t *__restrict__ offsets,
                                const int32_t *__restrict__ levelM, const ResidentArgs &a,
                                int32_t *__restrict__ levels_hist, double *__restrict__ norms_hist,
                                ResidentOut *__restrict__ out, const ResidentRecord &rec)
{
    const int64_t N = P.n0 * P.n1 * P.n2;
    // this thread's points: p = threadIdx.x + k * blockDim.x
    int64_t pi[kPPT], c0[kPPT], c1[kPPT], c2[kPPT];
    double bv[kPPT], dinv[kPPT];
#pragma unroll
    for (int k = 0; k < kPPT; ++k) {
        const int64_t p = threadIdx.x + (int64_t)k * blockDim.x;
        pi[k] = p < N ? p : -1;
        c0[k] = p % P.n0;
        c1[k] = (p / P.n0) % P.n1;
        c2[k] = p / (P.n0 * P.n1);
        bv[k] = p < N ? bsrc[p] : 0.0;
        dinv[k] = p < N ? (P.diag ? P.dinv[p] : P.dinvconst) : 0.0;
    }
    __syncthreads();
    auto norm_of = [&](const double *u) -> double {
        double acc = 0.0;
#pragma unroll
        for (int k = 0; k < kPPT; ++k) {
            if (pi[k] < 0) continue;
            const double r = bv[k] - row_s(P, u, pi[k], c0[k], c1[k], c2[k]);
            acc += r * r;
        }
        return sqrt(group_sum(acc, red));
    };
    const double norm0 = norm_of(cur);
    const double r0 = a.r0_given > 0.0 ? a.r0_given : norm0;
    const double target = a.tol_mode == SRJ_TOL_RELATIVE ? a.tol * r0 : a.tol;
    // the update test (section 4.2.2, Eq. (25)): stop at the first sweep whose
    // largest |x' - x| is below tol; the selector still runs on cycle-end norms
    constexpr bool upd = UPD;
    if (threadIdx.x == 0) norms_hist[0] = norm0;
    int status = SRJ_ERR_NOT_CONVERGED, cycles = 0, level = a.start_level, last_level = a.start_level;
    int64_t sweeps = 0;
    double prev = norm0, last = norm0, margin = INFINITY;
    if (!isfinite(norm0)) {
        status = SRJ_ERR_NONFINITE;
    } else if (norm0 == 0.0 || (!upd && norm0 < target)) {
        status = SRJ_OK;
    } else {
        for (int cycle = 0; cycle < a.max_cycles; ++cycle) {
            const int lv = a.rule == SRJ_RULE_FIXED ? a.fixed_level : level;
            const int M = levelM[lv];
            if (sweeps + M > a.max_sweeps) break;
            const double *w = omega + offsets[lv];
            double wnext = w[0];
            int done = M;          // sweeps of this cycle that count
            bool stopped = false;  // the update test held after sweep done - 1
            for (int j = 0; j < M; ++j) {
                const double wj = wnext;
                if (j + 1 < M) wnext = w[j + 1];  // in flight during this sweep
                unsigned long long dmax = 0ull;
#pragma unroll
                for (int k = 0; k < kPPT; ++k) {
                    if (pi[k] < 0) continue;
                    const double s = row_s(P, cur, pi[k], c0[k], c1[k], c2[k]);
                    const double r = bv[k] - s;
                    const double t = dinv[k] * r;
                    const double xn = cur[pi[k]] + wj * t;
                    nxt[pi[k]] = xn;
                    if (upd) {
                        const unsigned long long d =
                            (unsigned long long)__double_as_longlong(fabs(xn - cur[pi[k]]));
                        dmax = d > dmax ? d : dmax;
                    }
                }
                __syncthreads();
                double *tmp = cur;
                cur = nxt;
                nxt = tmp;
                if (upd && __longlong_as_double((long long)group_max_bits(dmax, red)) < a.tol) {
                    done = j + 1;  // every thread takes the same decision
                    stopped = true;
                    break;
                }
            }
            sweeps += done;
            const double norm = norm_of(cur);
            cycles = cycle + 1;
            last = norm;
            last_level = lv;
            if (threadIdx.x == 0) {
                levels_hist[cycle] = lv;
                norms_hist[cycle + 1] = norm;
            }
            if (!isfinite(norm)) {
                status = SRJ_ERR_NONFINITE;
                break;
            }
            if (upd ? stopped : norm < target) {
                status = SRJ_OK;
                break;
            }
            const double ratio = norm / prev;
            prev = norm;
            int nl = level;
            if (a.rule == SRJ_RULE_HEURISTIC) {
                margin = fmin(margin, fmin(fabs(ratio - 0.2), fabs(ratio - 0.4)));
                if (ratio > 0.4)
                    nl = level + 1;
                else if (ratio < 0.4 && ratio > 0.2)
                    nl = level - 1;
            } else if (a.rule == SRJ_RULE_INCREASING) {
                nl = level + 1;
            }
            level = nl < 0 ? 0 : (nl > a.max_level ? a.max_level : nl);
        }
    }
    if (threadIdx.x == 0) {
        out->status = status;
        out->converged = status == SRJ_OK;
        out->cycles = cycles;
        out->final_level = cycles > 0 ? last_level : a.start_level;
        out->sweeps = sweeps;
        out->r0 = r0;
        out->r_final = last;
        out->min_margin = margin;
        if (rec.sweeps) {
            // appended to the caller's device record in stream order
            const int32_t i = *rec.count;
            if (i < rec.cap) rec.sweeps[i] = sweeps;
            *rec.count = i + 1;
            if (status != SRJ_OK && status != SRJ_ERR_NOT_CONVERGED) *rec.bad = status;
        }
    }
    return cur;
}

}  // namespace srj
