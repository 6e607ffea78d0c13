// Whole solve of a small problem inside one workgroup (one launch).
//
// For grids of at most kResidentMax points the iterate lives in LDS (two
// ping-pong copies) and one workgroup (one thread per point up to 1024
// threads, then up to four points per thread) runs every cycle of the
// solve: the sweeps of the cycle's scheme (Islam & Wang, arXiv 2011.06636,
// section 2, Eq. 3 and Eq. 7, Eq. (17) factors in the library's execution
// order), the L2 residual norm after the cycle (a fixed-order block
// reduction), the next level from Algorithm 1 (section 3) and the stopping
// test — with no host round trip per cycle.  Every thread takes the same
// decisions from the same broadcast norm.  The per-point arithmetic is the
// binary64 expression of the other kernels, so iterates are bit-identical;
// the norms differ from the multi-kernel path only in summation order.
#include <math.h>

#include <algorithm>
#include <string>

#include "internal.h"
#include "resident_run.h"
#include "rowsum.h"

#pragma clang fp contract(off)

namespace srj {

namespace {

// One workgroup solves the whole grid: x is copied into LDS, solved there
// and copied back.
template <bool UPD>
__global__ __launch_bounds__(kThreads) void k_resident(DevProblem P, double *__restrict__ x,
                                                       const double *__restrict__ omega,
                                                       const int32_t *__restrict__ offsets,
                                                       const int32_t *__restrict__ levelM,
                                                       ResidentArgs a, int32_t *__restrict__ levels_hist,
                                                       double *__restrict__ norms_hist,
                                                       ResidentOut *__restrict__ out,
                                                       ResidentRecord rec)
{
    extern __shared__ double lds[];
    const int64_t N = P.n0 * P.n1 * P.n2;
    double *cur = lds, *nxt = lds + N, *red = lds + 2 * N;
    for (int64_t p = threadIdx.x; p < N; p += blockDim.x) cur[p] = x[p];
    double *fin = resident_run<UPD>(P, cur, nxt, red, P.b, omega, offsets, levelM, a, levels_hist,
                                    norms_hist, out, rec);
    for (int64_t p = threadIdx.x; p < N; p += blockDim.x) x[p] = fin[p];
}

}  // namespace

bool resident_fits(const DevProblem &P) { return P.n0 * P.n1 * P.n2 <= kResidentMax; }

namespace {

constexpr size_t kOutBytes = 256, kLmBytes = 128, kOffsBytes = 128;

ResidentArgs resident_args(const srj_solve_opts *o)
{
    ResidentArgs a{};
    a.rule = o->rule;
    a.fixed_level = o->fixed_level;
    a.max_level = o->max_level;
    a.max_cycles = o->max_cycles;
    a.start_level = o->start_level;
    a.tol_mode = o->tol_mode;
    a.max_sweeps = o->max_sweeps;
    a.tol = o->tol;
    a.r0_given = o->r0;
    return a;
}

// Device buffers kept by the context from one solve to the next: the result
// record, the level sizes and offsets (fixed size), the histories.
srj_status resident_buffers(srj_ctx *c, int max_cycles)
{
    static_assert(sizeof(ResidentOut) <= kOutBytes, "result record");
    static_assert(sizeof(int32_t) * SRJ_NUM_LEVELS <= kLmBytes, "level sizes");
    static_assert(sizeof(int32_t) * (SRJ_NUM_LEVELS + 1) <= kOffsBytes, "level offsets");
    if (c->offsets.size() > (size_t)SRJ_NUM_LEVELS + 1)
        return fail(SRJ_ERR_INVALID, "scheme family larger than the level table");
    if (!c->rs_fixed && hipMalloc(&c->rs_fixed, kOutBytes + kLmBytes + kOffsBytes) != hipSuccess) {
        c->rs_fixed = nullptr;
        return fail(SRJ_ERR_NOMEM, "hipMalloc failed for resident solve");
    }
    if (c->rs_cap < max_cycles) {
        (void)hipFree(c->rs_levels);
        (void)hipFree(c->rs_norms);
        c->rs_levels = nullptr;
        c->rs_norms = nullptr;
        c->rs_cap = 0;
        if (hipMalloc(&c->rs_levels, sizeof(int32_t) * (size_t)max_cycles) != hipSuccess ||
            hipMalloc(&c->rs_norms, sizeof(double) * ((size_t)max_cycles + 1)) != hipSuccess) {
            (void)hipFree(c->rs_levels);
            c->rs_levels = nullptr;
            c->rs_norms = nullptr;
            return fail(SRJ_ERR_NOMEM, "hipMalloc failed for resident solve");
        }
        c->rs_cap = max_cycles;
    }
    return SRJ_OK;
}

std::vector<int32_t> level_sizes(const srj_ctx *c)
{
    std::vector<int32_t> lmh(SRJ_NUM_LEVELS);
    for (int l = 0; l < SRJ_NUM_LEVELS; ++l) lmh[l] = l < c->nlevels ? c->levelM[l] : 0;
    return lmh;
}

size_t resident_shmem(int64_t N) { return sizeof(double) * (size_t)(2 * N + kThreads / 64 + 1); }

// one point per thread up to 1024 points (latency hiding across waves), then
// up to kPPT points per thread
int resident_threads(int64_t N)
{
    return (int)std::min<int64_t>(kThreads, std::max<int64_t>(64, (N + 63) / 64 * 64));
}

}  // namespace

srj_status resident_prepare(srj_ctx *c, int max_cycles)
{
    srj_status st = resident_buffers(c, max_cycles);
    if (st != SRJ_OK) return st;
    char *fixed = static_cast<char *>(c->rs_fixed);
    const std::vector<int32_t> lmh = level_sizes(c);
    SRJ_HIP_CHECK(hipMemcpy(fixed + kOutBytes, lmh.data(), sizeof(int32_t) * SRJ_NUM_LEVELS,
                            hipMemcpyHostToDevice));
    SRJ_HIP_CHECK(hipMemcpy(fixed + kOutBytes + kLmBytes, c->offsets.data(),
                            sizeof(int32_t) * c->offsets.size(), hipMemcpyHostToDevice));
    return SRJ_OK;
}

srj_status resident_launch_recorded(srj_ctx *c, double *x, const srj_solve_opts *o,
                                    const ResidentRecord &rec)
{
    if (o->tol_mode == SRJ_TOL_UPDATE_INF || o->max_cycles > c->rs_cap || !c->rs_fixed)
        return fail(SRJ_ERR_INVALID, "resident launch: buffers not prepared for these options");
    char *fixed = static_cast<char *>(c->rs_fixed);
    ResidentOut *dout = reinterpret_cast<ResidentOut *>(fixed);
    const int32_t *lm = reinterpret_cast<const int32_t *>(fixed + kOutBytes);
    const int32_t *offs = reinterpret_cast<const int32_t *>(fixed + kOutBytes + kLmBytes);
    const int64_t N = c->npoints;
    hipLaunchKernelGGL(k_resident<false>, dim3(1), dim3(resident_threads(N)), resident_shmem(N),
                       c->stream, c->P, x, c->omega_dev, offs, lm, resident_args(o), c->rs_levels,
                       c->rs_norms, dout, rec);
    SRJ_HIP_CHECK(hipGetLastError());
    return SRJ_OK;
}

srj_status resident_solve(srj_ctx *c, double *x, const srj_solve_opts *o, srj_solve_result *res,
                          int32_t *levels_out, double *norms_out)
{
    const ResidentArgs a = resident_args(o);
    const int64_t N = c->npoints;
    const std::vector<int32_t> lmh = level_sizes(c);
    {
        const srj_status sb = resident_buffers(c, o->max_cycles);
        if (sb != SRJ_OK) return sb;
    }
    int32_t *lh = c->rs_levels;
    double *nh = c->rs_norms;
    char *fixed = static_cast<char *>(c->rs_fixed);
    ResidentOut *dout = reinterpret_cast<ResidentOut *>(fixed);
    int32_t *lm = reinterpret_cast<int32_t *>(fixed + kOutBytes);
    int32_t *offs = reinterpret_cast<int32_t *>(fixed + kOutBytes + kLmBytes);
    srj_status st = SRJ_OK;
    ResidentOut h{};
    if (st == SRJ_OK) {
        hipError_t e = hipMemcpyAsync(lm, lmh.data(), sizeof(int32_t) * SRJ_NUM_LEVELS,
                                      hipMemcpyHostToDevice, c->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(offs, c->offsets.data(), sizeof(int32_t) * c->offsets.size(),
                               hipMemcpyHostToDevice, c->stream);
        const size_t shmem = resident_shmem(N);
        if (c->profiling && e == hipSuccess) e = hipEventRecord(c->ev0, c->stream);
        if (e == hipSuccess) {
            const int threads = resident_threads(N);
            if (a.tol_mode == SRJ_TOL_UPDATE_INF)
                hipLaunchKernelGGL(k_resident<true>, dim3(1), dim3(threads), shmem, c->stream, c->P,
                                   x, c->omega_dev, offs, lm, a, lh, nh, dout, ResidentRecord{});
            else
                hipLaunchKernelGGL(k_resident<false>, dim3(1), dim3(threads), shmem, c->stream,
                                   c->P, x, c->omega_dev, offs, lm, a, lh, nh, dout, ResidentRecord{});
            e = hipGetLastError();
        }
        if (c->profiling && e == hipSuccess) e = hipEventRecord(c->ev1, c->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(&h, dout, sizeof(h), hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e == hipSuccess && levels_out && o->max_cycles > 0)
            e = hipMemcpy(levels_out, lh, sizeof(int32_t) * (size_t)o->max_cycles,
                          hipMemcpyDeviceToHost);
        if (e == hipSuccess && norms_out)
            e = hipMemcpy(norms_out, nh, sizeof(double) * ((size_t)h.cycles + 1),
                          hipMemcpyDeviceToHost);
        if (e == hipSuccess && c->profiling) {
            float ms = 0.f;
            e = hipEventElapsedTime(&ms, c->ev0, c->ev1);
            c->prof_ms += ms;
            c->prof_launches += 1;
            c->prof_sweeps += h.sweeps;
        }
        if (e != hipSuccess) st = fail(SRJ_ERR_HIP, std::string("resident solve: ") + hipGetErrorString(e));
    }
    if (st != SRJ_OK) return st;
    res->converged = h.converged;
    res->cycles = h.cycles;
    res->final_level = h.final_level;
    res->sweeps = h.sweeps;
    res->r0 = h.r0;
    res->r_final = h.r_final;
    res->min_margin = h.min_margin;
    if (h.status == SRJ_ERR_NONFINITE) return fail(SRJ_ERR_NONFINITE, "residual norm is not finite");
    if (h.status == SRJ_ERR_NOT_CONVERGED) return fail(SRJ_ERR_NOT_CONVERGED, "cycle or sweep cap reached");
    return SRJ_OK;
}

}  // namespace srj
