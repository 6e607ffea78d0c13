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
#include <string.h>

#include <algorithm>
#include <string>

#include "internal.h"
#include "resident_run.h"
#include "rowsum.h"
#include "tile2d.h"

#pragma clang fp contract(off)

namespace srj {

namespace {

// Constant-coefficient 1D grids of at most 64 K points in one wave: lane l
// holds points l K .. l K + K - 1 in registers, the neighbours across lanes
// come by DPP, and nothing waits at a barrier.  The per-point arithmetic is
// the sweep's expression (row_s order: D u, then the lower and the upper
// neighbour, ghost terms omitted), so iterates are bit-identical to the
// workgroup kernel's; the norm is a fixed-order wave reduction (each lane's
// points in order, then a shift-down tree), broadcast from lane 0.  The
// factor table is staged in LDS as far as the levels reached need it, up to
// its first kWaveTab values (the library's family up to level 21); a level
// beyond them is staged cycle by cycle, kWaveW factors at a time.  Each
// sweep's factor is read from LDS one sweep ahead.
constexpr int kWaveTab = 6144;
constexpr int kWaveW = 2048;
constexpr int64_t kWaveMaxPoints = 64 * 8;

// dst[0 .. n) = src[0 .. n) by one wave, eight loads per lane in flight at a
// time (each load is unconditional, at an index clamped into the array)
__device__ __forceinline__ void wave_stage(double *dst, const double *__restrict__ src, int n)
{
    const int lane = threadIdx.x;
    for (int i0 = 0; i0 < n; i0 += 64 * 8) {
        double v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int i = i0 + q * 64 + lane;
            v[q] = src[i < n ? i : n - 1];
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int i = i0 + q * 64 + lane;
            if (i < n) dst[i] = v[q];
        }
    }
}

__device__ __forceinline__ double wave_bcast0(double v)
{
    const int lo = __builtin_amdgcn_readfirstlane(__double2loint(v));
    const int hi = __builtin_amdgcn_readfirstlane(__double2hiint(v));
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double wave_total(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return wave_bcast0(v);
}

template <bool UPD, int K>
__global__ __launch_bounds__(64) void k_resident_wave1d(DevProblem P, double *__restrict__ x,
                                                        const double *__restrict__ omega,
                                                        const int32_t *__restrict__ offsets,
                                                        const int32_t *__restrict__ levelM,
                                                        ResidentArgs a,
                                                        int32_t *__restrict__ levels_hist,
                                                        double *__restrict__ norms_hist,
                                                        ResidentOut *__restrict__ out,
                                                        ResidentRecord rec)
{
    __shared__ double tab[kWaveTab];
    __shared__ double wl[kWaveW];
    const int lane = threadIdx.x;
    int staged = 0;  // factors [0, staged) of the table are in tab
    const int64_t N = P.n0;
    const double D = P.dconst, c = P.c[0], Dinv = P.dinvconst;
    double u[K], bv[K];
    bool in[K], lo[K], hi[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int64_t p = (int64_t)lane * K + k;
        in[k] = p < N;
        lo[k] = p > 0;
        hi[k] = p < N - 1;
        u[k] = in[k] ? x[p] : 0.0;
        bv[k] = in[k] ? P.b[p] : 0.0;
    }
    // s_p = D u_p - c u_{p-1} - c u_{p+1}, ghost terms omitted
    auto row = [&](const double *v, int k, double left, double right) {
        double s = D * v[k];
        if (lo[k]) s = s - c * (k > 0 ? v[k - 1] : left);
        if (hi[k]) s = s - c * (k + 1 < K ? v[k + 1] : right);
        return s;
    };
    auto norm_of = [&]() -> double {
        const double left = dpp_prev(u[K - 1]), right = dpp_next(u[0]);
        double acc = 0.0;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const double r = bv[k] - row(u, k, left, right);
            acc = in[k] ? acc + r * r : acc;
        }
        return sqrt(wave_total(acc));
    };
    const double norm0 = norm_of();
    const double r0 = a.r0_given > 0.0 ? a.r0_given : norm0;
    const double target = a.tol_mode == SRJ_TOL_RELATIVE ? a.tol * r0 : a.tol;
    if (lane == 0) norms_hist[0] = norm0;
    int status = SRJ_ERR_NOT_CONVERGED, cycles = 0, level = a.start_level, last_level = a.start_level;
    int64_t sweeps = 0;
    double prev = norm0, last = norm0, margin = INFINITY;
    if (!isfinite(norm0)) {
        status = SRJ_ERR_NONFINITE;
    } else if (norm0 == 0.0 || (!UPD && norm0 < target)) {
        status = SRJ_OK;
    } else {
        for (int cycle = 0; cycle < a.max_cycles; ++cycle) {
            const int lv = a.rule == SRJ_RULE_FIXED ? a.fixed_level : level;
            const int M = levelM[lv];
            if (sweeps + M > a.max_sweeps) break;
            const int off = offsets[lv];
            int done = M;          // sweeps of this cycle that count
            bool stopped = false;  // the update test held after sweep done - 1
            // sweeps base .. base + cnt - 1 of the cycle with factors src[0 ..)
            auto sweep_run = [&](const double *src, int base, int cnt) {
                double wnext = src[0];
                for (int j = 0; j < cnt; ++j) {
                    const double wj = wnext;
                    if (j + 1 < cnt) wnext = src[j + 1];  // in flight during this sweep
                    const double left = dpp_prev(u[K - 1]), right = dpp_next(u[0]);
                    double un[K];
                    unsigned long long dmax = 0ull;
#pragma unroll
                    for (int k = 0; k < K; ++k) {
                        const double r = bv[k] - row(u, k, left, right);
                        const double t = Dinv * r;
                        const double xn = u[k] + wj * t;
                        // points past N are never read by a point of the grid (its
                        // neighbour terms beyond N - 1 are omitted), so whatever
                        // the sweep makes of them stays unused: no select
                        un[k] = xn;
                        if (UPD && in[k]) {
                            const unsigned long long d =
                                (unsigned long long)__double_as_longlong(fabs(xn - u[k]));
                            dmax = d > dmax ? d : dmax;
                        }
                    }
#pragma unroll
                    for (int k = 0; k < K; ++k) u[k] = un[k];
                    if (UPD) {
#pragma unroll
                        for (int sh = 32; sh > 0; sh >>= 1) {
                            const unsigned long long o = __shfl_xor(dmax, sh);
                            dmax = o > dmax ? o : dmax;
                        }
                        if (__longlong_as_double((long long)dmax) < a.tol) {
                            done = base + j + 1;
                            stopped = true;
                            return;
                        }
                    }
                }
            };
            if (off + M <= kWaveTab) {
                if (off + M > staged) {  // stage up to this level's last factor
                    wave_stage(tab + staged, omega + staged, off + M - staged);
                    __syncthreads();
                    staged = off + M;
                }
                if (M > 0) sweep_run(tab + off, 0, M);
            } else {
                for (int base = 0; base < M && !stopped; base += kWaveW) {
                    const int cnt = M - base < kWaveW ? M - base : kWaveW;
                    __syncthreads();  // the previous chunk's factors are read
                    wave_stage(wl, omega + off + base, cnt);
                    __syncthreads();
                    sweep_run(wl, base, cnt);
                }
            }
            sweeps += done;
            const double norm = norm_of();
            cycles = cycle + 1;
            last = norm;
            last_level = lv;
            if (lane == 0) {
                levels_hist[cycle] = lv;
                norms_hist[cycle + 1] = norm;
            }
            if (!isfinite(norm)) {
                status = SRJ_ERR_NONFINITE;
                break;
            }
            if (UPD ? stopped : norm < target) {
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
#pragma unroll
    for (int k = 0; k < K; ++k)
        if (in[k]) x[(int64_t)lane * K + k] = u[k];
    if (lane == 0) {
        out->status = status;
        out->converged = status == SRJ_OK;
        out->cycles = cycles;
        out->final_level = cycles > 0 ? last_level : a.start_level;
        out->sweeps = sweeps;
        out->r0 = r0;
        out->r_final = last;
        out->min_margin = margin;
        if (rec.sweeps) {
            const int32_t i = *rec.count;
            if (i < rec.cap) rec.sweeps[i] = sweeps;
            *rec.count = i + 1;
            if (status != SRJ_OK && status != SRJ_ERR_NOT_CONVERGED) *rec.bad = status;
        }
    }
}

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

// Layout of the pinned mirror: the record, then the norms (cap + 1), then
// the levels (cap).
size_t mirror_bytes(int64_t cap) { return kOutBytes + sizeof(double) * (size_t)(cap + 1) + sizeof(int32_t) * (size_t)cap; }

// After a solve: the record and its cycles' levels and norms into the mirror
// (host memory, written through its device mapping).
__global__ __launch_bounds__(256) void k_resident_publish(const ResidentOut *__restrict__ dout,
                                                          const int32_t *__restrict__ lh,
                                                          const double *__restrict__ nh,
                                                          char *__restrict__ mirror, int64_t cap)
{
    const ResidentOut h = *dout;
    const int64_t nc = h.cycles < 0 ? 0 : (h.cycles > cap ? cap : h.cycles);
    double *mn = reinterpret_cast<double *>(mirror + kOutBytes);
    int32_t *ml = reinterpret_cast<int32_t *>(mirror + kOutBytes + sizeof(double) * (cap + 1));
    for (int64_t k = threadIdx.x; k <= nc; k += blockDim.x) mn[k] = nh[k];
    for (int64_t k = threadIdx.x; k < nc; k += blockDim.x) ml[k] = lh[k];
    if (threadIdx.x == 0) *reinterpret_cast<ResidentOut *>(mirror) = h;
}

// Device buffers kept by the context from one solve to the next: the result
// record, the level sizes and offsets (fixed size), the histories, and the
// pinned mirror of the record and histories.
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
        (void)hipHostFree(c->rs_host);
        c->rs_levels = nullptr;
        c->rs_norms = nullptr;
        c->rs_host = c->rs_host_dev = nullptr;
        c->rs_cap = 0;
        if (hipMalloc(&c->rs_levels, sizeof(int32_t) * (size_t)max_cycles) != hipSuccess ||
            hipMalloc(&c->rs_norms, sizeof(double) * ((size_t)max_cycles + 1)) != hipSuccess ||
            hipHostMalloc(&c->rs_host, mirror_bytes(max_cycles), 0) != hipSuccess ||
            hipHostGetDevicePointer(&c->rs_host_dev, c->rs_host, 0) != hipSuccess) {
            (void)hipFree(c->rs_levels);
            (void)hipFree(c->rs_norms);
            (void)hipHostFree(c->rs_host);
            c->rs_levels = nullptr;
            c->rs_norms = nullptr;
            c->rs_host = c->rs_host_dev = nullptr;
            return fail(SRJ_ERR_NOMEM, "allocation failed for resident solve");
        }
        c->rs_cap = max_cycles;
    }
    return SRJ_OK;
}

// The level sizes and the offsets of c's scheme family into the tables of
// rs_fixed, on c's stream, when they differ from what the tables hold.
srj_status resident_upload_tables(srj_ctx *c)
{
    std::vector<int32_t> t(SRJ_NUM_LEVELS);
    for (int l = 0; l < SRJ_NUM_LEVELS; ++l) t[l] = l < c->nlevels ? c->levelM[l] : 0;
    t.insert(t.end(), c->offsets.begin(), c->offsets.end());
    if (t == c->rs_tables) return SRJ_OK;
    c->rs_tables.clear();
    char *fixed = static_cast<char *>(c->rs_fixed);
    SRJ_HIP_CHECK(hipMemcpyAsync(fixed + kOutBytes, t.data(), sizeof(int32_t) * SRJ_NUM_LEVELS,
                                 hipMemcpyHostToDevice, c->stream));
    SRJ_HIP_CHECK(hipMemcpyAsync(fixed + kOutBytes + kLmBytes, t.data() + SRJ_NUM_LEVELS,
                                 sizeof(int32_t) * c->offsets.size(), hipMemcpyHostToDevice,
                                 c->stream));
    SRJ_HIP_CHECK(hipStreamSynchronize(c->stream));  // t is a local buffer
    c->rs_tables = std::move(t);
    return SRJ_OK;
}

size_t resident_shmem(int64_t N) { return sizeof(double) * (size_t)(2 * N + kThreads / 64 + 1); }

// one point per thread up to 1024 points (latency hiding across waves), then
// up to kPPT points per thread
int resident_threads(int64_t N)
{
    return (int)std::min<int64_t>(kThreads, std::max<int64_t>(64, (N + 63) / 64 * 64));
}

// Constant-coefficient grids of one row (any dimension: with n1 = n2 = 1 the
// axis-1 and axis-2 neighbours are all ghosts, whose terms the expression
// omits, so it is the 1D one; the coarsest grids of 2D and 3D multigrid
// hierarchies are such) of at most kWaveMaxPoints points.
bool wave1d_fits(const DevProblem &P)
{
    return P.n1 == 1 && P.n2 == 1 && !P.diag && !P.face[0] && !P.face[1] && !P.face[2] &&
           !P.ell_len && P.n0 <= kWaveMaxPoints;
}

// The resident kernel for c's grid: one wave for small constant-coefficient
// 1D grids, else one workgroup with the grid in LDS.
template <bool UPD>
void launch_resident(const srj_ctx *c, double *x, const int32_t *offs, const int32_t *lm,
                     const ResidentArgs &a, int32_t *lh, double *nh, ResidentOut *dout,
                     const ResidentRecord &rec)
{
    const int64_t N = c->npoints;
    if (wave1d_fits(c->P)) {
        const int64_t K = (N + 63) / 64;
#define SRJ_W1(KK)                                                                              \
        hipLaunchKernelGGL((k_resident_wave1d<UPD, KK>), dim3(1), dim3(64), 0, c->stream, c->P, x, \
                           c->omega_dev, offs, lm, a, lh, nh, dout, rec)
        if (K <= 1) SRJ_W1(1);
        else if (K <= 2) SRJ_W1(2);
        else if (K <= 4) SRJ_W1(4);
        else SRJ_W1(8);
#undef SRJ_W1
        return;
    }
    hipLaunchKernelGGL(k_resident<UPD>, dim3(1), dim3(resident_threads(N)), resident_shmem(N),
                       c->stream, c->P, x, c->omega_dev, offs, lm, a, lh, nh, dout, rec);
}

}  // namespace

srj_status resident_prepare(srj_ctx *c, int max_cycles)
{
    srj_status st = resident_buffers(c, max_cycles);
    if (st != SRJ_OK) return st;
    return resident_upload_tables(c);
}

srj_status resident_tables(srj_ctx *c, const srj_solve_opts *o, ResidentArgs *a,
                           const int32_t **level_m, const int32_t **offsets)
{
    if (o->tol_mode == SRJ_TOL_UPDATE_INF || o->max_cycles > c->rs_cap || !c->rs_fixed)
        return fail(SRJ_ERR_INVALID, "resident tables: buffers not prepared for these options");
    const char *fixed = static_cast<const char *>(c->rs_fixed);
    *level_m = reinterpret_cast<const int32_t *>(fixed + kOutBytes);
    *offsets = reinterpret_cast<const int32_t *>(fixed + kOutBytes + kLmBytes);
    *a = resident_args(o);
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
    launch_resident<false>(c, x, offs, lm, resident_args(o), c->rs_levels, c->rs_norms, dout, rec);
    SRJ_HIP_CHECK(hipGetLastError());
    return SRJ_OK;
}

srj_status resident_solve(srj_ctx *c, double *x, const srj_solve_opts *o, srj_solve_result *res,
                          int32_t *levels_out, double *norms_out)
{
    const ResidentArgs a = resident_args(o);
    {
        srj_status sb = resident_buffers(c, o->max_cycles);
        if (sb == SRJ_OK) sb = resident_upload_tables(c);
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
    {
        hipError_t e = hipSuccess;
        if (c->profiling) e = hipEventRecord(c->ev0, c->stream);
        if (e == hipSuccess) {
            if (a.tol_mode == SRJ_TOL_UPDATE_INF)
                launch_resident<true>(c, x, offs, lm, a, lh, nh, dout, ResidentRecord{});
            else
                launch_resident<false>(c, x, offs, lm, a, lh, nh, dout, ResidentRecord{});
            e = hipGetLastError();
        }
        if (c->profiling && e == hipSuccess) e = hipEventRecord(c->ev1, c->stream);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(k_resident_publish, dim3(1), dim3(256), 0, c->stream, dout, lh, nh,
                               static_cast<char *>(c->rs_host_dev), c->rs_cap);
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e == hipSuccess) {
            const char *m = static_cast<const char *>(c->rs_host);
            memcpy(&h, m, sizeof(h));
            const int64_t nc = std::min<int64_t>(std::max(h.cycles, 0), c->rs_cap);
            if (norms_out) memcpy(norms_out, m + kOutBytes, sizeof(double) * (size_t)(nc + 1));
            if (levels_out)
                memcpy(levels_out, m + kOutBytes + sizeof(double) * (size_t)(c->rs_cap + 1),
                       sizeof(int32_t) * (size_t)nc);
        }
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
