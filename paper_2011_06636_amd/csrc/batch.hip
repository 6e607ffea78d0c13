// Batched SRJ solves: many independent problems of uneven sizes advanced by
// the same launches, each with its own scheme choice (Islam & Wang, arXiv
// 2011.06636, section 3, Algorithm 1) and its own stopping test.
//
// Every instance's arrays live packed in a few large buffers.  Per-instance
// device state holds the level, the number of sweeps done in the current
// cycle, the parities of its ping-pong buffers, its norms and its refinement
// scale.  One step is
//   1. sweeps: every active instance advances its cycle by T sweeps (2D and
//      1D instances: register tiles, T <= tile halo; 3D instances: one
//      sweep of register plane tiles streamed along axis 2); waves loop over
//      (instance, tile) work items;
//   2. outer pass over the points of the instances whose cycle just ended:
//      binary64 residual (refinement: after x += d / s, with the scaled cast
//      of the residual for the next cycle and the next correction zeroed),
//      one partial sum of squares per work item;
//   3. finalize, one block per instance: fold its partials in a fixed order,
//      and at a cycle end apply Algorithm 1, the stop test and the caps.
// A fixed number of steps is captured in a hipGraph; the graph is replayed
// until every instance is done (the done count is the only value read back
// per replay).  Problems must have constant couplings and diagonal.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "internal.h"
#include "storage.h"
#include "stream3d.h"
#include "tile2d.h"
#include "plane3d.h"
#include "plane3d_fused.h"
#include "block2d.h"

#pragma clang fp contract(off)

namespace srj {

namespace {

constexpr int kOuterPts = 2048;  // points per outer-pass work item (256 threads x 8)
// 3D plane tiles of the batched sweep (rows per tile, planes per work item)
#define SRJ_BATCH_PLANE(X) X(2, 16) X(4, 8) X(4, 16) X(8, 8) X(8, 16)

struct BDesc {
    int32_t ndim;
    int32_t pad0;
    int64_t n0, n1, n2, npts, off;
    double c[3], D, Dinv, sqrtN;
    float c32[3], D32, Dinv32, pad1;
    int32_t tiles_x, gx3, gy3, pad2;     // 2D tile columns; 3D plane-tile grid (x, y)
    int32_t oitem_first, oitem_count;    // outer-pass work items
};

struct BState {
    int32_t level, pos, pu, px;
    int32_t cycles, done, status, pad;
    int64_t sweeps;
    double r0, prev, target, s, min_margin, last;
};

struct BParams {
    int32_t rule, fixed_level, max_level, max_cycles;
    int64_t max_sweeps;
    int32_t tol_mode, T2, T3, pad3_;
    double tol, tgt_rms, r0_given;
    const int32_t *levelM;
    const int32_t *offsets;
    const double *omega64;
    const float *omega32;
};

template <class A>
struct Sel;
template <>
struct Sel<double> {
    __device__ static const double *omega(const BParams &p) { return p.omega64; }
    __device__ static Coef2D<double> coef2(const BDesc &d) { return {d.D, d.Dinv, d.c[0], d.c[1]}; }
    __device__ static Stencil3<double> sten(const BDesc &d)
    {
        return {d.n0, d.n1, d.n2, {d.c[0], d.c[1], d.c[2]}, {nullptr, nullptr, nullptr},
                d.D, d.Dinv, nullptr, nullptr};
    }
};
template <>
struct Sel<float> {
    __device__ static const float *omega(const BParams &p) { return p.omega32; }
    __device__ static Coef2D<float> coef2(const BDesc &d) { return {d.D32, d.Dinv32, d.c32[0], d.c32[1]}; }
    __device__ static Stencil3<float> sten(const BDesc &d)
    {
        return {d.n0, d.n1, d.n2, {d.c32[0], d.c32[1], d.c32[2]}, {nullptr, nullptr, nullptr},
                d.D32, d.Dinv32, nullptr, nullptr};
    }
};

__device__ __forceinline__ int sweeps_this_step(const BDesc &d, const BState &s, const BParams &p)
{
    const int M = p.levelM[s.level];
    const int left = M - s.pos;
    const int T = d.ndim == 3 ? p.T3 : p.T2;
    return left < T ? left : T;
}

__device__ __forceinline__ double pow2_scale_dev(double norm, double sqrtN, double tgt)
{
    if (!(norm > 0.0) || !isfinite(norm)) return 1.0;
    const double q = tgt * sqrtN / norm;
    int e = 0;
    frexp(q, &e);
    return ldexp(1.0, e - 1);
}

// 1. sweeps, 2D/1D instances: one wave per (instance, tile) item
template <class V, int H, int HALO>
__global__ __launch_bounds__(256) void k_bsweep2d(const BDesc *__restrict__ desc,
                                                  const BState *__restrict__ st,
                                                  const int2 *__restrict__ items, int nitems,
                                                  typename V::T *ua, typename V::T *ub,
                                                  const typename V::T *__restrict__ rhs, BParams prm)
{
    using A = typename V::A;
    const int lane = threadIdx.x & 63;
    const int nwaves = gridDim.x * 4;
    for (int item = blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); item < nitems; item += nwaves) {
        const int2 it = items[item];
        const BState s = st[it.x];
        if (s.done) continue;
        const BDesc &d = desc[it.x];
        const int T = sweeps_this_step(d, s, prm);
        const A *w = Sel<A>::omega(prm) + prm.offsets[s.level] + s.pos;
        const typename V::T *uin = (s.pu ? ub : ua) + d.off;
        typename V::T *uout = (s.pu ? ua : ub) + d.off;
        tile2d_run<V, H, HALO, false>(d.n0, d.n1, uin, uout, rhs + d.off, w, T, Sel<A>::coef2(d),
                                      it.y % d.tiles_x, it.y / d.tiles_x, lane, nullptr);
    }
}

// 1 (blocks). sweeps, 2D/1D instances: one workgroup of NW cooperating waves
// per (instance, block) item.  The workgroups of one XCD take the items of
// one contiguous range in turn (hardware places workgroup i on XCD i % 8), so
// neighbouring blocks of an instance share that XCD's L2.
template <class V, int HW, int HALO, int NW>
__global__ __launch_bounds__(64 * NW) void k_bsweep2d_blk(const BDesc *__restrict__ desc,
                                                          const BState *__restrict__ st,
                                                          const int2 *__restrict__ items, int nitems,
                                                          typename V::T *ua, typename V::T *ub,
                                                          const typename V::T *__restrict__ rhs,
                                                          BParams prm)
{
    using A = typename V::A;
    __shared__ A edge[2 * 2 * NW * 64];
    const int per_xcd = (nitems + 7) / 8;
    const int xcd = blockIdx.x % 8, stride = gridDim.x / 8;
    const int end = min((xcd + 1) * per_xcd, nitems);
    int kbase = 0;
    for (int item = xcd * per_xcd + blockIdx.x / 8; item < end; item += stride) {
        const int2 it = items[item];
        const BState s = st[it.x];
        if (s.done) continue;  // uniform over the workgroup
        const BDesc &d = desc[it.x];
        const int T = sweeps_this_step(d, s, prm);
        const A *w = Sel<A>::omega(prm) + prm.offsets[s.level] + s.pos;
        const typename V::T *uin = (s.pu ? ub : ua) + d.off;
        typename V::T *uout = (s.pu ? ua : ub) + d.off;
        block2d_item<V, HW, HALO, NW, 1>(d.n0, d.n1, uin, uout, rhs + d.off, w, T,
                                         Sel<A>::coef2(d), it.y % d.tiles_x, it.y / d.tiles_x,
                                         false, threadIdx.x >> 6, threadIdx.x & 63, edge, kbase);
        kbase += T;
    }
}

// 1'. sweeps, 3D instances: one wave per (instance, plane tile) item; a
// tile is 62 written columns x PH rows x ZC planes, or with TWO (two sweeps
// per step) 60 written columns, and an instance with two sweeps left in its
// cycle takes both in one pass
template <class V, int PH, int ZC, bool TWO>
__global__ __launch_bounds__(256) void k_bsweep3d(const BDesc *__restrict__ desc,
                                                  const BState *__restrict__ st,
                                                  const int2 *__restrict__ items, int nitems,
                                                  typename V::T *ua, typename V::T *ub,
                                                  const typename V::T *__restrict__ rhs, BParams prm)
{
    using A = typename V::A;
    const int nwaves = gridDim.x * 4;
    for (int item = blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); item < nitems; item += nwaves) {
        const int2 it = items[item];
        const BState s = st[it.x];
        if (s.done) continue;
        const BDesc &d = desc[it.x];
        const int tx = it.y % d.gx3, ty = (it.y / d.gx3) % d.gy3, tz = it.y / (d.gx3 * d.gy3);
        const A *w = Sel<A>::omega(prm) + prm.offsets[s.level] + s.pos;
        const typename V::T *uin = (s.pu ? ub : ua) + d.off;
        typename V::T *uout = (s.pu ? ua : ub) + d.off;
        if (TWO && sweeps_this_step(d, s, prm) == 2)
            plane3d2_run<V, PH, ZC>(Sel<A>::sten(d), uin, uout, rhs + d.off, w[0], w[1], tx, ty, tz,
                                    threadIdx.x & 63);
        else
            plane3d_run<V, PH, ZC, false, false, TWO ? 60 : 62>(Sel<A>::sten(d), uin, uout,
                                                                rhs + d.off, w[0], tx, ty, tz,
                                                                threadIdx.x & 63);
    }
}

__device__ __forceinline__ double block_sum256(double v, double *lds)
{
    v = wave_sum64(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();  // lds may still be read from the previous call
    if (lane == 0) lds[wave] = v;
    __syncthreads();
    return ((lds[0] + lds[1]) + lds[2]) + lds[3];
}

enum { OUT_STEP = 0, OUT_NORM = 1, OUT_CAST = 2 };

// The points of one outer-pass item: thread t takes points base + t + 256 k,
// k = 0..7.  Every load is unconditional: a neighbour outside the grid, and
// a point beyond the instance, read a valid point (the centre, the last
// point) and a select then drops the value, so that the term subtracted is
// c * 0 = 0 and leaves the sum's bits unchanged; the loads of four points
// are then in flight together (with a branch around each neighbour's load
// the compiler waited for every load in turn; unrolled by 8 the registers
// held occupancy at 2 waves per SIMD, no faster).  The sum of
// squares accumulates in k order.  Returns this thread's sum of squares of
// the binary64 residual.
template <class St, bool REFINE, int MODE>
__device__ __forceinline__ double outer_points(const BDesc d, const double *__restrict__ x,
                                               const typename St::T *__restrict__ dl,
                                               double *__restrict__ xn,
                                               typename St::T *__restrict__ dz,
                                               typename St::T *__restrict__ rh,
                                               const double *__restrict__ bb, double inv_s,
                                               double s_next, int64_t base)
{
    const int64_t s1 = d.n0, s2 = d.n0 * d.n1;
    // instances below 2^31 points (every one of the batched workloads) split
    // the point index with two 32-bit divisions instead of three 64-bit ones
    const bool idx32 = d.npts < ((int64_t)1 << 31);
    auto xv = [&](int64_t pp) -> double {
        if (REFINE && MODE == OUT_STEP)
            return x[pp] + static_cast<double>(St::load(dl[pp])) * inv_s;
        return x[pp];
    };
    double acc = 0.0;
#pragma unroll 4
    for (int k = 0; k < kOuterPts / 256; ++k) {
        const int64_t qr = base + k * 256 + threadIdx.x;
        const bool valid = qr < d.npts;
        const int64_t q = valid ? qr : d.npts - 1;
        int64_t i0, i1, i2;
        if (idx32) {
            const uint32_t qq = (uint32_t)q, m0 = (uint32_t)d.n0, m1 = (uint32_t)d.n1;
            const uint32_t a0 = qq / m0, a1 = a0 / m1;
            i0 = qq - a0 * m0;
            i1 = a0 - a1 * m1;
            i2 = a1;
        } else {
            i0 = q % d.n0;
            i1 = (q / d.n0) % d.n1;
            i2 = q / s2;
        }
        const bool h0 = i0 > 0, h1 = i0 < d.n0 - 1;
        const bool h2 = d.ndim >= 2 && i1 > 0, h3 = d.ndim >= 2 && i1 < d.n1 - 1;
        const bool h4 = d.ndim >= 3 && i2 > 0, h5 = d.ndim >= 3 && i2 < d.n2 - 1;
        const double xc = xv(q);
        const double v0 = xv(h0 ? q - 1 : q), v1 = xv(h1 ? q + 1 : q);
        const double v2 = xv(h2 ? q - s1 : q), v3 = xv(h3 ? q + s1 : q);
        const double v4 = xv(h4 ? q - s2 : q), v5 = xv(h5 ? q + s2 : q);
        const double bq = bb[q];
        double sacc = d.D * xc;
        sacc = sacc - d.c[0] * (h0 ? v0 : 0.0);
        sacc = sacc - d.c[0] * (h1 ? v1 : 0.0);
        if (d.ndim >= 2) {
            sacc = sacc - d.c[1] * (h2 ? v2 : 0.0);
            sacc = sacc - d.c[1] * (h3 ? v3 : 0.0);
        }
        if (d.ndim >= 3) {
            sacc = sacc - d.c[2] * (h4 ? v4 : 0.0);
            sacc = sacc - d.c[2] * (h5 ? v5 : 0.0);
        }
        const double r = bq - sacc;
        if (valid) {
            acc += r * r;
            if (REFINE && MODE != OUT_NORM) {
                if (MODE == OUT_STEP) xn[q] = xc;
                rh[q] = St::store(static_cast<float>(s_next * r));
                dz[q] = St::store(0.0f);
            }
        }
    }
    return acc;
}

// 2. outer pass: one block of 256 threads per (instance, 2048 points) item.
// REFINE: u = correction d (storage St), x ping-pong in binary64.
// !REFINE: u is x itself (binary64).
template <class St, bool REFINE>
__global__ __launch_bounds__(256) void k_bouter(const BDesc *__restrict__ desc,
                                                const BState *__restrict__ st,
                                                const int2 *__restrict__ items, int nitems,
                                                const double *__restrict__ b, double *xa, double *xb,
                                                void *uav, void *ubv, typename St::T *rhat,
                                                double *__restrict__ partials, BParams prm, int mode)
{
    typename St::T *ua = static_cast<typename St::T *>(uav);
    typename St::T *ub = static_cast<typename St::T *>(ubv);
    __shared__ double lds[4];
    __shared__ int nact;
    __shared__ int act[256];
    // The block owns items blockIdx.x + j gridDim.x.  Most of them have
    // nothing to do in a given step (their instance is not at a cycle end):
    // each thread tests one of the next 256 at once, so the state loads
    // overlap, and the block then works through the active ones.  Every item
    // writes only its own partial sum, so the order does not matter.
    for (int first = blockIdx.x; first < nitems; first += gridDim.x * 256) {
        if (threadIdx.x == 0) nact = 0;
        __syncthreads();
        const int mine = first + threadIdx.x * gridDim.x;
        if (mine < nitems) {
            const int2 it = items[mine];
            const BState s = st[it.x];
            bool on = !s.done;
            if (on && mode == OUT_STEP)
                on = s.pos + sweeps_this_step(desc[it.x], s, prm) == prm.levelM[s.level];
            if (on) act[atomicAdd(&nact, 1)] = mine;
        }
        __syncthreads();
        const int n = nact;
        for (int a = 0; a < n; ++a) {
            const int item = act[a];
            const int2 it = items[item];
            const BState s = st[it.x];
            const BDesc d = desc[it.x];
            // which buffers hold the current iterate
            const double *x;
            const typename St::T *dl = nullptr;  // latest correction (REFINE, step)
            typename St::T *dz = nullptr;        // correction buffer to clear
            double *xn = nullptr;                // updated x (REFINE, step)
            double inv_s = 0.0, s_next = 0.0;
            if (REFINE) {
                x = (s.px ? xb : xa) + d.off;
                if (mode == OUT_STEP) {
                    dl = (s.pu ? ua : ub) + d.off;  // the sweep just wrote u[pu ^ 1]
                    dz = (s.pu ? ub : ua) + d.off;  // stale: becomes the next cycle's zero start
                    xn = (s.px ? xa : xb) + d.off;
                    inv_s = 1.0 / s.s;
                    s_next = pow2_scale_dev(s.prev, d.sqrtN, prm.tgt_rms);
                } else if (mode == OUT_CAST) {
                    dz = (s.pu ? ub : ua) + d.off;  // u[pu] starts the first cycle at zero
                    s_next = s.s;
                }
            } else {
                const double *u64 = static_cast<const double *>(uav);
                const double *v64 = static_cast<const double *>(ubv);
                // step: the sweep just wrote u[pu ^ 1]; norm: u[pu] is current
                const int cur = mode == OUT_STEP ? (s.pu ^ 1) : s.pu;
                x = (cur ? v64 : u64) + d.off;
            }
            const int64_t base = (int64_t)(it.y - d.oitem_first) * kOuterPts;
            double acc;
            if (REFINE && mode == OUT_STEP)
                acc = outer_points<St, REFINE, OUT_STEP>(d, x, dl, xn, dz, rhat + d.off, b + d.off,
                                                         inv_s, s_next, base);
            else if (REFINE && mode == OUT_CAST)
                acc = outer_points<St, REFINE, OUT_CAST>(d, x, dl, xn, dz, rhat + d.off, b + d.off,
                                                         inv_s, s_next, base);
            else
                acc = outer_points<St, REFINE, OUT_NORM>(d, x, dl, xn, dz, rhat + d.off, b + d.off,
                                                         inv_s, s_next, base);
            const double t = block_sum256(acc, lds);
            if (threadIdx.x == 0) partials[item] = t;
        }
        __syncthreads();  // act and nact are reused by the next group
    }
}

__device__ int next_level_dev(int rule, int level, double ratio, int max_level)
{
    int nl = level;
    if (rule == SRJ_RULE_HEURISTIC) {
        if (ratio > 0.4)
            nl = level + 1;
        else if (ratio < 0.4 && ratio > 0.2)
            nl = level - 1;
    } else if (rule == SRJ_RULE_INCREASING) {
        nl = level + 1;
    }
    return nl < 0 ? 0 : (nl > max_level ? max_level : nl);
}

enum { FIN_STEP = 0, FIN_INIT = 1 };

// 3. finalize: one block per instance.
template <bool REFINE>
__global__ __launch_bounds__(256) void k_bfinal(const BDesc *__restrict__ desc, BState *st,
                                                const double *__restrict__ partials,
                                                int32_t *__restrict__ levels_hist,
                                                double *__restrict__ norms_hist, BParams prm,
                                                int mode)
{
    __shared__ double lds[4];
    const int i = blockIdx.x;
    const BState s = st[i];
    if (s.done) return;
    const BDesc &d = desc[i];
    int T = 0;
    if (mode == FIN_STEP) {
        T = sweeps_this_step(d, s, prm);
        const bool end = s.pos + T == prm.levelM[s.level];
        if (!end) {
            if (threadIdx.x == 0) {
                st[i].pos = s.pos + T;
                st[i].pu = s.pu ^ 1;
                st[i].sweeps = s.sweeps + T;
            }
            return;
        }
    }
    double v = 0.0;
    for (int k = threadIdx.x; k < d.oitem_count; k += 256) v += partials[d.oitem_first + k];
    const double sum = block_sum256(v, lds);
    if (threadIdx.x != 0) return;
    const double norm = sqrt(sum);
    BState n = s;
    const int hist = prm.max_cycles + 1;
    if (mode == FIN_INIT) {
        n.r0 = prm.r0_given > 0.0 ? prm.r0_given : norm;
        n.prev = norm;
        n.last = norm;
        n.target = prm.tol_mode == SRJ_TOL_RELATIVE ? prm.tol * n.r0 : prm.tol;
        n.s = pow2_scale_dev(norm, d.sqrtN, prm.tgt_rms);
        norms_hist[(int64_t)i * hist] = norm;
        if (!isfinite(norm)) {
            n.done = 1;
            n.status = SRJ_ERR_NONFINITE;
        } else if (norm == 0.0 || norm < n.target) {
            n.done = 1;
            n.status = SRJ_OK;
        }
        st[i] = n;
        return;
    }
    // end of a cycle
    const int lv = s.level;
    n.sweeps = s.sweeps + T;
    n.cycles = s.cycles + 1;
    n.last = norm;
    levels_hist[(int64_t)i * prm.max_cycles + s.cycles] = lv;
    norms_hist[(int64_t)i * hist + n.cycles] = norm;
    if (REFINE) {
        n.px = s.px ^ 1;  // x' was written to the other buffer
        n.s = pow2_scale_dev(s.prev, d.sqrtN, prm.tgt_rms);
        // u[pu] was cleared: the next cycle starts from zero there
    } else {
        n.pu = s.pu ^ 1;
    }
    n.pos = 0;
    if (!isfinite(norm)) {
        n.done = 1;
        n.status = SRJ_ERR_NONFINITE;
    } else if (norm < s.target) {
        n.done = 1;
        n.status = SRJ_OK;
    } else {
        const double ratio = norm / s.prev;
        n.prev = norm;
        if (prm.rule == SRJ_RULE_HEURISTIC) {
            const double m = fmin(fabs(ratio - 0.2), fabs(ratio - 0.4));
            n.min_margin = fmin(s.min_margin, m);
        }
        n.level = prm.rule == SRJ_RULE_FIXED ? prm.fixed_level
                                             : next_level_dev(prm.rule, lv, ratio, prm.max_level);
        if (n.cycles >= prm.max_cycles || n.sweeps + prm.levelM[n.level] > prm.max_sweeps) {
            n.done = 1;
            n.status = SRJ_ERR_NOT_CONVERGED;
        }
    }
    st[i] = n;
}

__global__ void k_fill_f64(double *__restrict__ a, int64_t n, double v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = v;
}

__global__ __launch_bounds__(256) void k_count_done(const BState *__restrict__ st, int n,
                                                    int32_t *__restrict__ out)
{
    __shared__ double lds[4];
    double v = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) v += st[i].done ? 1.0 : 0.0;
    const double t = block_sum256(v, lds);
    if (threadIdx.x == 0) *out = static_cast<int32_t>(t);
}

}  // namespace
}  // namespace srj

using namespace srj;

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
struct srj_batch {
    hipStream_t user_stream = nullptr;  // the caller's stream
    hipStream_t stream = nullptr;       // the batch's own stream (graphs are captured on it)
    int cus = 256;
    int count = 0;
    std::vector<BDesc> hdesc;
    BDesc *desc = nullptr;
    BState *state = nullptr;
    std::vector<const double *> b_user;
    int64_t total = 0;
    double *b = nullptr;                 // packed right-hand sides
    double *xa = nullptr, *xb = nullptr; // packed binary64 iterates
    void *ua = nullptr, *ub = nullptr, *rhat = nullptr;  // packed corrections (storage)
    int ubytes = 0;
    std::vector<int2> hitems2, hitems3, hoitems;
    int2 *items2 = nullptr, *items3 = nullptr, *oitems = nullptr;
    double *partials = nullptr;
    int32_t *levelM = nullptr, *offsets = nullptr;
    double *omega64 = nullptr;
    float *omega32 = nullptr;
    int32_t *levels_hist = nullptr;
    double *norms_hist = nullptr;
    int64_t hist_cap = 0;
    // instances finished, counted on the device into pinned host memory
    // (done_dev: the device mapping of done_host)
    int32_t *done_dev = nullptr, *done_host = nullptr;
    // plan
    int tile_rows = 24, halo = 4, T2 = 4, waves = 1, steps_per_graph = 16;
    bool use_graph = true;
    int ph3 = 4, zc3 = 8;  // 3D plane tile: rows, planes per work item
    int t3 = 2;            // most sweeps per step of a 3D instance (1 or 2)
    int device = 0;        // current device at setup; caller arrays must live there
};

namespace {

void batch_free(srj_batch *B)
{
    if (!B) return;
    if (B->stream) (void)hipStreamSynchronize(B->stream);
    else (void)hipDeviceSynchronize();
    for (void *p : {(void *)B->desc, (void *)B->state, (void *)B->b, (void *)B->xa, (void *)B->xb,
                    B->ua, B->ub, B->rhat, (void *)B->items2, (void *)B->items3, (void *)B->oitems,
                    (void *)B->partials, (void *)B->levelM, (void *)B->offsets, (void *)B->omega64,
                    (void *)B->omega32, (void *)B->levels_hist, (void *)B->norms_hist})
        (void)hipFree(p);
    (void)hipHostFree(B->done_host);  // done_dev is its device mapping
    if (B->stream) (void)hipStreamDestroy(B->stream);
    delete B;
}

// tile shapes (rows, halo) of the batched 2D sweep kernel
#define SRJ_BATCH_2D(X) X(16, 2) X(24, 4) X(32, 4) X(32, 6) X(48, 8)

// cooperative block shapes (rows per wave, halo, waves per block)
#define SRJ_BATCH_BLOCK(X) X(8, 4, 8) X(8, 8, 8) X(12, 8, 8) X(16, 8, 4)

// the halo of a plan, 0 if there is no such plan
int batch_plan_halo(int rows, int T, int waves)
{
    if (T < 1) return 0;
    if (waves == 1) {
#define SRJ_OK_(R, HL) if (rows == R && T <= HL) return HL;
        SRJ_BATCH_2D(SRJ_OK_)
#undef SRJ_OK_
        return 0;
    }
#define SRJ_OK_(HW, HL, NW) if (rows == HW && waves == NW && T <= HL) return HL;
    SRJ_BATCH_BLOCK(SRJ_OK_)
#undef SRJ_OK_
    return 0;
}

template <class V>
hipError_t launch_bsweep2d(srj_batch *B, void *ua, void *ub, const void *rhs, const BParams &prm,
                           int grid)
{
    using T = typename V::T;
    if (B->waves > 1) {
        // a few resident workgroups per CU, a multiple of 8 (one set per XCD)
        const int64_t items = (int64_t)B->hitems2.size();
        const int g = (int)std::max<int64_t>(8, std::min<int64_t>((items + 7) / 8 * 8,
                                                                  (int64_t)B->cus * 3 / 8 * 8));
#define SRJ_GOB(HW, HL, NW)                                                                    \
        if (B->tile_rows == HW && B->halo == HL && B->waves == NW) {                           \
            hipLaunchKernelGGL((k_bsweep2d_blk<V, HW, HL, NW>), dim3(g), dim3(64 * NW), 0,     \
                               B->stream, B->desc, B->state, B->items2, (int)items, (T *)ua,   \
                               (T *)ub, (const T *)rhs, prm);                                  \
            return hipGetLastError();                                                          \
        }
        SRJ_BATCH_BLOCK(SRJ_GOB)
#undef SRJ_GOB
        return hipErrorInvalidValue;
    }
#define SRJ_GO(R, HL)                                                                         \
    if (B->tile_rows == R && B->halo == HL) {                                                 \
        hipLaunchKernelGGL((k_bsweep2d<V, R, HL>), dim3(grid), dim3(256), 0, B->stream, B->desc, \
                           B->state, B->items2, (int)B->hitems2.size(), (T *)ua, (T *)ub,        \
                           (const T *)rhs, prm);                                              \
        return hipGetLastError();                                                             \
    }
    SRJ_BATCH_2D(SRJ_GO)
#undef SRJ_GO
    return hipErrorInvalidValue;
}

int device_cus()
{
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 256;
    return cus > 0 ? cus : 256;
}

// One step: sweeps, outer pass, finalize.
template <class St, bool REFINE>
srj_status enqueue_step(srj_batch *B, const BParams &prm)
{
    using V = typename std::conditional<REFINE, St, StF64>::type;
    void *ua = REFINE ? B->ua : (void *)B->xa;
    void *ub = REFINE ? B->ub : (void *)B->xb;
    const void *rhs = REFINE ? B->rhat : (const void *)B->b;
    const int cus = B->cus;
    if (!B->hitems2.empty()) {
        const int grid = (int)std::min<int64_t>((B->hitems2.size() + 3) / 4, (int64_t)cus * 8);
        SRJ_HIP_CHECK(launch_bsweep2d<V>(B, ua, ub, rhs, prm, grid));
    }
    if (!B->hitems3.empty()) {
        const int grid = (int)std::min<int64_t>((B->hitems3.size() + 3) / 4, (int64_t)cus * 8);
        bool launched = false;
#define SRJ_GO3(PH, ZC)                                                                           \
        if (!launched && B->ph3 == PH && B->zc3 == ZC) {                                          \
            if (B->t3 == 2)                                                                        \
                hipLaunchKernelGGL((k_bsweep3d<V, PH, ZC, true>), dim3(grid), dim3(256), 0,       \
                                   B->stream, B->desc, B->state, B->items3,                        \
                                   (int)B->hitems3.size(), (typename V::T *)ua,                    \
                                   (typename V::T *)ub, (const typename V::T *)rhs, prm);          \
            else                                                                                   \
                hipLaunchKernelGGL((k_bsweep3d<V, PH, ZC, false>), dim3(grid), dim3(256), 0,      \
                                   B->stream, B->desc, B->state, B->items3,                        \
                                   (int)B->hitems3.size(), (typename V::T *)ua,                    \
                                   (typename V::T *)ub, (const typename V::T *)rhs, prm);          \
            launched = true;                                                                       \
        }
        SRJ_BATCH_PLANE(SRJ_GO3)
#undef SRJ_GO3
        if (!launched) return fail(SRJ_ERR_INVALID, "3D plane tile not available");
        SRJ_HIP_CHECK(hipGetLastError());
    }
    const int og = (int)std::min<int64_t>(B->hoitems.size(), (int64_t)cus * 8);
    hipLaunchKernelGGL((k_bouter<St, REFINE>), dim3(og), dim3(256), 0, B->stream, B->desc, B->state,
                       B->oitems, (int)B->hoitems.size(), B->b, B->xa, B->xb, ua, ub,
                       (typename St::T *)B->rhat, B->partials, prm, (int)OUT_STEP);
    SRJ_HIP_CHECK(hipGetLastError());
    hipLaunchKernelGGL((k_bfinal<REFINE>), dim3(B->count), dim3(256), 0, B->stream, B->desc, B->state,
                       B->partials, B->levels_hist, B->norms_hist, prm, (int)FIN_STEP);
    SRJ_HIP_CHECK(hipGetLastError());
    return SRJ_OK;
}

BParams make_params(const srj_batch *B, const srj_solve_opts *o)
{
    BParams prm{};
    prm.rule = o->rule;
    prm.fixed_level = o->fixed_level;
    prm.max_level = o->max_level;
    prm.max_cycles = o->max_cycles;
    prm.max_sweeps = o->max_sweeps;
    prm.tol_mode = o->tol_mode;
    prm.T2 = B->T2;
    prm.T3 = B->t3;
    prm.tol = o->tol;
    prm.tgt_rms = o->scale_target > 0.0 ? o->scale_target
                  : (o->precision == SRJ_PREC_F16_REFINE ? ldexp(1.0, -8) : 1.0);
    prm.r0_given = o->r0;
    prm.levelM = B->levelM;
    prm.offsets = B->offsets;
    prm.omega64 = B->omega64;
    prm.omega32 = B->omega32;
    return prm;
}

template <class St, bool REFINE>
srj_status ensure_batch_buffers(srj_batch *B, int max_cycles)
{
    const int n = B->count;
    if (REFINE && B->ubytes < St::bytes) {
        (void)hipFree(B->ua);
        (void)hipFree(B->ub);
        (void)hipFree(B->rhat);
        B->ua = B->ub = B->rhat = nullptr;
        B->ubytes = 0;
        if (hipMalloc(&B->ua, (size_t)B->total * St::bytes) != hipSuccess ||
            hipMalloc(&B->ub, (size_t)B->total * St::bytes) != hipSuccess ||
            hipMalloc(&B->rhat, (size_t)B->total * St::bytes) != hipSuccess)
            return fail(SRJ_ERR_NOMEM, "hipMalloc failed for batched corrections");
        B->ubytes = St::bytes;
    }
    const int64_t hist = (int64_t)max_cycles + 1;
    if (B->hist_cap < hist) {
        (void)hipFree(B->levels_hist);
        (void)hipFree(B->norms_hist);
        B->levels_hist = nullptr;
        B->norms_hist = nullptr;
        B->hist_cap = 0;
        if (hipMalloc(&B->levels_hist, sizeof(int32_t) * (size_t)n * max_cycles) != hipSuccess ||
            hipMalloc(&B->norms_hist, sizeof(double) * (size_t)n * hist) != hipSuccess)
            return fail(SRJ_ERR_NOMEM, "hipMalloc failed for batch histories");
        B->hist_cap = hist;
    }
    return SRJ_OK;
}

// Fresh per-instance state and the initial passes (norms; for refinement the
// scaled cast of r0 and zeroed corrections).  x0 must already be in xa.
template <class St, bool REFINE>
srj_status batch_init(srj_batch *B, const srj_solve_opts *o, const BParams &prm)
{
    const int n = B->count;
    std::vector<BState> hs(n);
    for (int i = 0; i < n; ++i) {
        BState &s = hs[i];
        memset(&s, 0, sizeof(s));
        s.level = o->rule == SRJ_RULE_FIXED ? o->fixed_level : o->start_level;
        s.min_margin = INFINITY;
        s.status = SRJ_ERR_NOT_CONVERGED;
    }
    SRJ_HIP_CHECK(hipMemcpyAsync(B->state, hs.data(), sizeof(BState) * n, hipMemcpyHostToDevice,
                                 B->stream));
    const int og = (int)std::min<int64_t>(B->hoitems.size(), (int64_t)B->cus * 8);
    void *ua = REFINE ? B->ua : (void *)B->xa;
    void *ub = REFINE ? B->ub : (void *)B->xb;
    hipLaunchKernelGGL((k_bouter<St, REFINE>), dim3(og), dim3(256), 0, B->stream, B->desc, B->state,
                       B->oitems, (int)B->hoitems.size(), B->b, B->xa, B->xb, ua, ub,
                       (typename St::T *)B->rhat, B->partials, prm, (int)OUT_NORM);
    SRJ_HIP_CHECK(hipGetLastError());
    hipLaunchKernelGGL((k_bfinal<REFINE>), dim3(n), dim3(256), 0, B->stream, B->desc, B->state,
                       B->partials, B->levels_hist, B->norms_hist, prm, (int)FIN_INIT);
    SRJ_HIP_CHECK(hipGetLastError());
    if (REFINE) {
        hipLaunchKernelGGL((k_bouter<St, REFINE>), dim3(og), dim3(256), 0, B->stream, B->desc,
                           B->state, B->oitems, (int)B->hoitems.size(), B->b, B->xa, B->xb, ua, ub,
                           (typename St::T *)B->rhat, B->partials, prm, (int)OUT_CAST);
        SRJ_HIP_CHECK(hipGetLastError());
    }
    return SRJ_OK;
}

// Times `steps` steps from a fresh state with x0 = 0 (tuning).
template <class St, bool REFINE>
srj_status batch_time_steps(srj_batch *B, const srj_solve_opts *o, int steps, float *ms)
{
    srj_status st = ensure_batch_buffers<St, REFINE>(B, o->max_cycles);
    if (st != SRJ_OK) return st;
    const BParams prm = make_params(B, o);
    hipLaunchKernelGGL(k_fill_f64, dim3((unsigned)((B->total + 255) / 256)), dim3(256), 0,
                       B->stream, B->xa, B->total, 0.0);
    SRJ_HIP_CHECK(hipGetLastError());
    st = batch_init<St, REFINE>(B, o, prm);
    if (st != SRJ_OK) return st;
    hipEvent_t e0, e1;
    SRJ_HIP_CHECK(hipEventCreate(&e0));
    SRJ_HIP_CHECK(hipEventCreate(&e1));
    st = enqueue_step<St, REFINE>(B, prm);  // warm-up
    hipError_t e = hipEventRecord(e0, B->stream);
    for (int k = 0; k < steps && st == SRJ_OK && e == hipSuccess; ++k) st = enqueue_step<St, REFINE>(B, prm);
    if (e == hipSuccess) e = hipEventRecord(e1, B->stream);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != SRJ_OK) return st;
    SRJ_HIP_CHECK(e);
    return SRJ_OK;
}

template <class St, bool REFINE>
srj_status batch_solve_t(srj_batch *B, double *const *xs, const srj_solve_opts *o,
                         srj_solve_result *res, int32_t *levels_out)
{
    const int n = B->count;
    // the caller's x arrays are read on the batch stream: wait for their producers
    SRJ_HIP_CHECK(hipStreamSynchronize(B->user_stream));
    srj_status bst = ensure_batch_buffers<St, REFINE>(B, o->max_cycles);
    if (bst != SRJ_OK) return bst;
    // pack the initial iterates (binary64 into xa)
    for (int i = 0; i < n; ++i)
        SRJ_HIP_CHECK(hipMemcpyAsync(B->xa + B->hdesc[i].off, xs[i],
                                     sizeof(double) * (size_t)B->hdesc[i].npts,
                                     hipMemcpyDeviceToDevice, B->stream));
    const BParams prm = make_params(B, o);
    bst = batch_init<St, REFINE>(B, o, prm);
    if (bst != SRJ_OK) return bst;
    std::vector<BState> hs(n);

    // steps, replayed from a graph until every instance is done
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    const int K = std::max(1, B->steps_per_graph);
    if (B->use_graph) {
        SRJ_HIP_CHECK(hipStreamBeginCapture(B->stream, hipStreamCaptureModeThreadLocal));
        srj_status st = SRJ_OK;
        for (int k = 0; k < K && st == SRJ_OK; ++k) st = enqueue_step<St, REFINE>(B, prm);
        if (st == SRJ_OK) {
            hipLaunchKernelGGL(k_count_done, dim3(1), dim3(256), 0, B->stream, B->state, n,
                               B->done_dev);
        }
        hipError_t e = hipStreamEndCapture(B->stream, &graph);
        if (st != SRJ_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return st;
        }
        SRJ_HIP_CHECK(e);
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            (void)hipGraphDestroy(graph);
            return fail(SRJ_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
        }
    }
    // every step advances each live instance by at least one sweep; bound the replays
    int64_t max_sweeps_any = 0;
    for (int i = 0; i < n; ++i) max_sweeps_any = std::max<int64_t>(max_sweeps_any, o->max_sweeps);
    const int64_t max_steps =
        std::min<int64_t>(max_sweeps_any, (int64_t)o->max_cycles * SRJ_MAX_M) + (int64_t)o->max_cycles + 2;
    srj_status status = SRJ_OK;
    for (int64_t done_steps = 0;; done_steps += K) {
        if (B->use_graph) {
            hipError_t e = hipGraphLaunch(exec, B->stream);
            if (e != hipSuccess) {
                status = fail(SRJ_ERR_HIP, std::string("hipGraphLaunch: ") + hipGetErrorString(e));
                break;
            }
        } else {
            for (int k = 0; k < K; ++k) {
                status = enqueue_step<St, REFINE>(B, prm);
                if (status != SRJ_OK) break;
            }
            if (status != SRJ_OK) break;
            hipLaunchKernelGGL(k_count_done, dim3(1), dim3(256), 0, B->stream, B->state, n,
                               B->done_dev);
        }
        // k_count_done wrote the count straight into the pinned done_host
        hipError_t e = hipStreamSynchronize(B->stream);
        if (e != hipSuccess) {
            status = fail(SRJ_ERR_HIP, std::string("batch step: ") + hipGetErrorString(e));
            break;
        }
        if (*B->done_host >= n) break;
        if (done_steps > max_steps) {
            status = fail(SRJ_ERR_HIP, "batch did not finish within its step bound");
            break;
        }
    }
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (status != SRJ_OK) return status;

    // results
    SRJ_HIP_CHECK(hipMemcpyAsync(hs.data(), B->state, sizeof(BState) * n, hipMemcpyDeviceToHost,
                                 B->stream));
    SRJ_HIP_CHECK(hipStreamSynchronize(B->stream));
    for (int i = 0; i < n; ++i) {
        const BState &s = hs[i];
        const double *src;
        if (REFINE)
            src = (s.px ? B->xb : B->xa) + B->hdesc[i].off;
        else
            src = (s.pu ? B->xb : B->xa) + B->hdesc[i].off;
        SRJ_HIP_CHECK(hipMemcpyAsync(xs[i], src, sizeof(double) * (size_t)B->hdesc[i].npts,
                                     hipMemcpyDeviceToDevice, B->stream));
    }
    if (levels_out)
        SRJ_HIP_CHECK(hipMemcpyAsync(levels_out, B->levels_hist,
                                     sizeof(int32_t) * (size_t)n * o->max_cycles,
                                     hipMemcpyDeviceToHost, B->stream));
    SRJ_HIP_CHECK(hipStreamSynchronize(B->stream));
    srj_status first_bad = SRJ_OK;
    for (int i = 0; i < n; ++i) {
        const BState &s = hs[i];
        srj_solve_result &r = res[i];
        memset(&r, 0, sizeof(r));
        r.converged = s.status == SRJ_OK;
        r.cycles = s.cycles;
        r.final_level = s.cycles > 0 ? s.level : o->start_level;
        r.sweeps = s.sweeps;
        r.r0 = s.r0;
        r.r_final = s.last;
        r.min_margin = s.min_margin;
        if (s.status != SRJ_OK && first_bad == SRJ_OK) first_bad = (srj_status)s.status;
    }
    // the level of the last cycle run (state.level already holds the next choice)
    if (levels_out) {
        for (int i = 0; i < n; ++i)
            if (hs[i].cycles > 0)
                res[i].final_level = levels_out[(int64_t)i * o->max_cycles + hs[i].cycles - 1];
    } else {
        std::vector<int32_t> tmp((size_t)n * o->max_cycles);
        SRJ_HIP_CHECK(hipMemcpyAsync(tmp.data(), B->levels_hist, sizeof(int32_t) * tmp.size(),
                                     hipMemcpyDeviceToHost, B->stream));
        SRJ_HIP_CHECK(hipStreamSynchronize(B->stream));
        for (int i = 0; i < n; ++i)
            if (hs[i].cycles > 0) res[i].final_level = tmp[(size_t)i * o->max_cycles + hs[i].cycles - 1];
    }
    if (first_bad != SRJ_OK) set_error("at least one instance did not converge");
    return first_bad;
}

}  // namespace

extern "C" {

srj_status srj_batch_setup(int32_t count, const srj_problem *probs, void *hip_stream,
                           srj_batch **out)
{
    if (!out) return fail(SRJ_ERR_INVALID, "out is NULL");
    *out = nullptr;
    if (count < 1 || !probs) return fail(SRJ_ERR_INVALID, "count must be >= 1 and probs non-NULL");
    int64_t total = 0;
    for (int i = 0; i < count; ++i) {
        const srj_problem &p = probs[i];
        if (p.ndim < 1 || p.ndim > 3) return fail(SRJ_ERR_INVALID, "ndim must be 1, 2 or 3");
        for (int d = 0; d < 3; ++d) {
            if (p.n[d] < 1) return fail(SRJ_ERR_INVALID, "every n[d] must be >= 1");
            if (d >= p.ndim && p.n[d] != 1) return fail(SRJ_ERR_INVALID, "n[d] must be 1 for d >= ndim");
            if (d < p.ndim && p.face[d])
                return fail(SRJ_ERR_UNSUPPORTED, "batched solves take constant couplings only");
            if (d < p.ndim && !(p.cconst[d] >= 0.0 && isfinite(p.cconst[d])))
                return fail(SRJ_ERR_INVALID, "cconst[d] must be finite and >= 0");
        }
        if (!points_fit(p.n)) return fail(SRJ_ERR_INVALID, "n[0] n[1] n[2] must be <= 2^38");
        total += p.n[0] * p.n[1] * p.n[2];
        if (total > kMaxPoints) return fail(SRJ_ERR_INVALID, "the instances hold more than 2^38 points");
        if (p.diag) return fail(SRJ_ERR_UNSUPPORTED, "batched solves take a constant diagonal only");
        if (!(p.dconst > 0.0) || !isfinite(p.dconst)) return fail(SRJ_ERR_INVALID, "dconst must be > 0");
        if (!p.b) return fail(SRJ_ERR_INVALID, "b is NULL");
    }
    int dev = 0;
    SRJ_HIP_CHECK(hipGetDevice(&dev));
    for (int i = 0; i < count; ++i) {
        const srj_problem &p = probs[i];
        const size_t nb = sizeof(double) * (size_t)(p.n[0] * p.n[1] * p.n[2]);
        srj_status chk = check_device_array(p.b, nb, dev, "b");
        if (chk != SRJ_OK) return chk;
    }
    srj_batch *B = new srj_batch();
    B->device = dev;
    B->user_stream = static_cast<hipStream_t>(hip_stream);
    B->cus = device_cus();
    if (hipStreamCreateWithFlags(&B->stream, hipStreamNonBlocking) != hipSuccess) {
        delete B;
        return fail(SRJ_ERR_HIP, "hipStreamCreateWithFlags failed");
    }
    // the caller's b arrays are read on the batch stream: wait for their producers
    if (hipStreamSynchronize(B->user_stream) != hipSuccess) {
        batch_free(B);
        return fail(SRJ_ERR_HIP, "synchronising the caller's stream failed");
    }
    B->count = count;
    B->hdesc.resize(count);
    B->b_user.resize(count);
    int64_t off = 0;
    for (int i = 0; i < count; ++i) {
        const srj_problem &p = probs[i];
        BDesc &d = B->hdesc[i];
        memset(&d, 0, sizeof(d));
        d.ndim = p.ndim;
        d.n0 = p.n[0];
        d.n1 = p.n[1];
        d.n2 = p.n[2];
        d.npts = d.n0 * d.n1 * d.n2;
        d.off = off;
        for (int k = 0; k < 3; ++k) {
            d.c[k] = k < p.ndim ? p.cconst[k] : 0.0;
            d.c32[k] = static_cast<float>(d.c[k]);
        }
        d.D = p.dconst;
        d.Dinv = 1.0 / p.dconst;
        d.D32 = static_cast<float>(p.dconst);
        d.Dinv32 = static_cast<float>(1.0 / p.dconst);
        d.sqrtN = sqrt(static_cast<double>(d.npts));
        B->b_user[i] = p.b;
        off += d.npts;
    }
    B->total = off;
    auto nomem = [&](const char *what) {
        batch_free(B);
        return fail(SRJ_ERR_NOMEM, std::string("hipMalloc failed for ") + what);
    };
    const size_t bytes = sizeof(double) * (size_t)B->total;
    if (hipMalloc(&B->b, bytes) != hipSuccess) return nomem("packed b");
    if (hipMalloc(&B->xa, bytes) != hipSuccess || hipMalloc(&B->xb, bytes) != hipSuccess)
        return nomem("packed x");
    for (int i = 0; i < count; ++i) {
        hipError_t e = hipMemcpyAsync(B->b + B->hdesc[i].off, B->b_user[i],
                                      sizeof(double) * (size_t)B->hdesc[i].npts,
                                      hipMemcpyDeviceToDevice, B->stream);
        if (e != hipSuccess) {
            batch_free(B);
            return fail(SRJ_ERR_HIP, std::string("packing b: ") + hipGetErrorString(e));
        }
    }
    // scheme tables
    std::vector<double> table;
    std::vector<int32_t> offsets;
    full_table(table, offsets);
    std::vector<float> table32(table.size());
    for (size_t k = 0; k < table.size(); ++k) table32[k] = static_cast<float>(table[k]);
    std::vector<int32_t> lm(SRJ_NUM_LEVELS);
    for (int l = 0; l < SRJ_NUM_LEVELS; ++l) lm[l] = level_m(l);
    if (hipMalloc(&B->omega64, sizeof(double) * table.size()) != hipSuccess ||
        hipMalloc(&B->omega32, sizeof(float) * table.size()) != hipSuccess ||
        hipMalloc(&B->offsets, sizeof(int32_t) * offsets.size()) != hipSuccess ||
        hipMalloc(&B->levelM, sizeof(int32_t) * lm.size()) != hipSuccess)
        return nomem("scheme tables");
    hipError_t e = hipMemcpyAsync(B->omega64, table.data(), sizeof(double) * table.size(),
                                  hipMemcpyHostToDevice, B->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(B->omega32, table32.data(), sizeof(float) * table32.size(),
                           hipMemcpyHostToDevice, B->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(B->offsets, offsets.data(), sizeof(int32_t) * offsets.size(),
                           hipMemcpyHostToDevice, B->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(B->levelM, lm.data(), sizeof(int32_t) * lm.size(), hipMemcpyHostToDevice,
                           B->stream);
    if (hipMalloc(&B->state, sizeof(BState) * count) != hipSuccess ||
        hipMalloc(&B->desc, sizeof(BDesc) * count) != hipSuccess ||
        hipHostMalloc(&B->done_host, sizeof(int32_t), 0) != hipSuccess ||
        hipHostGetDevicePointer((void **)&B->done_dev, B->done_host, 0) != hipSuccess)
        return nomem("batch state");
    if (e == hipSuccess) e = hipStreamSynchronize(B->stream);
    if (e != hipSuccess) {
        batch_free(B);
        return fail(SRJ_ERR_HIP, std::string("batch setup: ") + hipGetErrorString(e));
    }
    srj_status st = srj_batch_set_plan(B, B->tile_rows, B->T2, B->waves, B->steps_per_graph, 1);
    if (st != SRJ_OK) {
        batch_free(B);
        return st;
    }
    *out = B;
    return SRJ_OK;
}

srj_status srj_batch_set_plan(srj_batch *B, int32_t tile_rows, int32_t sweeps_per_launch,
                              int32_t waves_per_block, int32_t steps_per_graph, int32_t use_graph)
{
    if (!B) return fail(SRJ_ERR_INVALID, "batch is NULL");
    const int halo = batch_plan_halo(tile_rows, sweeps_per_launch, waves_per_block);
    if (halo == 0)
        return fail(SRJ_ERR_UNSUPPORTED, "tile rows / sweeps per launch / waves not available");
    if (steps_per_graph < 1 || steps_per_graph > 1024)
        return fail(SRJ_ERR_INVALID, "steps_per_graph must be 1..1024");
    B->tile_rows = tile_rows;
    B->T2 = sweeps_per_launch;
    B->waves = waves_per_block;
    B->steps_per_graph = steps_per_graph;
    B->use_graph = use_graph != 0;
    B->halo = halo;
    // output columns and rows per work item (a single-wave tile or a block)
    const int OW = 64 - 2 * halo, OH = tile_rows * waves_per_block - 2 * halo;
    // work items
    B->hitems2.clear();
    B->hitems3.clear();
    B->hoitems.clear();
    for (int i = 0; i < B->count; ++i) {
        BDesc &d = B->hdesc[i];
        if (d.ndim == 3) {
            const int W = B->t3 == 2 ? 60 : 62;  // written columns per plane tile
            d.gx3 = (int)((d.n0 + W - 1) / W);
            d.gy3 = (int)((d.n1 + B->ph3 - 1) / B->ph3);
            const int gz = (int)((d.n2 + B->zc3 - 1) / B->zc3);
            for (int k = 0; k < d.gx3 * d.gy3 * gz; ++k) B->hitems3.push_back({i, k});
        } else {
            d.tiles_x = (int)((d.n0 + OW - 1) / OW);
            const int ty = (int)((d.n1 + OH - 1) / OH);
            for (int k = 0; k < d.tiles_x * ty; ++k) B->hitems2.push_back({i, k});
        }
        d.oitem_first = (int)B->hoitems.size();
        d.oitem_count = (int)((d.npts + kOuterPts - 1) / kOuterPts);
        for (int k = 0; k < d.oitem_count; ++k) B->hoitems.push_back({i, d.oitem_first + k});
    }
    (void)hipFree(B->items2);
    (void)hipFree(B->items3);
    (void)hipFree(B->oitems);
    (void)hipFree(B->partials);
    B->items2 = B->items3 = B->oitems = nullptr;
    B->partials = nullptr;
    auto up = [&](int2 **dst, const std::vector<int2> &src) -> bool {
        if (src.empty()) return true;
        if (hipMalloc(dst, sizeof(int2) * src.size()) != hipSuccess) return false;
        return hipMemcpyAsync(*dst, src.data(), sizeof(int2) * src.size(), hipMemcpyHostToDevice,
                              B->stream) == hipSuccess;
    };
    if (!up(&B->items2, B->hitems2) || !up(&B->items3, B->hitems3) || !up(&B->oitems, B->hoitems))
        return fail(SRJ_ERR_NOMEM, "work item lists");
    if (hipMalloc(&B->partials, sizeof(double) * B->hoitems.size()) != hipSuccess)
        return fail(SRJ_ERR_NOMEM, "batch partials");
    SRJ_HIP_CHECK(hipMemcpyAsync(B->desc, B->hdesc.data(), sizeof(BDesc) * B->count,
                                 hipMemcpyHostToDevice, B->stream));
    SRJ_HIP_CHECK(hipStreamSynchronize(B->stream));
    return SRJ_OK;
}

srj_status srj_batch_solve(srj_batch *B, double *const *xs, const srj_solve_opts *o,
                           srj_solve_result *res, int32_t *levels_out)
{
    if (!B || !xs || !res || !o) return fail(SRJ_ERR_INVALID, "NULL argument");
    for (int i = 0; i < B->count; ++i) {
        if (!xs[i]) return fail(SRJ_ERR_INVALID, "xs[i] is NULL");
        srj_status chk = check_device_array(xs[i], sizeof(double) * (size_t)B->hdesc[i].npts,
                                            B->device, "xs[i]");
        if (chk != SRJ_OK) return chk;
    }
    srj_solve_opts chk = *o;
    if (!(chk.tol > 0.0)) return fail(SRJ_ERR_INVALID, "tol must be > 0");
    if (chk.max_cycles < 1 || chk.max_sweeps < 1) return fail(SRJ_ERR_INVALID, "caps must be >= 1");
    if (chk.max_level < 0 || chk.max_level >= SRJ_NUM_LEVELS) return fail(SRJ_ERR_INVALID, "max_level outside 0..24");
    if (chk.start_level < 0 || chk.start_level > chk.max_level) return fail(SRJ_ERR_INVALID, "start_level outside 0..max_level");
    if (chk.rule < SRJ_RULE_HEURISTIC || chk.rule > SRJ_RULE_FIXED) return fail(SRJ_ERR_INVALID, "unknown rule");
    if (chk.rule == SRJ_RULE_FIXED && (chk.fixed_level < 0 || chk.fixed_level >= SRJ_NUM_LEVELS))
        return fail(SRJ_ERR_INVALID, "fixed_level outside 0..24");
    if (chk.tol_mode != SRJ_TOL_RELATIVE && chk.tol_mode != SRJ_TOL_ABSOLUTE)
        return fail(SRJ_ERR_INVALID, "unknown tol_mode");
    switch (o->precision) {
    case SRJ_PREC_F64: return batch_solve_t<StF32, false>(B, xs, o, res, levels_out);
    case SRJ_PREC_F32_REFINE: return batch_solve_t<StF32, true>(B, xs, o, res, levels_out);
    case SRJ_PREC_F16_REFINE: return batch_solve_t<StF16, true>(B, xs, o, res, levels_out);
    case SRJ_PREC_BF16_REFINE: return batch_solve_t<StBF16, true>(B, xs, o, res, levels_out);
    default: return fail(SRJ_ERR_INVALID, "unknown precision");
    }
}

srj_status srj_batch_get_plan(srj_batch *B, int32_t *tile_rows, int32_t *sweeps_per_launch,
                              int32_t *waves_per_block, int32_t *steps_per_graph,
                              int32_t *use_graph)
{
    if (!B || !tile_rows || !sweeps_per_launch || !waves_per_block || !steps_per_graph || !use_graph)
        return fail(SRJ_ERR_INVALID, "NULL argument");
    *tile_rows = B->tile_rows;
    *sweeps_per_launch = B->T2;
    *waves_per_block = B->waves;
    *steps_per_graph = B->steps_per_graph;
    *use_graph = B->use_graph ? 1 : 0;
    return SRJ_OK;
}

srj_status srj_batch_set_plan3d(srj_batch *B, int32_t tile_rows, int32_t planes, int32_t sweeps)
{
    if (!B) return fail(SRJ_ERR_INVALID, "batch is NULL");
    if (sweeps != 1 && sweeps != 2) return fail(SRJ_ERR_INVALID, "sweeps must be 1 or 2");
    bool ok = false;
#define SRJ_OK3(PH, ZC) ok = ok || (tile_rows == PH && planes == ZC);
    SRJ_BATCH_PLANE(SRJ_OK3)
#undef SRJ_OK3
    if (!ok) return fail(SRJ_ERR_UNSUPPORTED, "3D plane tile not available");
    B->ph3 = tile_rows;
    B->zc3 = planes;
    B->t3 = sweeps;
    // rebuild the work items with the current 2D plan
    return srj_batch_set_plan(B, B->tile_rows, B->T2, B->waves, B->steps_per_graph,
                              B->use_graph ? 1 : 0);
}

srj_status srj_batch_get_plan3d(srj_batch *B, int32_t *tile_rows, int32_t *planes,
                                int32_t *sweeps)
{
    if (!B || !tile_rows || !planes || !sweeps) return fail(SRJ_ERR_INVALID, "NULL argument");
    *tile_rows = B->ph3;
    *planes = B->zc3;
    *sweeps = B->t3;
    return SRJ_OK;
}

srj_status srj_batch_autotune(srj_batch *B, int32_t precision, int32_t sweeps,
                              double *best_us_per_sweep)
{
    if (!B || !best_us_per_sweep) return fail(SRJ_ERR_INVALID, "NULL argument");
    if (sweeps < 1 || sweeps > 100000) return fail(SRJ_ERR_INVALID, "sweeps must be 1..100000");
    if (precision < SRJ_PREC_F64 || precision > SRJ_PREC_BF16_REFINE)
        return fail(SRJ_ERR_INVALID, "unknown precision");
    SRJ_HIP_CHECK(hipStreamSynchronize(B->user_stream));
    srj_solve_opts o;
    srj_default_opts(&o);
    o.precision = (srj_precision)precision;
    o.tol = 1e-300;  // nothing converges while timing
    o.max_cycles = 1000000;
    o.max_sweeps = (int64_t)1 << 60;
    const int steps_per_graph = B->steps_per_graph;
    const bool use_graph = B->use_graph;
    auto time_steps = [&](int steps, float *ms) -> srj_status {
        switch (o.precision) {
        case SRJ_PREC_F64: return batch_time_steps<StF32, false>(B, &o, steps, ms);
        case SRJ_PREC_F32_REFINE: return batch_time_steps<StF32, true>(B, &o, steps, ms);
        case SRJ_PREC_F16_REFINE: return batch_time_steps<StF16, true>(B, &o, steps, ms);
        default: return batch_time_steps<StBF16, true>(B, &o, steps, ms);
        }
    };
    double best = INFINITY;
    // 2D/1D instances: tile or block plan, timed per sweep
    if (!B->hitems2.empty()) {
        int best_rows = B->tile_rows, best_T = B->T2, best_waves = B->waves;
        struct Cand {
            int rows, T, waves;
        };
        std::vector<Cand> cands;
#define SRJ_C(R, HL)                                        \
    cands.push_back({R, HL, 1});                            \
    if ((HL + 1) / 2 != HL) cands.push_back({R, (HL + 1) / 2, 1});
        SRJ_BATCH_2D(SRJ_C)
#undef SRJ_C
#define SRJ_CB(HW, HL, NW) cands.push_back({HW, HL, NW});
        SRJ_BATCH_BLOCK(SRJ_CB)
#undef SRJ_CB
        for (const Cand &cd : cands) {
            srj_status st = srj_batch_set_plan(B, cd.rows, cd.T, cd.waves, steps_per_graph, use_graph);
            if (st != SRJ_OK) return st;
            // every step moves 2D instances by up to T sweeps (3D instances by
            // their own plan's count)
            const int steps = std::max(1, (sweeps + cd.T - 1) / cd.T);
            float ms = 0.f;
            st = time_steps(steps, &ms);
            if (st != SRJ_OK) return st;
            const double us = 1e3 * ms / (steps * cd.T);
            if (us < best) {
                best = us;
                best_rows = cd.rows;
                best_T = cd.T;
                best_waves = cd.waves;
            }
        }
        srj_status st = srj_batch_set_plan(B, best_rows, best_T, best_waves, steps_per_graph,
                                           use_graph ? 1 : 0);
        if (st != SRJ_OK) return st;
    }
    // 3D instances: plane tile and sweeps per step, timed per sweep
    if (!B->hitems3.empty()) {
        int best_ph = B->ph3, best_zc = B->zc3, best_t3 = B->t3;
        double best3 = INFINITY;
        struct Tile {
            int ph, zc, t3;
        };
        std::vector<Tile> tiles;
#define SRJ_C3(PH, ZC) tiles.push_back({PH, ZC, 1}); tiles.push_back({PH, ZC, 2});
        SRJ_BATCH_PLANE(SRJ_C3)
#undef SRJ_C3
        for (const Tile &t : tiles) {
            srj_status st = srj_batch_set_plan3d(B, t.ph, t.zc, t.t3);
            if (st != SRJ_OK) return st;
            const int steps = std::max(1, (sweeps + t.t3 - 1) / t.t3);
            float ms = 0.f;
            st = time_steps(steps, &ms);
            if (st != SRJ_OK) return st;
            const double us = 1e3 * ms / (steps * t.t3);
            if (us < best3) {
                best3 = us;
                best_ph = t.ph;
                best_zc = t.zc;
                best_t3 = t.t3;
            }
        }
        srj_status st = srj_batch_set_plan3d(B, best_ph, best_zc, best_t3);
        if (st != SRJ_OK) return st;
        best = best3;
    }
    *best_us_per_sweep = best;
    return SRJ_OK;
}

srj_status srj_batch_destroy(srj_batch *B)
{
    batch_free(B);
    return SRJ_OK;
}

}  // extern "C"
