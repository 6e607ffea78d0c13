// Mixed-precision iterative refinement around the SRJ cycles.
//
// Not part of the paper (Islam & Wang, arXiv 2011.06636); it keeps the
// paper's cycle and selector and changes only where the cycle runs.  One
// outer step is one SRJ cycle on the correction equation A d = r:
//   r = b - A x in binary64 and its L2 norm (drives Algorithm 1 as in
//   section 3), rhat = storage(binary32(s * r)) with s a power of two,
//   d = 0, then the M sweeps of the cycle's scheme (Eq. 3, Eq. (17) factors
//   rounded to binary32) on A d = rhat in binary32 arithmetic, the iterate
//   rounded to the storage format (binary32, binary16 or bfloat16) after every
//   sweep, and finally x = x + d / s in binary64.
// With d starting at zero, one inner cycle gives d = (I - B_SRJ) A^-1 rhat,
// so in exact arithmetic the error moves as e' = B_SRJ e, exactly like a
// binary64 cycle (section 2, Eq. 7): the selector sees the same ratios.
//
// The scale applied to the residual of a pass comes from the last norm known
// before that pass (r0 for the first two passes, then the norm of the cycle
// before the previous one), so the update, the residual, its norm and the
// scaled cast are one fused pass over the grid.
#include <math.h>
#include <string.h>

#include <algorithm>

#include "internal.h"
#include "rowband.h"
#include "storage.h"
#include "tile2d.h"
#include "stream3d.h"
#include "wave2d.h"
#include "plane3d.h"
#include "plane3d_fused.h"
#include "block2d.h"
#include "block2d_face.h"

#pragma clang fp contract(off)

namespace srj {

namespace {

constexpr int kBlock = 256;
constexpr int kFinal = 1024;

__device__ __forceinline__ double block_sum256(double v, double *lds)
{
    v = wave_sum64(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) lds[wave] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0) t = ((lds[0] + lds[1]) + lds[2]) + lds[3];
    return t;
}

// One inner sweep on A d = rhat in binary32 (generic: any dimension,
// constant or per-face couplings).  Same expression order as binary64.
template <int ND, class St>
__global__ __launch_bounds__(kBlock) void k_inner_generic(DevProblem32 Q,
                                                          const typename St::T *__restrict__ d,
                                                          typename St::T *__restrict__ dout,
                                                          const typename St::T *__restrict__ rhat,
                                                          float w)
{
    const int64_t i0 = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i0 >= Q.n0) return;
    const int64_t i1 = blockIdx.y, i2 = blockIdx.z;
    const int64_t s1 = Q.n0, s2 = Q.n0 * Q.n1;
    const int64_t p = i0 + s1 * i1 + s2 * i2;
    const float dc = St::load(d[p]);
    float s = (Q.diag ? Q.diag[p] : Q.dconst) * dc;
    if (i0 > 0) s = s - (Q.face[0] ? Q.face[0][p - 1] : Q.c[0]) * St::load(d[p - 1]);
    if (i0 < Q.n0 - 1) s = s - (Q.face[0] ? Q.face[0][p] : Q.c[0]) * St::load(d[p + 1]);
    if (ND >= 2) {
        if (i1 > 0) s = s - (Q.face[1] ? Q.face[1][p - s1] : Q.c[1]) * St::load(d[p - s1]);
        if (i1 < Q.n1 - 1) s = s - (Q.face[1] ? Q.face[1][p] : Q.c[1]) * St::load(d[p + s1]);
    }
    if (ND >= 3) {
        if (i2 > 0) s = s - (Q.face[2] ? Q.face[2][p - s2] : Q.c[2]) * St::load(d[p - s2]);
        if (i2 < Q.n2 - 1) s = s - (Q.face[2] ? Q.face[2][p] : Q.c[2]) * St::load(d[p + s2]);
    }
    const float r = St::load(rhat[p]) - s;
    const float t = (Q.diag ? Q.dinv[p] : Q.dinvconst) * r;
    dout[p] = St::store(dc + w * t);
}

// Outer pass: x' = x + d / s_prev (UPDATE), r = b - A x' in binary64 with the
// neighbours' x' formed on the fly, partial sums of r^2, and
// rhat = storage(binary32(s_next * r)).  One unit of 256 columns x kNormRows
// rows per workgroup (rowband.h), as the residual norm: the partial of
// workgroup b goes to slot b (zero without a unit).  Neighbours are loaded
// from clamped indices unconditionally and a select drops the terms of ghost
// neighbours, which leaves every operation and its order unchanged.
template <int ND, class St, bool UPDATE>
__global__ __launch_bounds__(kBlock) void k_outer(DevProblem P, const double *__restrict__ x,
                                                  const typename St::T *__restrict__ d,
                                                  double inv_s, double *__restrict__ xo,
                                                  typename St::T *__restrict__ rhat, double s_next,
                                                  double *__restrict__ partials)
{
    __shared__ double lds[kBlock / 64];
    int64_t xb, y, i2;
    int ny;
    if (!row_unit(blockIdx.x, P.n0, P.n1, P.n2, kNormRows, xb, y, ny, i2)) {
        if (threadIdx.x == 0) partials[blockIdx.x] = 0.0;
        return;  // whole workgroup
    }
    const int64_t n0 = P.n0, n1 = P.n1, n2 = P.n2;
    const int64_t s1 = n0, s2 = n0 * n1;
    const int64_t i0 = xb * kBlock + threadIdx.x;
    const bool in = i0 < n0;
    const int64_t c0 = in ? i0 : n0 - 1;
    const bool h0 = c0 > 0, h1 = c0 < n0 - 1;
    const bool h4 = ND >= 3 && i2 > 0, h5 = ND >= 3 && i2 < n2 - 1;
    auto xn = [&](int64_t q) -> double {
        if (UPDATE) return x[q] + static_cast<double>(St::load(d[q])) * inv_s;
        return x[q];
    };
    double acc = 0.0;
#pragma unroll
    for (int j = 0; j < kNormRows; ++j) {
        // rows past the unit's last repeat its first row and are dropped
        const bool ok = in && j < ny;
        const int64_t i1 = y + (j < ny ? j : 0);
        const int64_t p = c0 + s1 * i1 + s2 * i2;
        const bool h2 = ND >= 2 && i1 > 0, h3 = ND >= 2 && i1 < n1 - 1;
        const int64_t q0 = h0 ? p - 1 : p, q1 = h1 ? p + 1 : p;
        const int64_t q2 = h2 ? p - s1 : p, q3 = h3 ? p + s1 : p;
        const int64_t q4 = h4 ? p - s2 : p, q5 = h5 ? p + s2 : p;
        const double xc = xn(p);
        double s = (P.diag ? P.diag[p] : P.dconst) * xc;
        {
            const double v0 = xn(q0), v1 = xn(q1);
            const double f0 = P.face[0] ? P.face[0][q0] : P.c[0];
            const double f1 = P.face[0] ? P.face[0][p] : P.c[0];
            s = h0 ? s - f0 * v0 : s;
            s = h1 ? s - f1 * v1 : s;
        }
        if (ND >= 2) {
            const double v2 = xn(q2), v3 = xn(q3);
            const double f2 = P.face[1] ? P.face[1][q2] : P.c[1];
            const double f3 = P.face[1] ? P.face[1][p] : P.c[1];
            s = h2 ? s - f2 * v2 : s;
            s = h3 ? s - f3 * v3 : s;
        }
        if (ND >= 3) {
            const double v4 = xn(q4), v5 = xn(q5);
            const double f4 = P.face[2] ? P.face[2][q4] : P.c[2];
            const double f5 = P.face[2] ? P.face[2][p] : P.c[2];
            s = h4 ? s - f4 * v4 : s;
            s = h5 ? s - f5 * v5 : s;
        }
        const double r = P.b[p] - s;
        if (ok) {
            if (UPDATE) xo[p] = xc;
            rhat[p] = St::store(static_cast<float>(s_next * r));
        }
        acc = j == 0 ? (ok ? r * r : 0.0) : acc + (ok ? r * r : 0.0);
    }
    const double t = block_sum256(acc, lds);
    if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

template <class T>
__global__ void k_zero(T *__restrict__ a, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = T(0);
}

__global__ void k_to_f32(const double *__restrict__ a, float *__restrict__ o, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) o[i] = static_cast<float>(a[i]);
}

__global__ void k_inv_to_f32(const double *__restrict__ a, float *__restrict__ o, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) o[i] = static_cast<float>(1.0 / a[i]);
}

// One workgroup per 256 points of a row (x), rows (y), planes (z).
dim3 point_grid(int64_t n0, int64_t n1, int64_t n2)
{
    return dim3((unsigned)((n0 + kBlock - 1) / kBlock), (unsigned)n1, (unsigned)n2);
}

// Fused inner-sweep variants (tile rows, halo); binary32 arithmetic keeps two
// values per register pair less than binary64, so taller tiles fit.
#define SRJ_INNER_VARIANTS(X) \
    X(16, 2) X(24, 4) X(32, 4) X(32, 6) X(48, 6) X(48, 8) X(64, 8)

template <class St>
hipError_t launch_inner_fused(const SweepPlan &plan, const DevProblem32 &Q, const void *d, void *dout,
                              const void *rhat, const float *w_dev, int T, hipStream_t s,
                              bool reverse = false)
{
    using TT = typename St::T;
    const Coef2D<float> k2{Q.dconst, Q.dinvconst, Q.c[0], Q.c[1]};
    const TT *dd = static_cast<const TT *>(d);
    TT *oo = static_cast<TT *>(dout);
    const TT *rr = static_cast<const TT *>(rhat);
    if (plan.kind == 7 || plan.kind == 8) {
#define SRJ_GO1(HW, HL, NW)                                                         \
    if (plan.by == HW && plan.occ == NW && plan.T <= HL)                            \
        return launch_block2d<St, HW, HL, NW, 1>(Q.n0, Q.n1, dd, oo, rr, w_dev, T, k2, s, reverse);
#define SRJ_GO2(HW, HL, NW)                                                         \
    if (plan.by == HW && plan.occ == NW && plan.T <= HL)                            \
        return launch_block2d<St, HW, HL, NW, 2>(Q.n0, Q.n1, dd, oo, rr, w_dev, T, k2, s, reverse);
        if (plan.kind == 7) { SRJ_INNER_BLOCK_VARIANTS(SRJ_GO1) }
        else { SRJ_INNER_BLOCK2_VARIANTS(SRJ_GO2) }
#undef SRJ_GO1
#undef SRJ_GO2
        return hipErrorInvalidValue;
    }
    if (plan.kind == 10) {
#define SRJ_GOF(HW, HL, NW)                                                                    \
    if (plan.by == HW && plan.occ == NW && plan.T <= HL)                                       \
        return launch_blockf2d<St, HW, HL, NW>(Q.n0, Q.n1, dd, oo, rr, Q.face[0], Q.face[1], Q.diag, \
                                               Q.dinv, w_dev, T, s, reverse);
        SRJ_INNER_BLOCKF_VARIANTS(SRJ_GOF)
#undef SRJ_GOF
        return hipErrorInvalidValue;
    }
    if (plan.kind == 12) {
        const Stencil3<float> S{Q.n0, Q.n1, Q.n2, {Q.c[0], Q.c[1], Q.c[2]},
                                {Q.face[0], Q.face[1], Q.face[2]}, Q.dconst, Q.dinvconst,
                                Q.diag, Q.dinv};
        // the last launch of an odd-length cycle does one sweep
        if (T == 1) return launch_plane3d<St, 4, 8>(S, dd, oo, rr, w_dev, s);
        if (T != 2) return hipErrorInvalidValue;
#define SRJ_GO(HH, ZZ) \
    if (plan.by == HH && plan.occ == ZZ) return launch_plane3d2f<St, HH, ZZ>(S, dd, oo, rr, w_dev, s);
        SRJ_INNER_PLANE2F_VARIANTS(SRJ_GO)
#undef SRJ_GO
        return hipErrorInvalidValue;
    }
    if (plan.kind == 11) {
        const Stencil3<float> S{Q.n0, Q.n1, Q.n2, {Q.c[0], Q.c[1], Q.c[2]},
                                {nullptr, nullptr, nullptr}, Q.dconst, Q.dinvconst, nullptr,
                                nullptr};
        // the last launch of an odd-length cycle does one sweep
        if (T == 1) return launch_plane3d<St, 4, 8>(S, dd, oo, rr, w_dev, s);
        if (T != 2) return hipErrorInvalidValue;
#define SRJ_GO(HH, ZZ) \
    if (plan.by == HH && plan.occ == ZZ) return launch_plane3d2<St, HH, ZZ>(S, dd, oo, rr, w_dev, s);
        SRJ_INNER_PLANE2_VARIANTS(SRJ_GO)
#undef SRJ_GO
        return hipErrorInvalidValue;
    }
    if (plan.kind == 6) {
        const Stencil3<float> S{Q.n0, Q.n1, Q.n2, {Q.c[0], Q.c[1], Q.c[2]},
                                {Q.face[0], Q.face[1], Q.face[2]}, Q.dconst, Q.dinvconst,
                                Q.diag, Q.dinv};
#define SRJ_GO(HH, ZZ) \
    if (plan.by == HH && plan.occ == ZZ) return launch_plane3d<St, HH, ZZ>(S, dd, oo, rr, w_dev, s);
        SRJ_PLANE_VARIANTS(SRJ_GO)
#undef SRJ_GO
        return hipErrorInvalidValue;
    }
    if (plan.kind == 5) {
#define SRJ_GO(OH, TM) \
    if (plan.by == OH && plan.T <= TM) return launch_wave2d<St, OH, TM>(T, Q.n0, Q.n1, dd, oo, rr, w_dev, k2, s);
        SRJ_WAVE_VARIANTS(SRJ_GO)
#undef SRJ_GO
        return hipErrorInvalidValue;
    }
    if (plan.kind == 3) {
        const Stencil3<float> S{Q.n0, Q.n1, Q.n2, {Q.c[0], Q.c[1], Q.c[2]},
                                {Q.face[0], Q.face[1], Q.face[2]}, Q.dconst, Q.dinvconst,
                                Q.diag, Q.dinv};
#define SRJ_GO(Z) if (plan.by == Z) return launch_stream3d<St, Z>(S, dd, oo, rr, w_dev, s);
        SRJ_3D_CHUNKS(SRJ_GO)
#undef SRJ_GO
        return hipErrorInvalidValue;
    }
#define SRJ_TRY(R, HL)                                                                      \
    if (plan.by == R && plan.T <= HL)                                                        \
        return launch_tile2d<St, R, HL, false, 1>(Q.n0, Q.n1, dd, oo, rr, w_dev, T, k2, s);
    SRJ_INNER_VARIANTS(SRJ_TRY)
#undef SRJ_TRY
    return hipErrorInvalidValue;
}

template <class St>
hipError_t launch_inner(const DevProblem32 &Q, const void *d, void *dout, const void *rhat, float w,
                        hipStream_t s)
{
    using T = typename St::T;
    const dim3 g = point_grid(Q.n0, Q.n1, Q.n2);
    const T *dd = static_cast<const T *>(d);
    T *oo = static_cast<T *>(dout);
    const T *rr = static_cast<const T *>(rhat);
    switch (Q.ndim) {
    case 1: hipLaunchKernelGGL((k_inner_generic<1, St>), g, dim3(kBlock), 0, s, Q, dd, oo, rr, w); break;
    case 2: hipLaunchKernelGGL((k_inner_generic<2, St>), g, dim3(kBlock), 0, s, Q, dd, oo, rr, w); break;
    default: hipLaunchKernelGGL((k_inner_generic<3, St>), g, dim3(kBlock), 0, s, Q, dd, oo, rr, w); break;
    }
    return hipGetLastError();
}

template <class St, bool UPDATE>
hipError_t launch_outer_t(const DevProblem &P, const double *x, const void *d, double inv_s,
                          double *xo, void *rhat, double s_next, double *partials, hipStream_t s)
{
    using T = typename St::T;
    const dim3 g((unsigned)residual_blocks(P));  // one workgroup per partial
    const T *dd = static_cast<const T *>(d);
    T *rh = static_cast<T *>(rhat);
    switch (P.ndim) {
    case 1: hipLaunchKernelGGL((k_outer<1, St, UPDATE>), g, dim3(kBlock), 0, s, P, x, dd, inv_s, xo, rh, s_next, partials); break;
    case 2: hipLaunchKernelGGL((k_outer<2, St, UPDATE>), g, dim3(kBlock), 0, s, P, x, dd, inv_s, xo, rh, s_next, partials); break;
    default: hipLaunchKernelGGL((k_outer<3, St, UPDATE>), g, dim3(kBlock), 0, s, P, x, dd, inv_s, xo, rh, s_next, partials); break;
    }
    return hipGetLastError();
}

template <class St>
hipError_t launch_outer(bool update, const DevProblem &P, const double *x, const void *d,
                        double inv_s, double *xo, void *rhat, double s_next, double *partials,
                        hipStream_t s)
{
    if (update) return launch_outer_t<St, true>(P, x, d, inv_s, xo, rhat, s_next, partials, s);
    return launch_outer_t<St, false>(P, x, d, inv_s, xo, rhat, s_next, partials, s);
}

}  // namespace

bool inner_fused_supported(const DevProblem &P, const SweepPlan &plan)
{
    if (P.ell_len) return false;
    if (plan.kind == 7 || plan.kind == 8) {
        if (!(P.ndim == 2 && !P.face[0] && !P.face[1] && !P.diag) || plan.T < 1) return false;
#define SRJ_CHK(HW, HL, NW) if (plan.by == HW && plan.occ == NW && plan.T <= HL) return true;
        if (plan.kind == 7) { SRJ_INNER_BLOCK_VARIANTS(SRJ_CHK) }
        else { SRJ_INNER_BLOCK2_VARIANTS(SRJ_CHK) }
#undef SRJ_CHK
        return false;
    }
    if (plan.kind == 10) {
        if (!(P.ndim == 2 && P.face[0] && P.face[1] && P.diag) || plan.T < 1) return false;
#define SRJ_CHK(HW, HL, NW) if (plan.by == HW && plan.occ == NW && plan.T <= HL) return true;
        SRJ_INNER_BLOCKF_VARIANTS(SRJ_CHK)
#undef SRJ_CHK
        return false;
    }
    if (plan.kind == 12) {
        if (!(P.ndim == 3 && P.face[0] && P.face[1] && P.face[2] && P.diag) || plan.T < 1 ||
            plan.T > 2)
            return false;
#define SRJ_CHK(HH, ZZ) if (plan.by == HH && plan.occ == ZZ) return true;
        SRJ_INNER_PLANE2F_VARIANTS(SRJ_CHK)
#undef SRJ_CHK
        return false;
    }
    if (plan.kind == 11) {
        if (!(P.ndim == 3 && !P.face[0] && !P.face[1] && !P.face[2] && !P.diag) || plan.T < 1 ||
            plan.T > 2)
            return false;
#define SRJ_CHK(HH, ZZ) if (plan.by == HH && plan.occ == ZZ) return true;
        SRJ_INNER_PLANE2_VARIANTS(SRJ_CHK)
#undef SRJ_CHK
        return false;
    }
    if (plan.kind == 6) {
        if (!plane3d_fits(P.ndim, P.face[0], P.face[1], P.face[2], P.diag) || plan.T != 1)
            return false;
#define SRJ_CHK(HH, ZZ) if (plan.by == HH && plan.occ == ZZ) return true;
        SRJ_PLANE_VARIANTS(SRJ_CHK)
#undef SRJ_CHK
        return false;
    }
    if (plan.kind == 5) {
        if (!(P.ndim == 2 && !P.face[0] && !P.face[1] && !P.diag) || plan.occ != 1 || plan.T < 1)
            return false;
#define SRJ_CHK(OH, TM) if (plan.by == OH && plan.T <= TM) return true;
        SRJ_WAVE_VARIANTS(SRJ_CHK)
#undef SRJ_CHK
        return false;
    }
    if (plan.kind == 3) {
        if (P.ndim != 3 || plan.T != 1 || plan.occ != 1) return false;
#define SRJ_CHK(Z) if (plan.by == Z) return true;
        SRJ_3D_CHUNKS(SRJ_CHK)
#undef SRJ_CHK
        return false;
    }
    if (plan.kind != 1 || plan.occ != 1 || plan.T < 1) return false;
    if (!(P.ndim == 2 && !P.face[0] && !P.face[1] && !P.diag)) return false;
#define SRJ_CHECK(R, HL) \
    if (plan.by == R && plan.T <= HL) return true;
    SRJ_INNER_VARIANTS(SRJ_CHECK)
#undef SRJ_CHECK
    return false;
}

int inner_plan_variants(int32_t *out, int cap)
{
    int n = 0;
#define SRJ_LIST7(HW, HL, NW)          \
    if (n < cap) {                     \
        out[4 * n + 0] = KIND;         \
        out[4 * n + 1] = HW;           \
        out[4 * n + 2] = HL;           \
        out[4 * n + 3] = NW;           \
    }                                  \
    ++n;
#define KIND 7
    SRJ_INNER_BLOCK_VARIANTS(SRJ_LIST7)
#undef KIND
#define KIND 8
    SRJ_INNER_BLOCK2_VARIANTS(SRJ_LIST7)
#undef KIND
#define KIND 10
    SRJ_INNER_BLOCKF_VARIANTS(SRJ_LIST7)
#undef KIND
#undef SRJ_LIST7
#define SRJ_LIST6(HH, ZZ)              \
    if (n < cap) {                     \
        out[4 * n + 0] = 6;            \
        out[4 * n + 1] = HH;           \
        out[4 * n + 2] = 1;            \
        out[4 * n + 3] = ZZ;           \
    }                                  \
    ++n;
    SRJ_PLANE_VARIANTS(SRJ_LIST6)
#undef SRJ_LIST6
#define SRJ_LIST11(HH, ZZ)             \
    if (n < cap) {                     \
        out[4 * n + 0] = 11;           \
        out[4 * n + 1] = HH;           \
        out[4 * n + 2] = 2;            \
        out[4 * n + 3] = ZZ;           \
    }                                  \
    ++n;
    SRJ_INNER_PLANE2_VARIANTS(SRJ_LIST11)
#undef SRJ_LIST11
#define SRJ_LIST12(HH, ZZ)             \
    if (n < cap) {                     \
        out[4 * n + 0] = 12;           \
        out[4 * n + 1] = HH;           \
        out[4 * n + 2] = 2;            \
        out[4 * n + 3] = ZZ;           \
    }                                  \
    ++n;
    SRJ_INNER_PLANE2F_VARIANTS(SRJ_LIST12)
#undef SRJ_LIST12
#define SRJ_LIST5(OH, TM)              \
    if (n < cap) {                     \
        out[4 * n + 0] = 5;            \
        out[4 * n + 1] = OH;           \
        out[4 * n + 2] = TM;           \
        out[4 * n + 3] = 1;            \
    }                                  \
    ++n;
    SRJ_WAVE_VARIANTS(SRJ_LIST5)
#undef SRJ_LIST5
#define SRJ_LIST3(Z)                   \
    if (n < cap) {                     \
        out[4 * n + 0] = 3;            \
        out[4 * n + 1] = Z;            \
        out[4 * n + 2] = 1;            \
        out[4 * n + 3] = 1;            \
    }                                  \
    ++n;
    SRJ_3D_CHUNKS(SRJ_LIST3)
#undef SRJ_LIST3
#define SRJ_LIST(R, HL)                \
    if (n < cap) {                     \
        out[4 * n + 0] = 1;            \
        out[4 * n + 1] = R;            \
        out[4 * n + 2] = HL;           \
        out[4 * n + 3] = 1;            \
    }                                  \
    ++n;
    SRJ_INNER_VARIANTS(SRJ_LIST)
#undef SRJ_LIST
    return n;
}

// ---------------------------------------------------------------------------
// Workspaces
// ---------------------------------------------------------------------------
struct Refine {
    int bytes = 0;                 // storage bytes per element the buffers hold
    void *da = nullptr, *db = nullptr, *rhat = nullptr;
    float *face32[3] = {nullptr, nullptr, nullptr};
    float *d32 = nullptr, *dinv32 = nullptr;
    bool op_ready = false;
};

void refine_free(srj_ctx *c)
{
    if (!c || !c->refine) return;
    Refine *R = c->refine;
    (void)hipFree(R->da);
    (void)hipFree(R->db);
    (void)hipFree(R->rhat);
    for (int d = 0; d < 3; ++d) (void)hipFree(R->face32[d]);
    (void)hipFree(R->d32);
    (void)hipFree(R->dinv32);
    delete R;
    c->refine = nullptr;
}

namespace {

int storage_bytes(srj_precision p) { return p == SRJ_PREC_F32_REFINE ? 4 : 2; }

srj_status ensure_workspace(srj_ctx *c, srj_precision prec)
{
    if (!c->refine) c->refine = new Refine();
    Refine *R = c->refine;
    const int64_t N = c->npoints;
    const int bytes = storage_bytes(prec);
    if (R->bytes < bytes) {
        (void)hipFree(R->da);
        (void)hipFree(R->db);
        (void)hipFree(R->rhat);
        R->da = R->db = R->rhat = nullptr;
        R->bytes = 0;
        if (hipMalloc(&R->da, (size_t)N * bytes) != hipSuccess ||
            hipMalloc(&R->db, (size_t)N * bytes) != hipSuccess ||
            hipMalloc(&R->rhat, (size_t)N * bytes) != hipSuccess)
            return fail(SRJ_ERR_NOMEM, "hipMalloc failed for refinement buffers");
        R->bytes = bytes;
    }
    if (!R->op_ready) {
        const int64_t blocks = (N + 255) / 256;
        for (int d = 0; d < c->P.ndim; ++d) {
            if (!c->P.face[d]) continue;
            if (hipMalloc(&R->face32[d], sizeof(float) * (size_t)N) != hipSuccess)
                return fail(SRJ_ERR_NOMEM, "hipMalloc failed for binary32 couplings");
            hipLaunchKernelGGL(k_to_f32, dim3((unsigned)blocks), dim3(256), 0, c->stream,
                               c->P.face[d], R->face32[d], N);
            SRJ_HIP_CHECK(hipGetLastError());
        }
        if (c->P.diag) {
            if (hipMalloc(&R->d32, sizeof(float) * (size_t)N) != hipSuccess ||
                hipMalloc(&R->dinv32, sizeof(float) * (size_t)N) != hipSuccess)
                return fail(SRJ_ERR_NOMEM, "hipMalloc failed for binary32 diagonal");
            hipLaunchKernelGGL(k_to_f32, dim3((unsigned)blocks), dim3(256), 0, c->stream,
                               c->P.diag, R->d32, N);
            SRJ_HIP_CHECK(hipGetLastError());
            hipLaunchKernelGGL(k_inv_to_f32, dim3((unsigned)blocks), dim3(256), 0, c->stream,
                               c->P.diag, R->dinv32, N);
            SRJ_HIP_CHECK(hipGetLastError());
        }
        R->op_ready = true;
    }
    return SRJ_OK;
}

DevProblem32 make_q(const srj_ctx *c)
{
    const DevProblem &P = c->P;
    const Refine *R = c->refine;
    DevProblem32 Q{};
    Q.ndim = P.ndim;
    Q.n0 = P.n0;
    Q.n1 = P.n1;
    Q.n2 = P.n2;
    for (int d = 0; d < 3; ++d) {
        Q.c[d] = static_cast<float>(P.c[d]);
        Q.face[d] = R->face32[d];
    }
    Q.diag = R->d32;
    Q.dinv = R->dinv32;
    Q.dconst = P.diag ? 0.f : static_cast<float>(P.dconst);
    Q.dinvconst = P.diag ? 0.f : static_cast<float>(1.0 / P.dconst);
    return Q;
}

// Largest power of two not above target_rms * sqrt(N) / norm (1 for a zero
// or non-finite norm).
double pow2_scale(double norm, int64_t N, double target_rms)
{
    if (!(norm > 0.0) || !isfinite(norm)) return 1.0;
    const double q = target_rms * sqrt(static_cast<double>(N)) / norm;
    int e = 0;
    frexp(q, &e);
    return ldexp(1.0, e - 1);
}

template <class St>
srj_status zero_storage(srj_ctx *c, void *a)
{
    const int64_t N = c->npoints;
    hipLaunchKernelGGL(k_zero<typename St::T>, dim3((unsigned)((N + 255) / 256)), dim3(256), 0,
                       c->stream, static_cast<typename St::T *>(a), N);
    SRJ_HIP_CHECK(hipGetLastError());
    return SRJ_OK;
}

template <class St>
srj_status solve_t(srj_ctx *c, double *x, const srj_solve_opts *o, srj_solve_result *res,
                   int32_t *levels_out, double *norms_out)
{
    srj_status st = ensure_workspace(c, o->precision);
    if (st != SRJ_OK) return st;
    Refine *R = c->refine;
    const DevProblem32 Q = make_q(c);
    const int64_t N = c->npoints;
    const double tgt = o->scale_target > 0.0 ? o->scale_target
                       : (o->precision == SRJ_PREC_F16_REFINE ? ldexp(1.0, -8) : 1.0);
    const int64_t nb = residual_blocks(c->P);
    const bool fused = inner_fused_supported(c->P, c->plan_inner);

    double *cur = x, *nxt = c->ws;
    double norm0 = 0.0;
    st = residual_norm(c, x, &norm0);
    if (st != SRJ_OK) return st;
    const double r0 = o->r0 > 0.0 ? o->r0 : norm0;
    res->r0 = r0;
    res->r_final = norm0;
    if (norms_out) norms_out[0] = norm0;
    const double target = o->tol_mode == SRJ_TOL_RELATIVE ? o->tol * r0 : o->tol;
    srj_status status = SRJ_ERR_NOT_CONVERGED;
    int level = o->start_level;
    double prev = norm0;
    if (!isfinite(norm0)) {
        status = fail(SRJ_ERR_NONFINITE, "initial residual norm is not finite");
    } else if (norm0 == 0.0 || norm0 < target) {
        res->converged = 1;
        status = SRJ_OK;
    } else {
        double s = pow2_scale(norm0, N, tgt);
        SRJ_HIP_CHECK(launch_outer<St>(false, c->P, cur, nullptr, 0.0, nullptr, R->rhat, s,
                                       c->rs.partials, c->stream));
        void *da = R->da, *db = R->db;
        for (int cycle = 0; cycle < o->max_cycles; ++cycle) {
            const int lv = o->rule == SRJ_RULE_FIXED ? o->fixed_level : level;
            const int M = c->levelM[lv];
            if (res->sweeps + M > o->max_sweeps) break;
            st = zero_storage<St>(c, da);
            if (st != SRJ_OK) return st;
            const float *w32dev = c->omega32_dev + c->offsets[lv];
            int64_t launches = 0;
            if (c->profiling) SRJ_HIP_CHECK(hipEventRecord(c->ev0, c->stream));
            if (fused) {
                for (int done = 0; done < M;) {
                    const int T = std::min(c->plan_inner.T, M - done);
                    SRJ_HIP_CHECK(launch_inner_fused<St>(c->plan_inner, Q, da, db, R->rhat,
                                                         w32dev + done, T, c->stream, c->reverse));
                    c->reverse = !c->reverse;
                    std::swap(da, db);
                    done += T;
                    ++launches;
                }
            } else {
                const std::vector<double> &w = c->factors[lv];
                for (int k = 0; k < M; ++k) {
                    SRJ_HIP_CHECK(launch_inner<St>(Q, da, db, R->rhat, static_cast<float>(w[k]),
                                                   c->stream));
                    std::swap(da, db);
                    ++launches;
                }
            }
            if (c->profiling) {
                SRJ_HIP_CHECK(hipEventRecord(c->ev1, c->stream));
                c->prof_pending = true;
                c->prof_pending_launches = launches;
                c->prof_pending_sweeps = M;
            }
            res->sweeps += M;
            const double s_next = pow2_scale(prev, N, tgt);
            SRJ_HIP_CHECK(launch_outer<St>(true, c->P, cur, da, 1.0 / s, nxt, R->rhat, s_next,
                                           c->rs.partials, c->stream));
            std::swap(cur, nxt);
            SRJ_HIP_CHECK(launch_fold(c->rs, nb, c->stream));  // into *rs.host_sum
            SRJ_HIP_CHECK(hipStreamSynchronize(c->stream));
            st = collect_profile(c);
            if (st != SRJ_OK) return st;
            const double norm = sqrt(*c->rs.host_sum);
            s = s_next;
            res->cycles = cycle + 1;
            res->r_final = norm;
            res->final_level = lv;
            if (levels_out) levels_out[cycle] = lv;
            if (norms_out) norms_out[cycle + 1] = norm;
            if (!isfinite(norm)) {
                status = fail(SRJ_ERR_NONFINITE, "residual norm is not finite");
                break;
            }
            if (norm < target) {
                res->converged = 1;
                status = SRJ_OK;
                break;
            }
            const double ratio = norm / prev;
            prev = norm;
            if (o->rule == SRJ_RULE_HEURISTIC) {
                const double m = std::min(fabs(ratio - 0.2), fabs(ratio - 0.4));
                res->min_margin = std::min(res->min_margin, m);
            }
            level = next_level(o->rule, level, ratio, o->max_level);
        }
        if (status == SRJ_ERR_NOT_CONVERGED) set_error("cycle or sweep cap reached");
    }
    if (cur != x)
        SRJ_HIP_CHECK(hipMemcpyAsync(x, cur, sizeof(double) * (size_t)N, hipMemcpyDeviceToDevice,
                                     c->stream));
    SRJ_HIP_CHECK(hipStreamSynchronize(c->stream));
    return status;
}

}  // namespace

// Runs `sweeps` binary32 inner sweeps with `plan` on the refinement
// workspaces (contents are scratch) and returns the elapsed milliseconds
// between HIP events on the context's stream.
srj_status time_inner_plan(srj_ctx *c, const SweepPlan &plan, int sweeps, const float *w_dev,
                           float *ms)
{
    srj_status st = ensure_workspace(c, SRJ_PREC_F32_REFINE);
    if (st != SRJ_OK) return st;
    Refine *R = c->refine;
    const DevProblem32 Q = make_q(c);
    const bool fused = plan.kind != 0;
    void *da = R->da, *db = R->db;
    st = zero_storage<StF32>(c, da);
    if (st != SRJ_OK) return st;
    st = zero_storage<StF32>(c, R->rhat);
    if (st != SRJ_OK) return st;
    bool reverse = false;
    auto run = [&](int n) -> srj_status {
        for (int done = 0; done < n;) {
            const int T = fused ? std::min(plan.T, n - done) : 1;
            if (fused) {
                SRJ_HIP_CHECK(launch_inner_fused<StF32>(plan, Q, da, db, R->rhat, w_dev, T, c->stream,
                                                        reverse));
                reverse = !reverse;
            } else {
                SRJ_HIP_CHECK(launch_inner<StF32>(Q, da, db, R->rhat, 0.6666667f, c->stream));
            }
            std::swap(da, db);
            done += T;
        }
        return SRJ_OK;
    };
    st = run(fused ? plan.T : 1);  // warm-up
    if (st != SRJ_OK) return st;
    SRJ_HIP_CHECK(hipEventRecord(c->ev0, c->stream));
    st = run(sweeps);
    if (st != SRJ_OK) return st;
    SRJ_HIP_CHECK(hipEventRecord(c->ev1, c->stream));
    SRJ_HIP_CHECK(hipEventSynchronize(c->ev1));
    SRJ_HIP_CHECK(hipEventElapsedTime(ms, c->ev0, c->ev1));
    return SRJ_OK;
}

srj_status refine_solve(srj_ctx *c, double *x, const srj_solve_opts *o, srj_solve_result *res,
                        int32_t *levels_out, double *norms_out)
{
    switch (o->precision) {
    case SRJ_PREC_F32_REFINE: return solve_t<StF32>(c, x, o, res, levels_out, norms_out);
    case SRJ_PREC_F16_REFINE: return solve_t<StF16>(c, x, o, res, levels_out, norms_out);
    case SRJ_PREC_BF16_REFINE: return solve_t<StBF16>(c, x, o, res, levels_out, norms_out);
    default: return fail(SRJ_ERR_INVALID, "not a refinement precision");
    }
}

}  // namespace srj
