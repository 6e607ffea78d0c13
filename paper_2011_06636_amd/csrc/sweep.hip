// Relaxed Jacobi sweeps in binary64 (Islam & Wang, arXiv 2011.06636,
// section 2, Eq. 3, written in residual form x' = x + w D^-1 (b - A x)).
//
// Every kernel evaluates the same per-point expression in the same order
//     s = D_p x_p; s -= c_lo x[p - e_0]; s -= c_hi x[p + e_0]; (then axes 1, 2)
//     x'_p = x_p + w * (Dinv_p * (b_p - s))
// with no fused multiply-add, so the iterate is bit-identical whatever kernel,
// tile shape or number of fused sweeps is used.  A ghost neighbour holds zero;
// subtracting c * 0 leaves s unchanged, which equals omitting the term.
#include "internal.h"
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

constexpr int kGenericBlock = 256;

// ---------------------------------------------------------------------------
// Generic kernel: one sweep per launch, any dimension, constant or per-face
// couplings, constant or per-point diagonal.  Block = 256 points of one row
// along the contiguous axis; grid = (row blocks, n1, n2).
// ---------------------------------------------------------------------------
template <int ND>
__global__ __launch_bounds__(kGenericBlock) void k_sweep_generic(DevProblem P,
                                                                 const double *__restrict__ x,
                                                                 double *__restrict__ xo,
                                                                 double w)
{
    const int64_t i0 = (int64_t)blockIdx.x * kGenericBlock + threadIdx.x;
    if (i0 >= P.n0) return;
    const int64_t i1 = blockIdx.y, i2 = blockIdx.z;
    const int64_t s1 = P.n0, s2 = P.n0 * P.n1;
    const int64_t p = i0 + s1 * i1 + s2 * i2;
    const double xc = x[p];
    double s = (P.diag ? P.diag[p] : P.dconst) * xc;
    if (i0 > 0) s = s - (P.face[0] ? P.face[0][p - 1] : P.c[0]) * x[p - 1];
    if (i0 < P.n0 - 1) s = s - (P.face[0] ? P.face[0][p] : P.c[0]) * x[p + 1];
    if (ND >= 2) {
        if (i1 > 0) s = s - (P.face[1] ? P.face[1][p - s1] : P.c[1]) * x[p - s1];
        if (i1 < P.n1 - 1) s = s - (P.face[1] ? P.face[1][p] : P.c[1]) * x[p + s1];
    }
    if (ND >= 3) {
        if (i2 > 0) s = s - (P.face[2] ? P.face[2][p - s2] : P.c[2]) * x[p - s2];
        if (i2 < P.n2 - 1) s = s - (P.face[2] ? P.face[2][p] : P.c[2]) * x[p + s2];
    }
    const double r = P.b[p] - s;
    const double t = (P.diag ? P.dinv[p] : P.dinvconst) * r;
    xo[p] = xc + w * t;
}

// The generic sweep with the update test of the Neumann Laplace problem
// (section 4.2.2, Eq. (25)): the same per-point expression, plus the largest
// |x' - x| of the sweep, reduced per block and merged with one 64-bit atomic
// max into one of 64 stripes (a maximum does not depend on the order or the
// grouping of the merges).  A launch whose
// predecessor's maximum is below tol does nothing but record the stop; so do
// all later launches.
template <int ND>
__global__ __launch_bounds__(kGenericBlock) void k_sweep_upd(DevProblem P, const double *__restrict__ x,
                                                             double *__restrict__ xo, double w,
                                                             double tol, UpdState *st, int64_t g)
{
    __shared__ unsigned long long red[kGenericBlock / 64];
    constexpr int kSlot = kUpdStripes * kUpdStride;
    const int lane = threadIdx.x & 63;
    const bool lead_block = blockIdx.x == 0 && blockIdx.y == 0 && blockIdx.z == 0;
    if (st->flag) return;  // an earlier sweep met the test
    if (g > 0) {
        // every wave folds the previous sweep's stripes (one per lane)
        unsigned long long m = st->maxbits[((g - 1) % 3) * kSlot + lane * kUpdStride];
        for (int off = 32; off > 0; off >>= 1) {
            const unsigned long long o = __shfl_xor(m, off);
            m = o > m ? o : m;
        }
        if (__longlong_as_double((long long)m) < tol) {
            if (lead_block && threadIdx.x == 0) {
                st->flag = 1;
                st->stop = g - 1;
            }
            return;
        }
    }
    if (lead_block && threadIdx.x < 64)  // the slot of the next sweep
        st->maxbits[((g + 1) % 3) * kSlot + lane * kUpdStride] = 0ull;
    const int64_t i0 = (int64_t)blockIdx.x * kGenericBlock + threadIdx.x;
    unsigned long long d = 0ull;
    if (i0 < P.n0) {
        const int64_t i1 = blockIdx.y, i2 = blockIdx.z;
        const int64_t s1 = P.n0, s2 = P.n0 * P.n1;
        const int64_t p = i0 + s1 * i1 + s2 * i2;
        const double xc = x[p];
        double s = (P.diag ? P.diag[p] : P.dconst) * xc;
        if (i0 > 0) s = s - (P.face[0] ? P.face[0][p - 1] : P.c[0]) * x[p - 1];
        if (i0 < P.n0 - 1) s = s - (P.face[0] ? P.face[0][p] : P.c[0]) * x[p + 1];
        if (ND >= 2) {
            if (i1 > 0) s = s - (P.face[1] ? P.face[1][p - s1] : P.c[1]) * x[p - s1];
            if (i1 < P.n1 - 1) s = s - (P.face[1] ? P.face[1][p] : P.c[1]) * x[p + s1];
        }
        if (ND >= 3) {
            if (i2 > 0) s = s - (P.face[2] ? P.face[2][p - s2] : P.c[2]) * x[p - s2];
            if (i2 < P.n2 - 1) s = s - (P.face[2] ? P.face[2][p] : P.c[2]) * x[p + s2];
        }
        const double r = P.b[p] - s;
        const double t = (P.diag ? P.dinv[p] : P.dinvconst) * r;
        const double xn = xc + w * t;
        xo[p] = xn;
        d = (unsigned long long)__double_as_longlong(fabs(xn - xc));
    }
    for (int off = 32; off > 0; off >>= 1) {
        const unsigned long long o = __shfl_xor(d, off);
        d = o > d ? o : d;
    }
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = d;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long m = red[0];
        for (int i = 1; i < kGenericBlock / 64; ++i) m = red[i] > m ? red[i] : m;
        const int stripe = (int)((blockIdx.x + (uint64_t)gridDim.x * (blockIdx.y + (uint64_t)gridDim.y * blockIdx.z)) % kUpdStripes);
        atomicMax(&st->maxbits[(g % 3) * kSlot + stripe * kUpdStride], m);
    }
}

// General sparse matrix: one sweep, one thread per row (ELL layout, so the
// k-th entries of consecutive rows are adjacent in memory).
__global__ __launch_bounds__(kGenericBlock) void k_sweep_ell(DevProblem P, const double *__restrict__ x,
                                                             double *__restrict__ xo, double w)
{
    const int64_t p = (int64_t)blockIdx.x * kGenericBlock + threadIdx.x;
    if (p >= P.n0) return;
    const double xc = x[p];
    double s = P.diag[p] * xc;
    const int len = P.ell_len[p];
    for (int j = 0; j < len; ++j)
        s = s + P.ell_val[(int64_t)j * P.n0 + p] * x[P.ell_col[(int64_t)j * P.n0 + p]];
    const double r = P.b[p] - s;
    const double t = P.dinv[p] * r;
    xo[p] = xc + w * t;
}

__global__ void k_dinv(const double *__restrict__ d, double *__restrict__ dinv, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dinv[i] = 1.0 / d[i];
}

// Tile variants: rows H, halo (= most sweeps per launch), b in LDS or not.
struct TileVariant {
    int rows, halo;
    bool blds;
    int occ;
};
#define SRJ_2D_VARIANTS(X)                                                              \
    X(16, 2, false, 1) X(16, 2, false, 4) X(24, 3, false, 1) X(24, 3, false, 3)          \
    X(24, 4, false, 1) X(24, 4, false, 3) X(32, 4, false, 1) X(32, 4, false, 2)          \
    X(32, 4, false, 3) X(32, 4, true, 1) X(32, 4, true, 4) X(40, 5, true, 3)             \
    X(48, 6, true, 2) X(48, 6, true, 3)
#define SRJ_VARIANT_ENTRY(R, HL, BL, OC) {R, HL, BL, OC},
constexpr TileVariant kVariants[] = {SRJ_2D_VARIANTS(SRJ_VARIANT_ENTRY)};
#undef SRJ_VARIANT_ENTRY

}  // namespace

hipError_t compute_dinv(const double *diag, double *dinv, int64_t n, hipStream_t s)
{
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(k_dinv, dim3((unsigned)blocks), dim3(256), 0, s, diag, dinv, n);
    return hipGetLastError();
}

hipError_t launch_sweep_upd(const DevProblem &P, const double *x, double *xo, double w, double tol,
                            UpdState *st, int64_t g, hipStream_t s)
{
    const dim3 grid((unsigned)((P.n0 + kGenericBlock - 1) / kGenericBlock), (unsigned)P.n1,
                    (unsigned)P.n2);
    switch (P.ndim) {
    case 1: hipLaunchKernelGGL(k_sweep_upd<1>, grid, dim3(kGenericBlock), 0, s, P, x, xo, w, tol, st, g); break;
    case 2: hipLaunchKernelGGL(k_sweep_upd<2>, grid, dim3(kGenericBlock), 0, s, P, x, xo, w, tol, st, g); break;
    default: hipLaunchKernelGGL(k_sweep_upd<3>, grid, dim3(kGenericBlock), 0, s, P, x, xo, w, tol, st, g); break;
    }
    return hipGetLastError();
}

hipError_t launch_sweep_generic(const DevProblem &P, const double *x, double *xo, double w,
                                hipStream_t s)
{
    const dim3 grid((unsigned)((P.n0 + kGenericBlock - 1) / kGenericBlock), (unsigned)P.n1,
                    (unsigned)P.n2);
    if (P.ell_len) {
        hipLaunchKernelGGL(k_sweep_ell, grid, dim3(kGenericBlock), 0, s, P, x, xo, w);
        return hipGetLastError();
    }
    switch (P.ndim) {
    case 1: hipLaunchKernelGGL(k_sweep_generic<1>, grid, dim3(kGenericBlock), 0, s, P, x, xo, w); break;
    case 2: hipLaunchKernelGGL(k_sweep_generic<2>, grid, dim3(kGenericBlock), 0, s, P, x, xo, w); break;
    default: hipLaunchKernelGGL(k_sweep_generic<3>, grid, dim3(kGenericBlock), 0, s, P, x, xo, w); break;
    }
    return hipGetLastError();
}

// One workgroup of 64 threads: lane k folds the stripes of sweep k of the
// launch that used `ring`; the first sweep below tol (in sweep order) sets
// flag and stop.  Then the slots of the other ring are cleared for the next
// launch.  Does nothing but the clearing once flag is set.
__global__ __launch_bounds__(64) void k_upd_check(UpdFState *st, int ring, int T, int64_t g0,
                                                  double tol, int64_t *pub)
{
    const int lane = threadIdx.x;
    if (!st->flag && T > 0) {
        bool below = false;
        if (lane < T) {
            unsigned long long m = 0ull;
            for (int j = 0; j < kUpdFStripes; ++j) {
                const unsigned long long v = st->maxbits[ring][lane][j * kUpdStride];
                m = v > m ? v : m;
            }
            below = __longlong_as_double((long long)m) < tol;
        }
        const unsigned long long mask = __ballot(below);
        if (mask && lane == 0) {
            st->flag = 1;
            st->stop = g0 + (__builtin_ctzll(mask));
        }
    }
    if (pub && lane == 0) {  // flag and stop for the host, in pinned memory
        pub[0] = st->flag;
        pub[1] = st->stop;
    }
    for (int i = lane; i < kUpdFMaxT * kUpdFStripes; i += 64)
        st->maxbits[ring ^ 1][i / kUpdFStripes][(i % kUpdFStripes) * kUpdStride] = 0ull;
}

hipError_t launch_upd_check(UpdFState *st, int ring, int T, int64_t g0, double tol, int64_t *pub,
                            hipStream_t s)
{
    if (!st || ring < 0 || ring > 1 || T < 0 || T > kUpdFMaxT) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_upd_check, dim3(1), dim3(64), 0, s, st, ring, T, g0, tol, pub);
    return hipGetLastError();
}

bool fused_upd_supported(const DevProblem &P, const SweepPlan &plan)
{
    return plan.kind == 10 && plan.T <= kUpdFMaxT && fused_supported(P, plan);
}

hipError_t launch_sweep_fused_upd(const DevProblem &P, const SweepPlan &plan, const double *x,
                                  double *xo, const double *w_dev, int T, UpdFState *st, int ring,
                                  hipStream_t s, bool reverse)
{
    if (plan.kind != 10) return hipErrorInvalidValue;
#define SRJ_GOF(HW, HL, NW)                                                                        \
    if (plan.by == HW && plan.occ == NW && plan.T <= HL)                                           \
        return launch_blockf2d<StF64, HW, HL, NW, true>(P.n0, P.n1, x, xo, P.b, P.face[0],         \
                                                        P.face[1], P.diag, P.dinv, w_dev, T, s,     \
                                                        reverse, st, ring);
    SRJ_BLOCKF_VARIANTS(SRJ_GOF)
#undef SRJ_GOF
    return hipErrorInvalidValue;
}

int plan_variants(int32_t *out, int cap)
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
    SRJ_BLOCK_VARIANTS(SRJ_LIST7)
#undef KIND
#define KIND 8
    SRJ_BLOCK2_VARIANTS(SRJ_LIST7)
#undef KIND
#define KIND 10
    SRJ_BLOCKF_VARIANTS(SRJ_LIST7)
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
    SRJ_PLANE2_VARIANTS(SRJ_LIST11)
#undef SRJ_LIST11
#define SRJ_LIST12(HH, ZZ)             \
    if (n < cap) {                     \
        out[4 * n + 0] = 12;           \
        out[4 * n + 1] = HH;           \
        out[4 * n + 2] = 2;            \
        out[4 * n + 3] = ZZ;           \
    }                                  \
    ++n;
    SRJ_PLANE2F_VARIANTS(SRJ_LIST12)
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
    for (const TileVariant &v : kVariants) {
        if (n < cap) {
            out[4 * n + 0] = v.blds ? 2 : 1;
            out[4 * n + 1] = v.rows;
            out[4 * n + 2] = v.halo;
            out[4 * n + 3] = v.occ;
        }
        ++n;
    }
    return n;
}

bool fused_supported(const DevProblem &P, const SweepPlan &plan)
{
    if (P.ell_len) return false;  // general sparse matrices: one sweep per launch
    if (plan.kind == 7 || plan.kind == 8) {
        if (!(P.ndim == 2 && !P.face[0] && !P.face[1] && !P.diag) || plan.T < 1) return false;
#define SRJ_CHK(HW, HL, NW) if (plan.by == HW && plan.occ == NW && plan.T <= HL) return true;
        if (plan.kind == 7) { SRJ_BLOCK_VARIANTS(SRJ_CHK) }
        else { SRJ_BLOCK2_VARIANTS(SRJ_CHK) }
#undef SRJ_CHK
        return false;
    }
    if (plan.kind == 10) {
        if (!(P.ndim == 2 && P.face[0] && P.face[1] && P.diag && P.dinv) || plan.T < 1) return false;
#define SRJ_CHK(HW, HL, NW) if (plan.by == HW && plan.occ == NW && plan.T <= HL) return true;
        SRJ_BLOCKF_VARIANTS(SRJ_CHK)
#undef SRJ_CHK
        return false;
    }
    if (plan.kind == 12) {
        if (!(P.ndim == 3 && P.face[0] && P.face[1] && P.face[2] && P.diag) || plan.T < 1 ||
            plan.T > 2)
            return false;
#define SRJ_CHK(HH, ZZ) if (plan.by == HH && plan.occ == ZZ) return true;
        SRJ_PLANE2F_VARIANTS(SRJ_CHK)
#undef SRJ_CHK
        return false;
    }
    if (plan.kind == 11) {
        if (!(P.ndim == 3 && !P.face[0] && !P.face[1] && !P.face[2] && !P.diag) || plan.T < 1 ||
            plan.T > 2)
            return false;
#define SRJ_CHK(HH, ZZ) if (plan.by == HH && plan.occ == ZZ) return true;
        SRJ_PLANE2_VARIANTS(SRJ_CHK)
#undef SRJ_CHK
        return false;
    }
    if (plan.kind == 6) {
        if (!plane3d_fits(P.ndim, P.face[0], P.face[1], P.face[2], P.diag) || plan.T != 1 ||
            plan.occ < 1)
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
    if (plan.kind == 1 || plan.kind == 2) {
        if (!(P.ndim == 2 && !P.face[0] && !P.face[1] && !P.diag && plan.T >= 1)) return false;
        for (const TileVariant &v : kVariants)
            if (v.rows == plan.by && v.blds == (plan.kind == 2) && plan.T <= v.halo &&
                v.occ == plan.occ)
                return true;
    }
    return false;
}

hipError_t launch_sweep_fused(const DevProblem &P, const SweepPlan &plan, const double *x,
                              double *xo, const double *w_dev, int T, hipStream_t s, bool reverse)
{
    if (plan.kind == 7 || plan.kind == 8) {
        const Coef2D<double> kb{P.dconst, P.dinvconst, P.c[0], P.c[1]};
#define SRJ_GO1(HW, HL, NW)                                                         \
    if (plan.by == HW && plan.occ == NW && plan.T <= HL)                            \
        return launch_block2d<StF64, HW, HL, NW, 1>(P.n0, P.n1, x, xo, P.b, w_dev, T, kb, s, reverse);
#define SRJ_GO2(HW, HL, NW)                                                         \
    if (plan.by == HW && plan.occ == NW && plan.T <= HL)                            \
        return launch_block2d<StF64, HW, HL, NW, 2>(P.n0, P.n1, x, xo, P.b, w_dev, T, kb, s, reverse);
        if (plan.kind == 7) { SRJ_BLOCK_VARIANTS(SRJ_GO1) }
        else { SRJ_BLOCK2_VARIANTS(SRJ_GO2) }
#undef SRJ_GO1
#undef SRJ_GO2
        return hipErrorInvalidValue;
    }
    if (plan.kind == 10) {
#define SRJ_GOF(HW, HL, NW)                                                                   \
    if (plan.by == HW && plan.occ == NW && plan.T <= HL)                                      \
        return launch_blockf2d<StF64, HW, HL, NW>(P.n0, P.n1, x, xo, P.b, P.face[0], P.face[1], \
                                                  P.diag, P.dinv, w_dev, T, s, reverse);
        SRJ_BLOCKF_VARIANTS(SRJ_GOF)
#undef SRJ_GOF
        return hipErrorInvalidValue;
    }
    if (plan.kind == 12) {
        const Stencil3<double> S{P.n0, P.n1, P.n2, {P.c[0], P.c[1], P.c[2]},
                                 {P.face[0], P.face[1], P.face[2]}, P.dconst, P.dinvconst,
                                 P.diag, P.dinv};
        // the last launch of an odd-length cycle does one sweep
        if (T == 1) return launch_plane3d<StF64, 4, 8>(S, x, xo, P.b, w_dev, s);
        if (T != 2) return hipErrorInvalidValue;
#define SRJ_GO(HH, ZZ) \
    if (plan.by == HH && plan.occ == ZZ) return launch_plane3d2f<StF64, HH, ZZ>(S, x, xo, P.b, w_dev, s);
        SRJ_PLANE2F_VARIANTS(SRJ_GO)
#undef SRJ_GO
        return hipErrorInvalidValue;
    }
    if (plan.kind == 11) {
        const Stencil3<double> S{P.n0, P.n1, P.n2, {P.c[0], P.c[1], P.c[2]},
                                 {nullptr, nullptr, nullptr}, P.dconst, P.dinvconst, nullptr,
                                 nullptr};
        // the last launch of an odd-length cycle does one sweep
        if (T == 1) return launch_plane3d<StF64, 4, 8>(S, x, xo, P.b, w_dev, s);
        if (T != 2) return hipErrorInvalidValue;
#define SRJ_GO(HH, ZZ) \
    if (plan.by == HH && plan.occ == ZZ) return launch_plane3d2<StF64, HH, ZZ>(S, x, xo, P.b, w_dev, s);
        SRJ_PLANE2_VARIANTS(SRJ_GO)
#undef SRJ_GO
        return hipErrorInvalidValue;
    }
    if (plan.kind == 6) {
        const Stencil3<double> S{P.n0, P.n1, P.n2, {P.c[0], P.c[1], P.c[2]},
                                 {P.face[0], P.face[1], P.face[2]}, P.dconst, P.dinvconst,
                                 P.diag, P.dinv};
#define SRJ_GO(HH, ZZ) \
    if (plan.by == HH && plan.occ == ZZ) return launch_plane3d<StF64, HH, ZZ>(S, x, xo, P.b, w_dev, s);
        SRJ_PLANE_VARIANTS(SRJ_GO)
#undef SRJ_GO
        return hipErrorInvalidValue;
    }
    if (plan.kind == 5) {
        const Coef2D<double> kw{P.dconst, P.dinvconst, P.c[0], P.c[1]};
#define SRJ_GO(OH, TM) \
    if (plan.by == OH && plan.T <= TM) return launch_wave2d<StF64, OH, TM>(T, P.n0, P.n1, x, xo, P.b, w_dev, kw, s);
        SRJ_WAVE_VARIANTS(SRJ_GO)
#undef SRJ_GO
        return hipErrorInvalidValue;
    }
    if (plan.kind == 3) {
        const Stencil3<double> S{P.n0, P.n1, P.n2, {P.c[0], P.c[1], P.c[2]},
                                 {P.face[0], P.face[1], P.face[2]}, P.dconst, P.dinvconst,
                                 P.diag, P.dinv};
#define SRJ_GO(Z) if (plan.by == Z) return launch_stream3d<StF64, Z>(S, x, xo, P.b, w_dev, s);
        SRJ_3D_CHUNKS(SRJ_GO)
#undef SRJ_GO
        return hipErrorInvalidValue;
    }
    const bool blds = plan.kind == 2;
    const Coef2D<double> k2{P.dconst, P.dinvconst, P.c[0], P.c[1]};
#define SRJ_TRY(R, HL, BL, OC)                                                             \
    if (plan.by == R && blds == BL && plan.T <= HL && plan.occ == OC)                      \
        return launch_tile2d<StF64, R, HL, BL, OC>(P.n0, P.n1, x, xo, P.b, w_dev, T, k2, s);
    SRJ_2D_VARIANTS(SRJ_TRY)
#undef SRJ_TRY
    return hipErrorInvalidValue;
}

}  // namespace srj
