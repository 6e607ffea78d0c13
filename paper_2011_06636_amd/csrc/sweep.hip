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

__global__ void k_dinv(const double *__restrict__ d, double *__restrict__ dinv, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dinv[i] = 1.0 / d[i];
}

// ---------------------------------------------------------------------------
// 2D register-tiled kernel, constant coefficients, T <= HALO sweeps fused.
//
// Each wave owns a tile of 64 columns x H rows of the grid (halo included):
// lane = column, the H rows of its column live in registers.  Vertical
// neighbours are the lane's own registers; horizontal neighbours come from
// the adjacent lanes through DPP wave shifts (full-rate VALU moves).  After
// sweep k the outermost k columns/rows of the tile hold stale values, so the
// (64 - 2 HALO) x (H - 2 HALO) centre is exact after up to HALO sweeps and is
// written back.  Points outside the grid (the Dirichlet ghosts) hold zero
// and are never updated.  Tiles that lie wholly inside the grid take a path
// without any masking.  b stays in registers (BLDS = false) or in LDS
// (BLDS = true, fewer registers, more waves per SIMD).  No barriers: waves
// are independent.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double lane_prev(double v)  // value of lane - 1 (lane 0: 0)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x138, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x138, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double lane_next(double v)  // value of lane + 1 (lane 63: 0)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x130, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x130, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}

template <int H, bool MASK, bool BLDS>
__device__ __forceinline__ void tile_sweeps(double (&xr)[H], const double (&br)[H],
                                            const double *__restrict__ bl, bool col_in,
                                            uint64_t rowbits, const double *__restrict__ wlist,
                                            int T, double D, double Dinv, double c0, double c1)
{
    for (int k = 0; k < T; ++k) {
        const double w = wlist[k];
        double up = 0.0;  // old value of the row above (zero above the tile)
#pragma unroll
        for (int r = 0; r < H; ++r) {
            const double xc = xr[r];
            const double xl = lane_prev(xc);
            const double xh = lane_next(xc);
            const double dn = (r + 1 < H) ? xr[r + 1] : 0.0;
            double s = D * xc;
            s = s - c0 * xl;
            s = s - c0 * xh;
            s = s - c1 * up;
            s = s - c1 * dn;
            const double bv = BLDS ? bl[r * 64] : br[r];
            const double rr = bv - s;
            const double t = Dinv * rr;
            const double nx = xc + w * t;
            up = xc;
            if (MASK)
                xr[r] = (col_in && ((rowbits >> r) & 1)) ? nx : 0.0;
            else
                xr[r] = nx;
        }
    }
}

template <int H, int HALO, bool BLDS, int WPB, int OCC>
__global__ __launch_bounds__(64 * WPB) __attribute__((amdgpu_waves_per_eu(OCC, 8))) void k_sweep2d_reg(DevProblem P, const double *__restrict__ x,
                                                     double *__restrict__ xo,
                                                     const double *__restrict__ wlist, int T,
                                                     int tiles_x, int tiles_y)
{
    constexpr int OW = 64 - 2 * HALO;  // output columns per tile
    constexpr int OH = H - 2 * HALO;   // output rows per tile
    static_assert(H <= 64, "row validity is a 64-bit mask");
    __shared__ double bsh[BLDS ? WPB * H * 64 : 1];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int tile = blockIdx.x * WPB + wave;
    if (tile >= tiles_x * tiles_y) return;  // whole wave leaves
    const int tx = tile % tiles_x, ty = tile / tiles_x;
    const int64_t n0 = P.n0, n1 = P.n1;
    const int64_t gx0 = (int64_t)tx * OW - HALO;
    const int64_t gy0 = (int64_t)ty * OH - HALO;
    const int64_t gx = gx0 + lane;
    const bool col_in = gx >= 0 && gx < n0;
    const bool interior = gx0 >= 0 && gx0 + 64 <= n0 && gy0 >= 0 && gy0 + H <= n1;
    uint64_t rowbits = 0;
#pragma unroll
    for (int r = 0; r < H; ++r)
        if (gy0 + r >= 0 && gy0 + r < n1) rowbits |= (uint64_t)1 << r;
    const double D = P.dconst, Dinv = P.dinvconst, c0 = P.c[0], c1 = P.c[1];

    double xr[H], br[H];
    double *bl = bsh + (BLDS ? wave * H * 64 + lane : 0);
#pragma unroll
    for (int r = 0; r < H; ++r) {
        const bool in = col_in && ((rowbits >> r) & 1);
        const int64_t p = (gy0 + r) * n0 + gx;
        xr[r] = in ? x[p] : 0.0;
        const double bv = in ? P.b[p] : 0.0;
        if (BLDS)
            bl[r * 64] = bv;
        else
            br[r] = bv;
    }
    if (interior)
        tile_sweeps<H, false, BLDS>(xr, br, bl, col_in, rowbits, wlist, T, D, Dinv, c0, c1);
    else
        tile_sweeps<H, true, BLDS>(xr, br, bl, col_in, rowbits, wlist, T, D, Dinv, c0, c1);
    if (lane >= HALO && lane < 64 - HALO && col_in) {
#pragma unroll
        for (int r = HALO; r < H - HALO; ++r) {
            if ((rowbits >> r) & 1) xo[(gy0 + r) * n0 + gx] = xr[r];
        }
    }
}

template <int H, int HALO, bool BLDS, int OCC>
hipError_t launch_2d_reg(const DevProblem &P, const double *x, double *xo, const double *w_dev,
                         int T, hipStream_t s)
{
    // b in LDS: one wave per block keeps the block's LDS at H * 512 bytes
    constexpr int WPB = BLDS ? 1 : 4;
    constexpr int OW = 64 - 2 * HALO, OH = H - 2 * HALO;
    const int tiles_x = (int)((P.n0 + OW - 1) / OW);
    const int tiles_y = (int)((P.n1 + OH - 1) / OH);
    const int64_t tiles = (int64_t)tiles_x * tiles_y;
    const int blocks = (int)((tiles + WPB - 1) / WPB);
    hipLaunchKernelGGL((k_sweep2d_reg<H, HALO, BLDS, WPB, OCC>), dim3(blocks), dim3(64 * WPB), 0, s, P,
                       x, xo, w_dev, T, tiles_x, tiles_y);
    return hipGetLastError();
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

hipError_t launch_sweep_generic(const DevProblem &P, const double *x, double *xo, double w,
                                hipStream_t s)
{
    const dim3 grid((unsigned)((P.n0 + kGenericBlock - 1) / kGenericBlock), (unsigned)P.n1,
                    (unsigned)P.n2);
    switch (P.ndim) {
    case 1: hipLaunchKernelGGL(k_sweep_generic<1>, grid, dim3(kGenericBlock), 0, s, P, x, xo, w); break;
    case 2: hipLaunchKernelGGL(k_sweep_generic<2>, grid, dim3(kGenericBlock), 0, s, P, x, xo, w); break;
    default: hipLaunchKernelGGL(k_sweep_generic<3>, grid, dim3(kGenericBlock), 0, s, P, x, xo, w); break;
    }
    return hipGetLastError();
}

int plan_variants(int32_t *out, int cap)
{
    int n = 0;
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
                              double *xo, const double *w_dev, int T, hipStream_t s)
{
    // the first variant (smallest halo) that covers the plan's sweeps per launch
    const bool blds = plan.kind == 2;
#define SRJ_TRY(R, HL, BL, OC)                                                             \
    if (plan.by == R && blds == BL && plan.T <= HL && plan.occ == OC)                      \
        return launch_2d_reg<R, HL, BL, OC>(P, x, xo, w_dev, T, s);
    SRJ_2D_VARIANTS(SRJ_TRY)
#undef SRJ_TRY
    return hipErrorInvalidValue;
}

}  // namespace srj
