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
// the adjacent lanes through cross-lane moves.  After sweep k the outermost
// k columns/rows of the tile hold stale values, so the (64 - 2 HALO) x
// (H - 2 HALO) centre is exact after up to HALO sweeps and is written back.
// Points outside the grid (the Dirichlet ghosts) hold zero and are never
// updated.  No LDS and no barriers: waves are independent.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double lane_prev(double v)  // value of lane - 1
{
    return __shfl_up(v, 1, 64);
}
__device__ __forceinline__ double lane_next(double v)  // value of lane + 1
{
    return __shfl_down(v, 1, 64);
}

template <int H, int HALO>
__global__ __launch_bounds__(256) void k_sweep2d_reg(DevProblem P, const double *__restrict__ x,
                                                     double *__restrict__ xo,
                                                     const double *__restrict__ wlist, int T,
                                                     int tiles_x, int tiles_y)
{
    constexpr int OW = 64 - 2 * HALO;  // output columns per tile
    constexpr int OH = H - 2 * HALO;   // output rows per tile
    const int lane = threadIdx.x & 63;
    const int tile = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (tile >= tiles_x * tiles_y) return;  // whole wave leaves
    const int tx = tile % tiles_x, ty = tile / tiles_x;
    const int64_t n0 = P.n0, n1 = P.n1;
    const int64_t gx = (int64_t)tx * OW - HALO + lane;
    const int64_t gy0 = (int64_t)ty * OH - HALO;
    const bool col_in = gx >= 0 && gx < n0;
    const double D = P.dconst, Dinv = P.dinvconst, c0 = P.c[0], c1 = P.c[1];

    double xr[H], br[H];
    bool in[H];
#pragma unroll
    for (int r = 0; r < H; ++r) {
        const int64_t gy = gy0 + r;
        in[r] = col_in && gy >= 0 && gy < n1;
        const int64_t p = gy * n0 + gx;
        xr[r] = in[r] ? x[p] : 0.0;
        br[r] = in[r] ? P.b[p] : 0.0;
    }
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
            const double rr = br[r] - s;
            const double t = Dinv * rr;
            const double nx = xc + w * t;
            up = xc;
            xr[r] = in[r] ? nx : 0.0;
        }
    }
    if (lane >= HALO && lane < 64 - HALO) {
#pragma unroll
        for (int r = HALO; r < H - HALO; ++r) {
            if (in[r]) xo[(gy0 + r) * n0 + gx] = xr[r];
        }
    }
}

template <int H, int HALO>
hipError_t launch_2d_reg(const DevProblem &P, const double *x, double *xo, const double *w_dev,
                         int T, hipStream_t s)
{
    constexpr int OW = 64 - 2 * HALO, OH = H - 2 * HALO;
    const int tiles_x = (int)((P.n0 + OW - 1) / OW);
    const int tiles_y = (int)((P.n1 + OH - 1) / OH);
    const int64_t tiles = (int64_t)tiles_x * tiles_y;
    const int blocks = (int)((tiles + 3) / 4);
    hipLaunchKernelGGL((k_sweep2d_reg<H, HALO>), dim3(blocks), dim3(256), 0, s, P, x, xo, w_dev,
                       T, tiles_x, tiles_y);
    return hipGetLastError();
}

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

bool fused_supported(const DevProblem &P, const SweepPlan &plan)
{
    if (plan.kind == 1) {
        return P.ndim == 2 && !P.face[0] && !P.face[1] && !P.diag && plan.T >= 1 &&
               ((plan.by == 32 && plan.T <= 4) || (plan.by == 48 && plan.T <= 6) ||
                (plan.by == 64 && plan.T <= 8));
    }
    return false;
}

hipError_t launch_sweep_fused(const DevProblem &P, const SweepPlan &plan, const double *x,
                              double *xo, const double *w_dev, int T, hipStream_t s)
{
    if (plan.kind == 1) {
        if (plan.by == 32) return launch_2d_reg<32, 4>(P, x, xo, w_dev, T, s);
        if (plan.by == 48) return launch_2d_reg<48, 6>(P, x, xo, w_dev, T, s);
        return launch_2d_reg<64, 8>(P, x, xo, w_dev, T, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace srj
