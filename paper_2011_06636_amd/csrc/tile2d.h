// 2D register-tiled relaxed Jacobi sweeps, templated on the value policy.
//
// One sweep of Islam & Wang (arXiv 2011.06636) section 2, Eq. 3 in residual
// form, constant coefficients:
//     s = D u_p - c0 u_{p-e0} - c0 u_{p+e0} - c1 u_{p-e1} - c1 u_{p+e1}
//     u'_p = u_p + w (Dinv (f_p - s))
// evaluated in exactly this order without fused multiply-add, so any tile
// shape and any number of sweeps per launch produce the same bits as the
// one-sweep kernels.
//
// Each wave owns a tile of 64 columns x H rows of the grid (halo included):
// lane = column, the H rows of its column live in registers.  Vertical
// neighbours are the lane's own registers; horizontal ones come from the
// adjacent lanes through DPP wave shifts.  After sweep k the outermost k
// columns/rows hold stale values, so the (64 - 2 HALO) x (H - 2 HALO) centre
// is exact after up to HALO sweeps and is written back.  Points outside the
// grid (the Dirichlet ghosts) hold zero and are never updated; tiles wholly
// inside the grid skip all masking.  The right-hand side stays in registers
// (BLDS = false) or in LDS (BLDS = true).  Waves are independent: no
// barriers.
//
// Value policy V: V::A is the arithmetic type, V::T the storage type;
// V::load(T) -> A, V::store(A) -> T, and V::round(A) applies the storage
// rounding that every sweep ends with (identity when T == A).
#pragma once

#include "internal.h"

#pragma clang fp contract(off)

namespace srj {

// Whole-wave shifts by one lane (DPP wave_shr / wave_shl).  With bound_ctrl
// set, the lane without a source (0 for prev, 63 for next) reads zero, so no
// initialising move is needed.
__device__ __forceinline__ float dpp_prev(float v)  // lane - 1 (lane 0 gets 0)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xf, 0xf, true));
}
__device__ __forceinline__ float dpp_next(float v)  // lane + 1 (lane 63 gets 0)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xf, 0xf, true));
}
__device__ __forceinline__ double dpp_prev(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x138, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x138, 0xf, 0xf, true);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double dpp_next(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x130, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x130, 0xf, 0xf, true);
    return __hiloint2double(hi, lo);
}

template <class A>
struct Coef2D {
    A D, Dinv, c0, c1;
};

// T sweeps over the tile in registers.  Products are formed once per point
// and moved, not recomputed: c0 * u_{p-e0} is lane p-1's c0 * u, shifted one
// lane, and c1 * u of a row serves the rows above and below it.  A product
// does not depend on the lane that forms it, so the result is the same as
// forming each term in place.  The lanes and rows where a shift or the tile
// edge supplies a zero are halo and are never written back.
template <class V, int H, bool MASK, bool BLDS>
__device__ __forceinline__ void tile_sweeps(typename V::A (&xr)[H], const typename V::A (&br)[H],
                                            const typename V::A *__restrict__ bl, bool col_in,
                                            uint64_t rowbits, const typename V::A *__restrict__ wlist,
                                            int T, Coef2D<typename V::A> k2)
{
    using A = typename V::A;
    for (int k = 0; k < T; ++k) {
        const A w = wlist[k];
        A c1up = k2.c1 * A(0);    // c1 * old row above (zero above the tile)
        A c1cur = k2.c1 * xr[0];  // c1 * old row r
#pragma unroll
        for (int r = 0; r < H; ++r) {
            const A xc = xr[r];
            const A c1dn = k2.c1 * ((r + 1 < H) ? xr[r + 1] : A(0));
            const A p0 = k2.c0 * xc;
            A s = k2.D * xc;
            s = s - dpp_prev(p0);
            s = s - dpp_next(p0);
            s = s - c1up;
            s = s - c1dn;
            const A bv = BLDS ? bl[r * 64] : br[r];
            const A rr = bv - s;
            const A t = k2.Dinv * rr;
            const A nx = V::round(xc + w * t);
            c1up = c1cur;
            c1cur = c1dn;
            if (MASK)
                xr[r] = (col_in && ((rowbits >> r) & 1)) ? nx : A(0);
            else
                xr[r] = nx;
        }
    }
}

// Body of one wave's tile (tile column tx, tile row ty); bl is this lane's
// slot in LDS when BLDS, else unused.
template <class V, int H, int HALO, bool BLDS>
__device__ __forceinline__ void tile2d_run(int64_t n0, int64_t n1, const typename V::T *__restrict__ x,
                                           typename V::T *__restrict__ xo,
                                           const typename V::T *__restrict__ b,
                                           const typename V::A *__restrict__ wlist, int T,
                                           Coef2D<typename V::A> k2, int tx, int ty, int lane,
                                           typename V::A *bl)
{
    using A = typename V::A;
    constexpr int OW = 64 - 2 * HALO;  // output columns per tile
    constexpr int OH = H - 2 * HALO;   // output rows per tile
    static_assert(H <= 64, "row validity is a 64-bit mask");
    const int64_t gx0 = (int64_t)tx * OW - HALO;
    const int64_t gy0 = (int64_t)ty * OH - HALO;
    const int64_t gx = gx0 + lane;
    const bool interior = gx0 >= 0 && gx0 + 64 <= n0 && gy0 >= 0 && gy0 + H <= n1;
    A xr[H], br[H];
    const int64_t p0 = gy0 * n0 + gx;
    if (interior) {
        // every row and column is in the grid: one base address, row strides
#pragma unroll
        for (int r = 0; r < H; ++r) {
            xr[r] = V::load(x[p0 + r * n0]);
            const A bv = V::load(b[p0 + r * n0]);
            if (BLDS)
                bl[r * 64] = bv;
            else
                br[r] = bv;
        }
        tile_sweeps<V, H, false, BLDS>(xr, br, bl, true, ~(uint64_t)0, wlist, T, k2);
        if (lane >= HALO && lane < 64 - HALO) {
#pragma unroll
            for (int r = HALO; r < H - HALO; ++r) xo[p0 + r * n0] = V::store(xr[r]);
        }
        return;
    }
    const bool col_in = gx >= 0 && gx < n0;
    uint64_t rowbits = 0;
#pragma unroll
    for (int r = 0; r < H; ++r)
        if (gy0 + r >= 0 && gy0 + r < n1) rowbits |= (uint64_t)1 << r;
#pragma unroll
    for (int r = 0; r < H; ++r) {
        const bool in = col_in && ((rowbits >> r) & 1);
        const int64_t p = (gy0 + r) * n0 + gx;
        xr[r] = in ? V::load(x[p]) : A(0);
        const A bv = in ? V::load(b[p]) : A(0);
        if (BLDS)
            bl[r * 64] = bv;
        else
            br[r] = bv;
    }
    tile_sweeps<V, H, true, BLDS>(xr, br, bl, col_in, rowbits, wlist, T, k2);
    if (lane >= HALO && lane < 64 - HALO && col_in) {
#pragma unroll
        for (int r = HALO; r < H - HALO; ++r) {
            if ((rowbits >> r) & 1) xo[(gy0 + r) * n0 + gx] = V::store(xr[r]);
        }
    }
}

template <class V, int H, int HALO, bool BLDS, int WPB, int OCC>
__global__ __launch_bounds__(64 * WPB) __attribute__((amdgpu_waves_per_eu(OCC, 8))) void
k_tile2d(int64_t n0, int64_t n1, const typename V::T *__restrict__ x, typename V::T *__restrict__ xo,
         const typename V::T *__restrict__ b, const typename V::A *__restrict__ wlist, int T,
         Coef2D<typename V::A> k2, int tiles_x, int tiles_y, int nblocks)
{
    using A = typename V::A;
    __shared__ A bsh[BLDS ? WPB * H * 64 : 1];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    // XCD-aware order: hardware places block i on XCD i % 8; each XCD takes a
    // contiguous range of logical blocks, so tiles that share halo rows and
    // columns are fetched through the same L2.
    const int per_xcd = (nblocks + 7) / 8;
    const int logical = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
    const int tile = logical * WPB + wave;
    if (logical >= nblocks || tile >= tiles_x * tiles_y) return;  // whole wave leaves
    A *bl = bsh + (BLDS ? wave * H * 64 + lane : 0);
    tile2d_run<V, H, HALO, BLDS>(n0, n1, x, xo, b, wlist, T, k2, tile % tiles_x, tile / tiles_x,
                                 lane, bl);
}

template <class V, int H, int HALO, bool BLDS, int OCC>
hipError_t launch_tile2d(int64_t n0, int64_t n1, const typename V::T *x, typename V::T *xo,
                         const typename V::T *b, const typename V::A *w_dev, int T,
                         Coef2D<typename V::A> k2, hipStream_t s)
{
    // b in LDS: one wave per block keeps the block's LDS at H * 64 values
    constexpr int WPB = BLDS ? 1 : 4;
    constexpr int OW = 64 - 2 * HALO, OH = H - 2 * HALO;
    const int tiles_x = (int)((n0 + OW - 1) / OW);
    const int tiles_y = (int)((n1 + OH - 1) / OH);
    const int64_t tiles = (int64_t)tiles_x * tiles_y;
    const int blocks = (int)((tiles + WPB - 1) / WPB);
    // a multiple of 8 blocks, so the XCD mapping covers every logical block
    const int grid = (blocks + 7) / 8 * 8;
    hipLaunchKernelGGL((k_tile2d<V, H, HALO, BLDS, WPB, OCC>), dim3(grid), dim3(64 * WPB), 0, s,
                       n0, n1, x, xo, b, w_dev, T, k2, tiles_x, tiles_y, blocks);
    return hipGetLastError();
}

}  // namespace srj
