// 2D relaxed Jacobi sweeps fused over blocks of cooperating waves.
//
// Same per-point expression as every other kernel (Islam & Wang, arXiv
// 2011.06636, section 2, Eq. 3 in residual form, no fused multiply-add), so
// results are bit-identical.
//
// A workgroup of NW waves owns a block of 64 C columns x NW HW rows, halo
// included: lane l holds the C adjacent columns l C .. l C + C - 1, and wave w
// holds rows w HW .. w HW + HW - 1 of the block, all in registers.  Horizontal
// neighbours inside a lane are its own registers and across lanes come from
// DPP wave shifts (one shift per direction for C columns); vertical
// neighbours are registers too, except the rows just above and below a
// wave's rows, which belong to the neighbouring waves: every wave publishes
// its first and last rows in LDS before each sweep (double-buffered, one
// barrier per sweep).  The halo is paid once per block instead of once per
// wave: after T sweeps the outer T rows and columns of the block are stale,
// and the (64 C - 2 HALO) x (NW HW - 2 HALO) centre is exact for T <= HALO.
// Ghost points (outside the grid) hold zero and are never updated.  Blocks
// are mapped so that consecutive blocks of a block row land on the same XCD.
#pragma once

#include "internal.h"
#include "tile2d.h"

#pragma clang fp contract(off)

namespace srj {

template <class T, int C>
struct alignas(C * sizeof(T)) BlockVec {
    T v[C];
};

// T sweeps of one wave's rows.  edge: [2 buffers][2: first row, last row][NW][C][64];
// sweep k uses buffer (kbase + k) & 1, so consecutive sweeps alternate
// buffers also across the blocks of a persistent workgroup.
template <class V, int HW, int NW, int C, bool MASK>
__device__ __forceinline__ void block_sweeps(typename V::A (&xr)[HW][C],
                                             const typename V::A (&br)[HW][C],
                                             const bool (&col_in)[C], uint32_t rowbits,
                                             const typename V::A *__restrict__ wlist, int T,
                                             Coef2D<typename V::A> k2, typename V::A *edge,
                                             int wave, int lane, int kbase)
{
    using A = typename V::A;
    for (int k = 0; k < T; ++k) {
        // the sweep's factor is requested before the barrier, so its load
        // completes while the wave waits there
        const A w = wlist[k];
        A *e = edge + ((kbase + k) & 1) * (2 * NW * C * 64);
#pragma unroll
        for (int c = 0; c < C; ++c) {
            e[(wave * C + c) * 64 + lane] = xr[0][c];
            e[((NW + wave) * C + c) * 64 + lane] = xr[HW - 1][c];
        }
        __syncthreads();
        // rows outside the block read zero (they only feed halo rows)
        A upv[C], dnv[C];
#pragma unroll
        for (int c = 0; c < C; ++c) {
            upv[c] = wave > 0 ? e[((NW + wave - 1) * C + c) * 64 + lane] : A(0);
            dnv[c] = wave + 1 < NW ? e[((wave + 1) * C + c) * 64 + lane] : A(0);
        }
        // products are formed once and moved: c0 u of a column serves the
        // columns on both sides (in the lane, or one lane over by a shift),
        // and c1 u of a row serves the rows on both sides
        A c1up[C], c1cur[C];
#pragma unroll
        for (int c = 0; c < C; ++c) {
            c1up[c] = k2.c1 * upv[c];
            c1cur[c] = k2.c1 * xr[0][c];
        }
#pragma unroll
        for (int r = 0; r < HW; ++r) {
            A p[C], c1dn[C];
#pragma unroll
            for (int c = 0; c < C; ++c) {
                p[c] = k2.c0 * xr[r][c];
                c1dn[c] = k2.c1 * ((r + 1 < HW) ? xr[r + 1][c] : dnv[c]);
            }
            const A pl = dpp_prev(p[C - 1]);  // c0 u of the column left of this lane
            const A ph = dpp_next(p[0]);      // c0 u of the column right of this lane
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const A xc = xr[r][c];
                A s = k2.D * xc;
                s = s - (c > 0 ? p[c > 0 ? c - 1 : 0] : pl);
                s = s - (c + 1 < C ? p[c + 1 < C ? c + 1 : 0] : ph);
                s = s - c1up[c];
                s = s - c1dn[c];
                const A rr = br[r][c] - s;
                const A t = k2.Dinv * rr;
                const A nx = V::round(xc + w * t);
                c1up[c] = c1cur[c];
                c1cur[c] = c1dn[c];
                if (MASK)
                    xr[r][c] = (col_in[c] && ((rowbits >> r) & 1)) ? nx : A(0);
                else
                    xr[r][c] = nx;
            }
        }
    }
}

// Block geometry: BW x BH values per block, halo included, of which the
// centre OW x OH is written.
template <int HW, int HALO, int NW, int C>
struct BlockShape {
    static constexpr int BW = 64 * C;
    static constexpr int OW = BW - 2 * HALO;
    static constexpr int BH = NW * HW;
    static constexpr int OH = BH - 2 * HALO;
    static_assert(HW <= 32, "row validity is a 32-bit mask");
    static_assert(OH > 0 && OW > 0, "halo larger than the block");
    static_assert(HALO % C == 0, "lane columns must stay aligned");
};

// One wave's part of one block: load, T sweeps, store.  Row starts are
// wave-uniform and each lane adds its 32-bit column offset.  EDGE blocks
// cross the grid's edge: rows outside it read a valid row (a wave-uniform
// clamp) and lanes outside it read column 0, so every load stays in bounds
// and needs no branch, and a select then makes every value outside the grid
// zero; such values stay zero and are not written.  Written this way the
// boundary path needs no more registers than the interior one.  kbase continues the LDS buffer parity of the
// workgroup's previous sweeps (0 for a fresh workgroup).
template <class V, int HW, int HALO, int NW, int C, bool EDGE>
__device__ __forceinline__ void block2d_run(int64_t n0, int64_t n1,
                                            const typename V::T *__restrict__ x,
                                            typename V::T *__restrict__ xo,
                                            const typename V::T *__restrict__ b,
                                            const typename V::A *__restrict__ wlist, int T,
                                            Coef2D<typename V::A> k2, int64_t bx0, int64_t by0,
                                            bool vec, int wv, int lane, typename V::A *edge,
                                            int kbase)
{
    using A = typename V::A;
    using ST = typename V::T;
    using VT = BlockVec<ST, C>;
    using S = BlockShape<HW, HALO, NW, C>;
    const int64_t gy0 = by0 + (int64_t)wv * HW;
    // with C-wide vectors n0 is a multiple of C and so is bx0 + lane C: the C
    // columns of a lane are inside or outside the grid together
    bool col_in[C];
    uint32_t off[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const int64_t gx = bx0 + (int64_t)lane * C + c;
        col_in[c] = !EDGE || (gx >= 0 && gx < n0);
        off[c] = col_in[c] ? (uint32_t)gx : 0u;
    }
    uint32_t rowbits = ~0u;
    if (EDGE) {
        rowbits = 0;
#pragma unroll
        for (int r = 0; r < HW; ++r)
            if (gy0 + r >= 0 && gy0 + r < n1) rowbits |= 1u << r;
    }
    auto row_of = [&](int r) -> int64_t {  // a row inside the grid
        const int64_t gy = gy0 + r;
        return EDGE ? (gy < 0 ? 0 : (gy >= n1 ? n1 - 1 : gy)) : gy;
    };
    A xr[HW][C], br[HW][C];
#pragma unroll
    for (int r = 0; r < HW; ++r) {
        const ST *xrow = x + row_of(r) * n0;
        const ST *brow = b + row_of(r) * n0;
        const bool rin = (rowbits >> r) & 1;
        if (C > 1 && vec) {
            const VT qx = *reinterpret_cast<const VT *>(xrow + off[0]);
            const VT qb = *reinterpret_cast<const VT *>(brow + off[0]);
#pragma unroll
            for (int c = 0; c < C; ++c) {
                xr[r][c] = (!EDGE || (rin && col_in[c])) ? V::load(qx.v[c]) : A(0);
                br[r][c] = (!EDGE || (rin && col_in[c])) ? V::load(qb.v[c]) : A(0);
            }
        } else {
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const ST vx = xrow[off[c]], vb = brow[off[c]];
                xr[r][c] = (!EDGE || (rin && col_in[c])) ? V::load(vx) : A(0);
                br[r][c] = (!EDGE || (rin && col_in[c])) ? V::load(vb) : A(0);
            }
        }
    }
    block_sweeps<V, HW, NW, C, EDGE>(xr, br, col_in, rowbits, wlist, T, k2, edge, wv, lane, kbase);
    if (!(lane * C >= HALO && lane * C < S::BW - HALO)) return;
    const int rlo = HALO - wv * HW, rhi = S::BH - HALO - wv * HW;
#pragma unroll
    for (int r = 0; r < HW; ++r) {
        if (r < rlo || r >= rhi || !((rowbits >> r) & 1)) continue;
        ST *orow = xo + row_of(r) * n0;
        if (C > 1 && vec) {
            if (col_in[0]) {
                VT v;
#pragma unroll
                for (int c = 0; c < C; ++c) v.v[c] = V::store(xr[r][c]);
                *reinterpret_cast<VT *>(orow + off[0]) = v;
            }
        } else {
#pragma unroll
            for (int c = 0; c < C; ++c)
                if (col_in[c]) orow[off[c]] = V::store(xr[r][c]);
        }
    }
}

// One block (bx, by): interior blocks take the path without masks.
template <class V, int HW, int HALO, int NW, int C>
__device__ __forceinline__ void block2d_item(int64_t n0, int64_t n1,
                                             const typename V::T *__restrict__ x,
                                             typename V::T *__restrict__ xo,
                                             const typename V::T *__restrict__ b,
                                             const typename V::A *__restrict__ wlist, int T,
                                             Coef2D<typename V::A> k2, int bx, int by, bool vec,
                                             int wave, int lane, typename V::A *edge, int kbase)
{
    using S = BlockShape<HW, HALO, NW, C>;
    const int64_t bx0 = (int64_t)bx * S::OW - HALO;
    const int64_t by0 = (int64_t)by * S::OH - HALO;
    const int wv = __builtin_amdgcn_readfirstlane(wave);
    if (bx0 >= 0 && bx0 + S::BW <= n0 && by0 >= 0 && by0 + S::BH <= n1)
        block2d_run<V, HW, HALO, NW, C, false>(n0, n1, x, xo, b, wlist, T, k2, bx0, by0, vec, wv,
                                               lane, edge, kbase);
    else
        block2d_run<V, HW, HALO, NW, C, true>(n0, n1, x, xo, b, wlist, T, k2, bx0, by0, vec, wv,
                                              lane, edge, kbase);
}

// One block per workgroup.
template <class V, int HW, int HALO, int NW, int C>
__global__ __launch_bounds__(64 * NW) void k_block2d(int64_t n0, int64_t n1,
                                                     const typename V::T *__restrict__ x,
                                                     typename V::T *__restrict__ xo,
                                                     const typename V::T *__restrict__ b,
                                                     const typename V::A *__restrict__ wlist, int T,
                                                     Coef2D<typename V::A> k2, int blocks_x,
                                                     int nblocks, int vec, int reverse)
{
    using A = typename V::A;
    __shared__ A edge[2 * 2 * NW * C * 64];
    // XCD-aware order: hardware places block i on XCD i % 8; each XCD takes a
    // contiguous range of logical blocks so neighbouring blocks share its L2.
    // Every other launch walks each range backwards, so a launch starts with
    // the blocks the previous one finished last, whose data its L2 still holds.
    const int per_xcd = (nblocks + 7) / 8;
    const int j = blockIdx.x / 8;
    const int logical = (blockIdx.x % 8) * per_xcd + (reverse ? per_xcd - 1 - j : j);
    if (logical >= nblocks) return;  // whole block leaves
    block2d_item<V, HW, HALO, NW, C>(n0, n1, x, xo, b, wlist, T, k2, logical % blocks_x,
                                     logical / blocks_x, vec != 0, threadIdx.x >> 6,
                                     threadIdx.x & 63, edge, 0);
}

// reverse: walk each XCD's range of blocks backwards (callers alternate it
// from launch to launch; the result does not depend on it).
template <class V, int HW, int HALO, int NW, int C>
hipError_t launch_block2d(int64_t n0, int64_t n1, const typename V::T *x, typename V::T *xo,
                          const typename V::T *b, const typename V::A *w_dev, int T,
                          Coef2D<typename V::A> k2, hipStream_t s, bool reverse = false)
{
    constexpr int OW = BlockShape<HW, HALO, NW, C>::OW, OH = BlockShape<HW, HALO, NW, C>::OH;
    if (T < 1 || T > HALO) return hipErrorInvalidValue;
    if (n0 > INT32_MAX) return hipErrorInvalidValue;  // column offsets are 32-bit
    const int64_t bxn = (n0 + OW - 1) / OW, byn = (n1 + OH - 1) / OH;
    const int64_t nblocks = bxn * byn;
    if (nblocks > (int64_t)1 << 28) return hipErrorInvalidValue;
    // C-wide vector accesses need every row start and every pointer aligned
    // to C values (the block origins are, since OW and HALO are multiples of C)
    const uintptr_t al = (uintptr_t)C * sizeof(typename V::T);
    const int vec = C > 1 && n0 % C == 0 && (uintptr_t)x % al == 0 && (uintptr_t)xo % al == 0 &&
                    (uintptr_t)b % al == 0;
    // a multiple of 8 blocks, so the XCD mapping covers every logical block
    const int grid = (int)((nblocks + 7) / 8 * 8);
    hipLaunchKernelGGL((k_block2d<V, HW, HALO, NW, C>), dim3(grid), dim3(64 * NW), 0, s, n0, n1,
                       x, xo, b, w_dev, T, k2, (int)bxn, (int)nblocks, vec, reverse ? 1 : 0);
    return hipGetLastError();
}

// (rows per wave, halo = most sweeps per launch, waves per block) of the
// binary64 block plans: one column per lane (kind 7) and two (kind 8)
#define SRJ_BLOCK_VARIANTS(X) X(8, 4, 8) X(8, 6, 8) X(8, 8, 8) X(12, 8, 8) X(16, 6, 4) X(16, 8, 4)
#define SRJ_BLOCK2_VARIANTS(X) X(4, 8, 8) X(8, 6, 8) X(8, 8, 8) X(8, 10, 8) X(12, 8, 4)

// the same for sweeps in binary32 arithmetic (two values per register pair
// fewer, so taller waves fit)
#define SRJ_INNER_BLOCK_VARIANTS(X) \
    X(8, 6, 8) X(8, 8, 8) X(12, 6, 8) X(12, 8, 8) X(16, 8, 4) X(24, 8, 4)
#define SRJ_INNER_BLOCK2_VARIANTS(X) X(6, 8, 8) X(8, 8, 8) X(8, 10, 8) X(12, 8, 4)

}  // namespace srj
