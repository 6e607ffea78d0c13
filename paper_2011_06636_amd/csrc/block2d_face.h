// 2D relaxed Jacobi sweeps with per-face couplings and a per-point diagonal,
// fused over blocks of cooperating waves (plan kind 10).
//
// Same per-point expression as every other kernel (Islam & Wang, arXiv
// 2011.06636, section 2, Eq. 3 in residual form, no fused multiply-add):
//   s = D_p x_p - f0[p-1] x[p-1] - f0[p] x[p+1] - f1[p-n0] x[p-n0] - f1[p] x[p+n0]
//   x'_p = x_p + w (Dinv_p (b_p - s))
// so results are bit-identical to the one-sweep kernel and the CPU reference.
// The value policy V (storage.h) gives the arithmetic and storage types: binary64
// for the plain sweeps, binary32 arithmetic with binary32, binary16 or bfloat16
// storage (rounded after every sweep) for the inner sweeps of the refinement
// modes, whose couplings, D and 1/D are binary32 copies.
//
// The block layout is that of block2d.h with one column per lane: NW waves
// hold HW rows each of 64 columns, halo included, with x, b, both face
// couplings, D and 1/D of every point in registers.  f0[p-1] x[p-1] is the
// left lane's own product f0 x, moved one lane by DPP; x[p+1] comes from the
// right lane by DPP.  f1[p-n0] x[p-n0] is the row below's product f1 x, kept
// from that row (formed from its value before the sweep) or, for a wave's
// first row, published in LDS by the wave below; x[p+n0] of a wave's last row
// is the wave above's first row, also through LDS (one barrier per sweep).
// Points outside the grid load zero values and zero coefficients, so their
// terms vanish (f x with x = 0) and they stay zero; the couplings stored for
// the last column and row (towards points outside the grid, never used) are
// taken as zero too.
#pragma once

#include "block2d.h"
#include "internal.h"
#include "storage.h"
#include "tile2d.h"

#pragma clang fp contract(off)

namespace srj {

// With UPD (binary64 only), each sweep also finds the largest |x' - x| over
// the block's written points and merges it into slot [ring][k] of st (see
// UpdFState): out_lane and [rlo, rhi) select the written lanes and rows.
template <class V, int HW, int NW, bool MASK, bool UPD>
__device__ __forceinline__ void blockf_sweeps(typename V::A (&xr)[HW],
                                              const typename V::A (&br)[HW],
                                              const typename V::A (&fe)[HW],
                                              const typename V::A (&fn)[HW],
                                              const typename V::A (&dd)[HW],
                                              const typename V::A (&di)[HW], bool col_in,
                                              uint32_t rowbits,
                                              const typename V::A *__restrict__ wlist, int T,
                                              typename V::A *edge, int wave, int lane,
                                              bool out_lane, int rlo, int rhi, UpdFState *st,
                                              int ring, unsigned long long *red)
{
    using A = typename V::A;
    // red: [2][NW] per-wave maxima of the previous sweeps; thread 0 merges
    // sweep k - 1 after sweep k's barrier (the last one after a final barrier)
    const int stripe = (int)(blockIdx.x % kUpdFStripes);
    auto merge = [&](int k) {
        unsigned long long m = red[(k & 1) * NW];
#pragma unroll
        for (int w2 = 1; w2 < NW; ++w2) m = red[(k & 1) * NW + w2] > m ? red[(k & 1) * NW + w2] : m;
        atomicMax(&st->maxbits[ring][k][stripe * kUpdStride], m);
    };
    for (int k = 0; k < T; ++k) {
        const A w = wlist[k];  // requested before the barrier (as in block2d.h)
        // edge: [2 buffers][0: first row's x, 1: last row's f1 x][NW][64]
        A *e = edge + (k & 1) * (2 * NW * 64);
        e[wave * 64 + lane] = xr[0];
        e[(NW + wave) * 64 + lane] = fn[HW - 1] * xr[HW - 1];
        __syncthreads();
        if (UPD && k > 0 && threadIdx.x == 0) merge(k - 1);
        unsigned long long dmax = 0ull;
        // rows outside the block read zero (they only feed halo rows)
        A pdown = wave > 0 ? e[(NW + wave - 1) * 64 + lane] : A(0);
        const A xup = wave + 1 < NW ? e[(wave + 1) * 64 + lane] : A(0);
#pragma unroll
        for (int r = 0; r < HW; ++r) {
            const A xc = xr[r];
            const A pl = dpp_prev(fe[r] * xc);  // f0[p-1] x[p-1]: the left lane's product
            const A xrt = dpp_next(xc);          // x[p+1]
            const A xu = r + 1 < HW ? xr[r + 1] : xup;
            const A pn = fn[r] * xc;  // f1 x of this row, the down term of the row above
            A s = dd[r] * xc;
            s = s - pl;
            s = s - fe[r] * xrt;
            s = s - pdown;
            s = s - fn[r] * xu;
            const A rr = br[r] - s;
            const A t = di[r] * rr;
            const A nx = V::round(xc + w * t);
            pdown = pn;
            if (UPD && r >= rlo && r < rhi) {
                const bool wr = out_lane && (!MASK || (col_in && ((rowbits >> r) & 1)));
                const unsigned long long d =
                    wr ? (unsigned long long)__double_as_longlong(fabs(nx - xc)) : 0ull;
                dmax = d > dmax ? d : dmax;
            }
            if (MASK)
                xr[r] = (col_in && ((rowbits >> r) & 1)) ? nx : A(0);
            else
                xr[r] = nx;
        }
        if (UPD) {
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) {
                const unsigned long long o = __shfl_xor(dmax, off);
                dmax = o > dmax ? o : dmax;
            }
            if (lane == 0) red[(k & 1) * NW + wave] = dmax;
        }
    }
    if (UPD) {
        __syncthreads();
        if (threadIdx.x == 0) merge(T - 1);
    }
}

// One wave's part of one block (see block2d_run for the addressing and the
// treatment of blocks that cross the grid's edge).
template <class V, int HW, int HALO, int NW, bool EDGE, bool UPD>
__device__ __forceinline__ void blockf_run(int64_t n0, int64_t n1,
                                           const typename V::T *__restrict__ x,
                                           typename V::T *__restrict__ xo,
                                           const typename V::T *__restrict__ b,
                                           const typename V::A *__restrict__ f0,
                                           const typename V::A *__restrict__ f1,
                                           const typename V::A *__restrict__ dg,
                                           const typename V::A *__restrict__ dgi,
                                           const typename V::A *__restrict__ wlist, int T,
                                           int64_t bx0, int64_t by0, int wv, int lane,
                                           typename V::A *edge, UpdFState *st, int ring,
                                           unsigned long long *red)
{
    using A = typename V::A;
    using S = BlockShape<HW, HALO, NW, 1>;
    const int64_t gy0 = by0 + (int64_t)wv * HW;
    const int64_t gx = bx0 + lane;
    const bool col_in = !EDGE || (gx >= 0 && gx < n0);
    const bool col_last = EDGE && gx == n0 - 1;
    const uint32_t off = col_in ? (uint32_t)gx : 0u;
    uint32_t rowbits = ~0u;
    if (EDGE) {
        rowbits = 0;
#pragma unroll
        for (int r = 0; r < HW; ++r)
            if (gy0 + r >= 0 && gy0 + r < n1) rowbits |= 1u << r;
    }
    auto row_of = [&](int r) -> int64_t {
        const int64_t gy = gy0 + r;
        return EDGE ? (gy < 0 ? 0 : (gy >= n1 ? n1 - 1 : gy)) : gy;
    };
    A xr[HW], br[HW], fe[HW], fn[HW], dd[HW], di[HW];
#pragma unroll
    for (int r = 0; r < HW; ++r) {
        const int64_t base = row_of(r) * n0 + off;
        const bool in = !EDGE || (((rowbits >> r) & 1) && col_in);
        const bool row_last = EDGE && gy0 + r == n1 - 1;
        const A vx = V::load(x[base]), vb = V::load(b[base]), v0 = f0[base], v1 = f1[base],
                vd = dg[base];
        // binary64: 1/D formed here (a correctly rounded division, the value
        // the stored array holds), 8 bytes less per point; below binary64 the
        // stored reciprocal (rounded from binary64) is read
        A vi;
        if constexpr (sizeof(A) == sizeof(double))
            vi = A(1) / vd;
        else
            vi = dgi[base];
        xr[r] = in ? vx : A(0);
        br[r] = in ? vb : A(0);
        fe[r] = in && !col_last ? v0 : A(0);
        fn[r] = in && !row_last ? v1 : A(0);
        dd[r] = in ? vd : A(0);
        di[r] = in ? vi : A(0);
    }
    const bool out_lane = lane >= HALO && lane < S::BW - HALO;
    const int rlo = HALO - wv * HW, rhi = S::BH - HALO - wv * HW;
    blockf_sweeps<V, HW, NW, EDGE, UPD>(xr, br, fe, fn, dd, di, col_in, rowbits, wlist, T, edge, wv,
                                        lane, out_lane, rlo, rhi, st, ring, red);
    if (!out_lane || !col_in) return;
#pragma unroll
    for (int r = 0; r < HW; ++r)
        if (r >= rlo && r < rhi && ((rowbits >> r) & 1)) xo[row_of(r) * n0 + off] = V::store(xr[r]);
}

template <class V, int HW, int HALO, int NW, bool UPD>
__global__ __launch_bounds__(64 * NW) void k_blockf2d(int64_t n0, int64_t n1,
                                                      const typename V::T *__restrict__ x,
                                                      typename V::T *__restrict__ xo,
                                                      const typename V::T *__restrict__ b,
                                                      const typename V::A *__restrict__ f0,
                                                      const typename V::A *__restrict__ f1,
                                                      const typename V::A *__restrict__ dg,
                                                      const typename V::A *__restrict__ dgi,
                                                      const typename V::A *__restrict__ wlist,
                                                      int T, int blocks_x, int nblocks,
                                                      int reverse, UpdFState *st, int ring)
{
    __shared__ typename V::A edge[2 * 2 * NW * 64];
    __shared__ unsigned long long red[UPD ? 2 * NW : 1];
    if (UPD && st->flag) return;  // an earlier sweep met the update test
    // XCD-aware order, each XCD's range walked backwards on alternate launches
    // (as in block2d.h)
    const int per_xcd = (nblocks + 7) / 8;
    const int j = blockIdx.x / 8;
    const int logical = (blockIdx.x % 8) * per_xcd + (reverse ? per_xcd - 1 - j : j);
    if (logical >= nblocks) return;  // whole block leaves
    using S = BlockShape<HW, HALO, NW, 1>;
    const int64_t bx0 = (int64_t)(logical % blocks_x) * S::OW - HALO;
    const int64_t by0 = (int64_t)(logical / blocks_x) * S::OH - HALO;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (bx0 >= 0 && bx0 + S::BW <= n0 && by0 >= 0 && by0 + S::BH <= n1)
        blockf_run<V, HW, HALO, NW, false, UPD>(n0, n1, x, xo, b, f0, f1, dg, dgi, wlist, T, bx0,
                                                by0, wv, lane, edge, st, ring, red);
    else
        blockf_run<V, HW, HALO, NW, true, UPD>(n0, n1, x, xo, b, f0, f1, dg, dgi, wlist, T, bx0,
                                               by0, wv, lane, edge, st, ring, red);
}

// UPD: the update-test form (binary64; st and ring as for blockf_sweeps).
template <class V, int HW, int HALO, int NW, bool UPD = false>
hipError_t launch_blockf2d(int64_t n0, int64_t n1, const typename V::T *x, typename V::T *xo,
                           const typename V::T *b, const typename V::A *f0,
                           const typename V::A *f1, const typename V::A *dg,
                           const typename V::A *dgi, const typename V::A *w_dev, int T,
                           hipStream_t s, bool reverse, UpdFState *st = nullptr, int ring = 0)
{
    static_assert(!UPD || sizeof(typename V::A) == sizeof(double), "the update test is binary64");
    if (UPD && (!st || T > kUpdFMaxT || ring < 0 || ring > 1)) return hipErrorInvalidValue;
    using S = BlockShape<HW, HALO, NW, 1>;
    if (T < 1 || T > HALO) return hipErrorInvalidValue;
    if (n0 > INT32_MAX) return hipErrorInvalidValue;  // column offsets are 32-bit
    if (!f0 || !f1 || !dg || !dgi) return hipErrorInvalidValue;
    const int64_t bxn = (n0 + S::OW - 1) / S::OW, byn = (n1 + S::OH - 1) / S::OH;
    const int64_t nblocks = bxn * byn;
    if (nblocks > (int64_t)1 << 28) return hipErrorInvalidValue;
    const int grid = (int)((nblocks + 7) / 8 * 8);
    hipLaunchKernelGGL((k_blockf2d<V, HW, HALO, NW, UPD>), dim3(grid), dim3(64 * NW), 0, s, n0, n1,
                       x, xo, b, f0, f1, dg, dgi, w_dev, T, (int)bxn, (int)nblocks,
                       reverse ? 1 : 0, st, ring);
    return hipGetLastError();
}

// (rows per wave, halo = most sweeps per launch, waves per block) of the
// per-face block plans (kind 10): binary64 sweeps, and the inner sweeps of
// the refinement modes
#define SRJ_BLOCKF_VARIANTS(X) X(4, 6, 8) X(4, 8, 16) X(4, 12, 16) X(6, 8, 8) X(8, 8, 8)
#define SRJ_INNER_BLOCKF_VARIANTS(X) X(4, 8, 16) X(8, 8, 8) X(8, 10, 8) X(12, 8, 8)

}  // namespace srj
