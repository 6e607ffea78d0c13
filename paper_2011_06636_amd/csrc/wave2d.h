// 2D relaxed Jacobi sweeps fused by a wavefront down a column strip.
//
// Same per-point expression as every other kernel (Islam & Wang, arXiv
// 2011.06636, section 2, Eq. 3 in residual form, no fused multiply-add), so
// results are bit-identical.
//
// A wave owns a strip of 64 columns (lane = column) and OH + 2T rows, and
// walks it from top to bottom.  Sweep level k runs two rows behind level k-1,
// so every loaded row is pushed through all T sweeps while it is still in
// registers and the T updates of one step are independent; each level keeps
// only its three latest rows, and the vertical halo costs 2T rows per strip
// chunk instead of 2T rows per tile.  Horizontal neighbours come from DPP wave
// shifts; the outer T lanes on each side are the horizontal halo.  Ghost
// points (outside the grid) hold zero at every level and are never updated.
// b is kept for the last 2T + 1 rows; windows are shifted every step, so
// indexing is static and everything lives in registers.  Blocks are mapped to strips so that
// consecutive strips of one chunk row land on the same XCD (shared halo rows
// stay in that XCD's L2).
#pragma once

#include "internal.h"
#include "tile2d.h"

#pragma clang fp contract(off)

namespace srj {

// Rows loaded ahead of the one being swept: a wave keeps the loads of the
// next kWavePrefetch rows in flight while it sweeps, so that one wave has
// several rows' worth of HBM requests outstanding instead of one.
constexpr int kWavePrefetch = 8;

template <class V, int OH, int T>
__device__ __forceinline__ void wave2d_run(int64_t n0, int64_t n1, const typename V::T *__restrict__ x,
                                           typename V::T *__restrict__ xo,
                                           const typename V::T *__restrict__ b,
                                           const typename V::A *__restrict__ wlist,
                                           Coef2D<typename V::A> k2, int tx, int ty, int lane)
{
    using A = typename V::A;
    constexpr int R = OH + 2 * T;  // rows of the strip chunk, halo included
    constexpr int OW = 64 - 2 * T;
    constexpr int PF = kWavePrefetch;
    const int64_t gx = (int64_t)tx * OW - T + lane;
    const int64_t gy0 = (int64_t)ty * OH - T;
    const bool col_in = gx >= 0 && gx < n0;
    const bool interior = (int64_t)tx * OW - T >= 0 && (int64_t)tx * OW - T + 64 <= n0 &&
                          gy0 >= 0 && gy0 + R <= n1;
    A w[T];
#pragma unroll
    for (int k = 0; k < T; ++k) w[k] = wlist[k];
    // Level k works two rows behind level k - 1: at step i it produces row
    // i - 2k from rows i - 2k - 1 .. i - 2k + 1 of level k - 1, which the
    // previous steps produced.  All levels of a step therefore read only the
    // windows left by the previous step and are independent of each other.
    // W[j][0..2]: the three latest rows of level j; Bw[m]: b of row i - m.
    A W[T][3], Bw[2 * T + 1];
#pragma unroll
    for (int j = 0; j < T; ++j) W[j][0] = W[j][1] = W[j][2] = A(0);
#pragma unroll
    for (int j = 0; j <= 2 * T; ++j) Bw[j] = A(0);
    // Loads are unconditional: a point outside the grid reads a point inside
    // it (row and column clamped), and when the row is used a select
    // replaces the value by the ghost's zero, so the compiler never branches
    // around a load and waits for it alone.  Rows past the chunk read its
    // last row and are dropped.
    const int64_t cx = gx < 0 ? 0 : (gx >= n0 ? n0 - 1 : gx);
    auto load_row = [&](int i, typename V::T &xv, typename V::T &bv) {
        const int64_t gy = gy0 + i;
        const int64_t cy = gy < 0 ? 0 : (gy >= n1 ? n1 - 1 : gy);
        const int64_t p = cy * n0 + cx;
        xv = x[p];
        bv = b[p];
    };
    auto row_ok = [&](int i) {
        const int64_t gy = gy0 + i;
        return i < R && (interior || (col_in && gy >= 0 && gy < n1));
    };
    typename V::T xq[PF], bq[PF];  // raw rows i .. i + PF - 1
#pragma unroll
    for (int j = 0; j < PF; ++j) load_row(j, xq[j], bq[j]);
#pragma unroll
    for (int i = 0; i < R + T; ++i) {
        // b of row i enters the ring
#pragma unroll
        for (int j = 2 * T; j > 0; --j) Bw[j] = Bw[j - 1];
        const bool ok = row_ok(i);
        const A xin = ok ? V::load(xq[0]) : A(0);
        Bw[0] = ok ? V::load(bq[0]) : A(0);
#pragma unroll
        for (int j = 0; j + 1 < PF; ++j) {
            xq[j] = xq[j + 1];
            bq[j] = bq[j + 1];
        }
        load_row(i + PF, xq[PF - 1], bq[PF - 1]);
        A nxt[T + 1];
#pragma unroll
        for (int k = 1; k <= T; ++k) {
            // row of level k produced at this step; rows outside [k, R-1-k] are
            // halo values that are computed but never stored
            const int r = i - 2 * k;
            const A xc = W[k - 1][1];
            const A up = W[k - 1][0];
            const A dn = W[k - 1][2];
            // c0 u_{p -+ e0} is the neighbour lane's c0 u, shifted one lane
            const A p0 = k2.c0 * xc;
            A s = k2.D * xc;
            s = s - dpp_prev(p0);
            s = s - dpp_next(p0);
            s = s - k2.c1 * up;
            s = s - k2.c1 * dn;
            const A rr = Bw[2 * k] - s;
            const A t = k2.Dinv * rr;
            A nx = V::round(xc + w[k - 1] * t);
            const int64_t gy = gy0 + r;
            if (!interior && !(col_in && gy >= 0 && gy < n1)) nx = A(0);  // ghosts stay zero
            nxt[k] = nx;
            if (k == T && r >= T && r < R - T && lane >= T && lane < 64 - T && col_in && gy < n1)
                xo[gy * n0 + gx] = V::store(nx);
        }
        // advance the windows: level 0 takes row i, level k < T its new row
        W[0][0] = W[0][1];
        W[0][1] = W[0][2];
        W[0][2] = xin;
#pragma unroll
        for (int k = 1; k < T; ++k) {
            W[k][0] = W[k][1];
            W[k][1] = W[k][2];
            W[k][2] = nxt[k];
        }
    }
}

template <class V, int OH, int T>
__global__ __launch_bounds__(256) void k_wave2d(int64_t n0, int64_t n1, const typename V::T *__restrict__ x,
                                                typename V::T *__restrict__ xo,
                                                const typename V::T *__restrict__ b,
                                                const typename V::A *__restrict__ wlist,
                                                Coef2D<typename V::A> k2, int strips_x, int chunks_y,
                                                int nblocks)
{
    // XCD-aware order: hardware places block i on XCD i % 8; give each XCD a
    // contiguous range of logical blocks so neighbouring strips share its L2.
    const int per_xcd = (nblocks + 7) / 8;
    const int logical = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
    const int item = logical * 4 + (threadIdx.x >> 6);
    if (logical >= nblocks || item >= strips_x * chunks_y) return;  // whole wave leaves
    wave2d_run<V, OH, T>(n0, n1, x, xo, b, wlist, k2, item % strips_x, item / strips_x,
                         threadIdx.x & 63);
}

template <class V, int OH, int T>
hipError_t launch_wave2d_t(int64_t n0, int64_t n1, const typename V::T *x, typename V::T *xo,
                           const typename V::T *b, const typename V::A *w_dev,
                           Coef2D<typename V::A> k2, hipStream_t s)
{
    constexpr int OW = 64 - 2 * T;
    const int strips_x = (int)((n0 + OW - 1) / OW);
    const int chunks_y = (int)((n1 + OH - 1) / OH);
    const int64_t items = (int64_t)strips_x * chunks_y;
    const int nblocks = (int)((items + 3) / 4);
    // launch a multiple of 8 blocks so the XCD mapping covers every logical block
    const int grid = (nblocks + 7) / 8 * 8;
    hipLaunchKernelGGL((k_wave2d<V, OH, T>), dim3(grid), dim3(256), 0, s, n0, n1, x, xo, b, w_dev,
                       k2, strips_x, chunks_y, nblocks);
    return hipGetLastError();
}

// Dispatch on the sweeps of this launch (1 .. TMAX) for output height OH.
template <class V, int OH, int TMAX>
hipError_t launch_wave2d(int T, int64_t n0, int64_t n1, const typename V::T *x, typename V::T *xo,
                         const typename V::T *b, const typename V::A *w_dev,
                         Coef2D<typename V::A> k2, hipStream_t s)
{
    switch (T) {
    case 1: return launch_wave2d_t<V, OH, 1>(n0, n1, x, xo, b, w_dev, k2, s);
    case 2: if (TMAX >= 2) return launch_wave2d_t<V, OH, (TMAX >= 2 ? 2 : 1)>(n0, n1, x, xo, b, w_dev, k2, s); break;
    case 3: if (TMAX >= 3) return launch_wave2d_t<V, OH, (TMAX >= 3 ? 3 : 1)>(n0, n1, x, xo, b, w_dev, k2, s); break;
    case 4: if (TMAX >= 4) return launch_wave2d_t<V, OH, (TMAX >= 4 ? 4 : 1)>(n0, n1, x, xo, b, w_dev, k2, s); break;
    case 5: if (TMAX >= 5) return launch_wave2d_t<V, OH, (TMAX >= 5 ? 5 : 1)>(n0, n1, x, xo, b, w_dev, k2, s); break;
    case 6: if (TMAX >= 6) return launch_wave2d_t<V, OH, (TMAX >= 6 ? 6 : 1)>(n0, n1, x, xo, b, w_dev, k2, s); break;
    case 7: if (TMAX >= 7) return launch_wave2d_t<V, OH, (TMAX >= 7 ? 7 : 1)>(n0, n1, x, xo, b, w_dev, k2, s); break;
    case 8: if (TMAX >= 8) return launch_wave2d_t<V, OH, (TMAX >= 8 ? 8 : 1)>(n0, n1, x, xo, b, w_dev, k2, s); break;
    default: break;
    }
    return hipErrorInvalidValue;
}

// (output rows per strip chunk, most sweeps per launch) of the wavefront plans (kind 5)
#define SRJ_WAVE_VARIANTS(X) X(8, 2) X(8, 4) X(12, 4) X(16, 4) X(32, 4) X(32, 8)

}  // namespace srj
