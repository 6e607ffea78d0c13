// Two relaxed Jacobi sweeps per launch on 3D grids with constant couplings
// and diagonal (plan kind 11).
//
// Same per-point expression and order as plane3d.h (Islam & Wang, arXiv
// 2011.06636, section 2, Eq. 3 in residual form, no fused multiply-add):
//   s = D u - c0 u_{-e0} - c0 u_{+e0} - c1 u_{-e1} - c1 u_{+e1}
//           - c2 u_{-e2} - c2 u_{+e2},   u' = u + w (Dinv (f - s)),
// so iterates are bit-identical to one sweep per launch.
//
// A wave owns 64 columns along axis 0 (lane = column; two halo lanes on each
// side, 60 written columns) and H written rows along axis 1, and walks ZC
// planes along axis 2.  The first sweep runs one plane ahead of the second:
// when input plane z + 1 arrives, the first sweep forms plane z (rows
// gy0 - 1 .. gy0 + H, from input rows gy0 - 2 .. gy0 + H + 1) and the second
// sweep forms plane z - 1 (rows gy0 .. gy0 + H - 1) from the first sweep's
// planes z - 2, z - 1 and z.  Registers hold three input planes of H + 4
// rows, three first-sweep planes of H + 2 rows and two planes of the
// right-hand side.  First-sweep values at points outside the grid are set to
// zero, as the ghosts are, so the second sweep sees the boundary exactly as
// the first.  Each input value is read once per wave, with the halo rows,
// lanes and the two planes before and after the chunk read again by the
// neighbouring waves (mostly from L2); per written point and launch that is
// 24 bytes in binary64 for two sweeps.
#pragma once

#include "internal.h"
#include "plane3d.h"
#include "stream3d.h"
#include "tile2d.h"

#pragma clang fp contract(off)

namespace srj {

template <class V, int H, int ZC>
__device__ __forceinline__ void plane3d2_run(const Stencil3<typename V::A> &S,
                                             const typename V::T *__restrict__ x,
                                             typename V::T *__restrict__ xo,
                                             const typename V::T *__restrict__ b,
                                             typename V::A w1, typename V::A w2, int tx, int ty,
                                             int tz, int lane)
{
    using A = typename V::A;
    constexpr int R0 = H + 4, R1 = H + 2;
    const int64_t n0 = S.n0, n1 = S.n1, n2 = S.n2;
    const int64_t s1 = n0, s2 = n0 * n1;
    const int64_t gx = (int64_t)tx * 60 - 2 + lane;
    const int64_t gy0 = (int64_t)ty * H;
    const int64_t z0 = (int64_t)tz * ZC;
    const int64_t z1 = z0 + ZC < n2 ? z0 + ZC : n2;
    const bool col_in = gx >= 0 && gx < n0;
    // addresses: a wave-uniform row offset (rows clamped into the grid, formed
    // once per tile) plus a plane offset (clamped, once per plane) plus a
    // 32-bit lane offset (lanes outside the grid read column 0); values outside
    // the grid are then replaced by zero, so every load is unconditional
    const uint32_t off = col_in ? (uint32_t)gx : 0u;
    const A c0 = S.c[0], c1 = S.c[1], c2 = S.c[2], D = S.dconst, Di = S.dinvconst;
    // input row i is gy0 - 2 + i; first-sweep row j is gy0 - 1 + j (input row j + 1)
    int64_t yoff[R0];
    uint32_t rows_in = 0;
#pragma unroll
    for (int i = 0; i < R0; ++i) {
        const int64_t gy = gy0 - 2 + i;
        yoff[i] = (gy < 0 ? 0 : (gy >= n1 ? n1 - 1 : gy)) * s1;
        if (gy >= 0 && gy < n1) rows_in |= 1u << i;
    }
    auto zoff = [&](int64_t z) { return (z < 0 ? 0 : (z >= n2 ? n2 - 1 : z)) * s2; };
    // per lane: the rows of plane z that lie in the grid (none outside it).
    // Kept per lane so that the selects below stay selects: a wave-uniform
    // condition would let the compiler branch around each load and wait for
    // it on its own
    auto lane_rows = [&](int64_t z) -> uint32_t {
        return (col_in && z >= 0 && z < n2) ? rows_in : 0u;
    };
    // input row i of the plane at offset zo
    auto ldx = [&](int64_t zo, uint32_t lr, int i) -> A {
        const A v = V::load(x[zo + yoff[i] + off]);
        return ((lr >> i) & 1) ? v : A(0);
    };
    auto ldb = [&](int64_t zo, uint32_t lr, int i) -> A {
        const A v = V::load(b[zo + yoff[i] + off]);
        return ((lr >> i) & 1) ? v : A(0);
    };
    A u0m[R0], u0c[R0], u0p[R0];
    A u1m[R1], u1c[R1], u1n[R1];
    A bp[R1], bc[R1];
    {
        const int64_t zm = zoff(z0 - 2), zc = zoff(z0 - 1);
        const uint32_t okm = lane_rows(z0 - 2), okc = lane_rows(z0 - 1);
#pragma unroll
        for (int i = 0; i < R0; ++i) {
            u0m[i] = ldx(zm, okm, i);
            u0c[i] = ldx(zc, okc, i);
        }
    }
#pragma unroll
    for (int j = 0; j < R1; ++j) u1m[j] = u1c[j] = bp[j] = A(0);
    for (int64_t z = z0 - 1; z <= z1; ++z) {
        const int64_t zn = zoff(z + 1), zc = zoff(z);
        const uint32_t okn = lane_rows(z + 1), okc = lane_rows(z);
#pragma unroll
        for (int i = 0; i < R0; ++i) u0p[i] = ldx(zn, okn, i);
#pragma unroll
        for (int j = 0; j < R1; ++j) bc[j] = ldb(zc, okc, j + 1);
        // first sweep, plane z
#pragma unroll
        for (int j = 0; j < R1; ++j) {
            const A xc = u0c[j + 1];
            A s = D * xc;
            const A p0 = c0 * xc;
            s = s - dpp_prev(p0);
            s = s - dpp_next(p0);
            s = s - c1 * u0c[j];
            s = s - c1 * u0c[j + 2];
            s = s - c2 * u0m[j + 1];
            s = s - c2 * u0p[j + 1];
            const A rr = bc[j] - s;
            const A t = Di * rr;
            const A nx = V::round(xc + w1 * t);
            u1n[j] = ((okc >> (j + 1)) & 1) ? nx : A(0);
        }
        // second sweep, plane z - 1
        if (z > z0) {
            const int64_t zo = zoff(z - 1);
#pragma unroll
            for (int r = 0; r < H; ++r) {
                const A xc = u1c[r + 1];
                A s = D * xc;
                const A p0 = c0 * xc;
                s = s - dpp_prev(p0);
                s = s - dpp_next(p0);
                s = s - c1 * u1c[r];
                s = s - c1 * u1c[r + 2];
                s = s - c2 * u1m[r + 1];
                s = s - c2 * u1n[r + 1];
                const A rr = bp[r + 1] - s;
                const A t = Di * rr;
                // plane z - 1 lies in the grid (z0 <= z - 1 < z1)
                if (lane >= 2 && lane < 62 && col_in && ((rows_in >> (r + 2)) & 1))
                    xo[zo + yoff[r + 2] + off] = V::store(xc + w2 * t);
            }
        }
#pragma unroll
        for (int i = 0; i < R0; ++i) {
            u0m[i] = u0c[i];
            u0c[i] = u0p[i];
        }
#pragma unroll
        for (int j = 0; j < R1; ++j) {
            u1m[j] = u1c[j];
            u1c[j] = u1n[j];
            bp[j] = bc[j];
        }
    }
}

template <class V, int H, int ZC>
__global__ __launch_bounds__(256) void k_plane3d2(Stencil3<typename V::A> S,
                                                  const typename V::T *__restrict__ x,
                                                  typename V::T *__restrict__ xo,
                                                  const typename V::T *__restrict__ b,
                                                  const typename V::A *__restrict__ wp,
                                                  int tiles_x, int tiles_y, int tiles_z)
{
    const int item = plane_item((int64_t)tiles_x * tiles_y * tiles_z);
    if (item < 0 || item >= tiles_x * tiles_y * tiles_z) return;  // whole wave leaves
    const int tx = item % tiles_x, ty = (item / tiles_x) % tiles_y, tz = item / (tiles_x * tiles_y);
    plane3d2_run<V, H, ZC>(S, x, xo, b, wp[0], wp[1], tx, ty, tz, threadIdx.x & 63);
}

// Two sweeps x -> xo with factors w_dev[0], w_dev[1] (device pointer).
template <class V, int H, int ZC>
hipError_t launch_plane3d2(const Stencil3<typename V::A> &S, const typename V::T *x,
                           typename V::T *xo, const typename V::T *b, const typename V::A *w_dev,
                           hipStream_t s)
{
    if (S.face[0] || S.face[1] || S.face[2] || S.diag) return hipErrorInvalidValue;
    if (S.n0 > INT32_MAX) return hipErrorInvalidValue;  // lane offsets are 32-bit
    const int64_t tx = (S.n0 + 59) / 60, ty = (S.n1 + H - 1) / H, tz = (S.n2 + ZC - 1) / ZC;
    const int64_t items = tx * ty * tz;
    if (items > INT32_MAX - 64) return hipErrorInvalidValue;
    const dim3 grid(plane_grid(items));
    hipLaunchKernelGGL((k_plane3d2<V, H, ZC>), grid, dim3(256), 0, s, S, x, xo, b, w_dev, (int)tx,
                       (int)ty, (int)tz);
    return hipGetLastError();
}

// Two sweeps per pass with per-face couplings and a per-point diagonal (plan
// kind 12), in the order of the per-face path of plane3d.h:
//   s = D u - f0[p-e0] u_{-e0} - f0[p] u_{+e0} - f1[p-e1] u_{-e1} - f1[p] u_{+e1}
//           - f2[p-e2] u_{-e2} - f2[p] u_{+e2},   u' = u + w (Dinv (f - s)).
// The tiling and the plane lag are those of plane3d2_run.  For the first
// sweep at plane z the pass loads, besides x and b, the couplings f0, f2, D
// (and 1/D, or in binary64 a correctly rounded 1/D formed in place) of the
// first-sweep rows and f1 of those rows and the row below; the second sweep
// at plane z - 1 reuses that plane's coefficients from the previous step and
// f2 of plane z - 2 from the step before.  Coefficients outside the grid are
// zero, as in plane3d.h.  Per written point and launch: x, b, three
// couplings, D (and 1/D below binary64) read once and x' written once, for
// two sweeps.
template <class V, int H, int ZC>
__device__ __forceinline__ void plane3d2f_run(const Stencil3<typename V::A> &S,
                                              const typename V::T *__restrict__ x,
                                              typename V::T *__restrict__ xo,
                                              const typename V::T *__restrict__ b,
                                              typename V::A w1, typename V::A w2, int tx, int ty,
                                              int tz, int lane)
{
    using A = typename V::A;
    constexpr bool kRecipInPlace = sizeof(A) == sizeof(double);
    constexpr int R0 = H + 4, R1 = H + 2;
    const int64_t n0 = S.n0, n1 = S.n1, n2 = S.n2;
    const int64_t s1 = n0, s2 = n0 * n1;
    const int64_t gx = (int64_t)tx * 60 - 2 + lane;
    const int64_t gy0 = (int64_t)ty * H;
    const int64_t z0 = (int64_t)tz * ZC;
    const int64_t z1 = z0 + ZC < n2 ? z0 + ZC : n2;
    const bool col_in = gx >= 0 && gx < n0;
    // addressing as in plane3d2_run
    const uint32_t off = col_in ? (uint32_t)gx : 0u;
    const A *__restrict__ F0 = S.face[0];
    const A *__restrict__ F1 = S.face[1];
    const A *__restrict__ F2 = S.face[2];
    const A *__restrict__ DG = S.diag;
    const A *__restrict__ DI = S.dinv;
    int64_t yoff[R0];  // input row i is gy0 - 2 + i; first-sweep row j is input row j + 1
    uint32_t rows_in = 0;
#pragma unroll
    for (int i = 0; i < R0; ++i) {
        const int64_t gy = gy0 - 2 + i;
        yoff[i] = (gy < 0 ? 0 : (gy >= n1 ? n1 - 1 : gy)) * s1;
        if (gy >= 0 && gy < n1) rows_in |= 1u << i;
    }
    auto zoff = [&](int64_t z) { return (z < 0 ? 0 : (z >= n2 ? n2 - 1 : z)) * s2; };
    auto lane_rows = [&](int64_t z) -> uint32_t {
        return (col_in && z >= 0 && z < n2) ? rows_in : 0u;
    };
    auto ldv = [&](const typename V::T *__restrict__ arr, int64_t zo, uint32_t lr, int i) -> A {
        const A v = V::load(arr[zo + yoff[i] + off]);
        return ((lr >> i) & 1) ? v : A(0);
    };
    auto ldc = [&](const A *__restrict__ arr, int64_t zo, uint32_t lr, int i) -> A {
        const A v = arr[zo + yoff[i] + off];
        return ((lr >> i) & 1) ? v : A(0);
    };
    A u0m[R0], u0c[R0], u0p[R0];
    A u1m[R1], u1c[R1], u1n[R1];
    // coefficients of the current plane z (index: first-sweep row j, f1 by
    // input row i) and of plane z - 1 (the previous step's), f2 of z - 1, z - 2
    A bc[R1], f0c[R1], f1c[R1 + 1], f2c[R1], dc[R1], ic[R1];
    A bp[R1], f0p[R1], f1p[R1 + 1], dp[R1], ip[R1];
    A f2m[R1], f2mm[R1];
    // couplings stored towards a point outside the grid (last column, row or
    // plane) are never used by the one-sweep kernel: taken as zero through
    // the per-lane row masks (rows of f1 without the last grid row, no rows
    // of f0 in the last column, no rows of f2 in the last plane)
    const uint32_t not_last_col = (col_in && gx == n0 - 1) ? 0u : ~0u;
    uint32_t not_last_row = ~0u;
#pragma unroll
    for (int i = 0; i < R0; ++i)
        if (gy0 - 2 + i == n1 - 1) not_last_row &= ~(1u << i);
    {
        const int64_t zm = zoff(z0 - 2), zc = zoff(z0 - 1);
        const uint32_t okm = lane_rows(z0 - 2), okc = lane_rows(z0 - 1);
#pragma unroll
        for (int i = 0; i < R0; ++i) {
            u0m[i] = ldv(x, zm, okm, i);
            u0c[i] = ldv(x, zc, okc, i);
        }
#pragma unroll
        for (int j = 0; j < R1; ++j) f2m[j] = ldc(F2, zm, okm, j + 1);  // plane z0 - 2 < n2 - 1
    }
#pragma unroll
    for (int j = 0; j < R1; ++j) {
        u1m[j] = u1c[j] = bp[j] = f0p[j] = dp[j] = ip[j] = f2mm[j] = A(0);
        f1p[j] = A(0);
    }
    f1p[R1] = A(0);
    for (int64_t z = z0 - 1; z <= z1; ++z) {
        const int64_t zn = zoff(z + 1), zc = zoff(z);
        const uint32_t okn = lane_rows(z + 1), okc = lane_rows(z);
#pragma unroll
        for (int i = 0; i < R0; ++i) u0p[i] = ldv(x, zn, okn, i);
#pragma unroll
        for (int j = 0; j < R1; ++j) {
            bc[j] = ldv(b, zc, okc, j + 1);
            f0c[j] = ldc(F0, zc, okc & not_last_col, j + 1);
            f2c[j] = ldc(F2, zc, okc & (z == n2 - 1 ? 0u : ~0u), j + 1);
            dc[j] = ldc(DG, zc, okc, j + 1);
            if constexpr (kRecipInPlace)
                ic[j] = ((okc >> (j + 1)) & 1) ? A(1) / dc[j] : A(0);
            else
                ic[j] = ldc(DI, zc, okc, j + 1);
        }
#pragma unroll
        for (int i = 0; i <= R1; ++i) f1c[i] = ldc(F1, zc, okc & not_last_row, i);
        // first sweep, plane z
#pragma unroll
        for (int j = 0; j < R1; ++j) {
            const A xc = u0c[j + 1];
            A s = dc[j] * xc;
            s = s - dpp_prev(f0c[j] * xc);
            s = s - f0c[j] * dpp_next(xc);
            s = s - f1c[j] * u0c[j];
            s = s - f1c[j + 1] * u0c[j + 2];
            s = s - f2m[j] * u0m[j + 1];
            s = s - f2c[j] * u0p[j + 1];
            const A rr = bc[j] - s;
            const A t = ic[j] * rr;
            const A nx = V::round(xc + w1 * t);
            u1n[j] = ((okc >> (j + 1)) & 1) ? nx : A(0);
        }
        // second sweep, plane z - 1 (coefficients of the previous step)
        if (z > z0) {
            const int64_t zo = zoff(z - 1);
#pragma unroll
            for (int r = 0; r < H; ++r) {
                const int j = r + 1;  // first-sweep row of output row r
                const A xc = u1c[j];
                A s = dp[j] * xc;
                s = s - dpp_prev(f0p[j] * xc);
                s = s - f0p[j] * dpp_next(xc);
                s = s - f1p[j] * u1c[j - 1];
                s = s - f1p[j + 1] * u1c[j + 1];
                s = s - f2mm[j] * u1m[j];
                s = s - f2m[j] * u1n[j];
                const A rr = bp[j] - s;
                const A t = ip[j] * rr;
                // plane z - 1 lies in the grid (z0 <= z - 1 < z1)
                if (lane >= 2 && lane < 62 && col_in && ((rows_in >> (r + 2)) & 1))
                    xo[zo + yoff[r + 2] + off] = V::store(xc + w2 * t);
            }
        }
#pragma unroll
        for (int i = 0; i < R0; ++i) {
            u0m[i] = u0c[i];
            u0c[i] = u0p[i];
        }
#pragma unroll
        for (int j = 0; j < R1; ++j) {
            u1m[j] = u1c[j];
            u1c[j] = u1n[j];
            bp[j] = bc[j];
            f0p[j] = f0c[j];
            dp[j] = dc[j];
            ip[j] = ic[j];
            f2mm[j] = f2m[j];
            f2m[j] = f2c[j];
        }
#pragma unroll
        for (int i = 0; i <= R1; ++i) f1p[i] = f1c[i];
    }
}

template <class V, int H, int ZC>
__global__ __launch_bounds__(256) void k_plane3d2f(Stencil3<typename V::A> S,
                                                   const typename V::T *__restrict__ x,
                                                   typename V::T *__restrict__ xo,
                                                   const typename V::T *__restrict__ b,
                                                   const typename V::A *__restrict__ wp,
                                                   int tiles_x, int tiles_y, int tiles_z)
{
    const int item = plane_item((int64_t)tiles_x * tiles_y * tiles_z);
    if (item < 0 || item >= tiles_x * tiles_y * tiles_z) return;  // whole wave leaves
    const int tx = item % tiles_x, ty = (item / tiles_x) % tiles_y, tz = item / (tiles_x * tiles_y);
    plane3d2f_run<V, H, ZC>(S, x, xo, b, wp[0], wp[1], tx, ty, tz, threadIdx.x & 63);
}

// Two sweeps x -> xo, per-face couplings and diagonal (1/D read below
// binary64), factors w_dev[0], w_dev[1] (device pointer).
template <class V, int H, int ZC>
hipError_t launch_plane3d2f(const Stencil3<typename V::A> &S, const typename V::T *x,
                            typename V::T *xo, const typename V::T *b,
                            const typename V::A *w_dev, hipStream_t s)
{
    if (!S.face[0] || !S.face[1] || !S.face[2] || !S.diag) return hipErrorInvalidValue;
    if (sizeof(typename V::A) != sizeof(double) && !S.dinv) return hipErrorInvalidValue;
    if (S.n0 > INT32_MAX) return hipErrorInvalidValue;  // lane offsets are 32-bit
    const int64_t tx = (S.n0 + 59) / 60, ty = (S.n1 + H - 1) / H, tz = (S.n2 + ZC - 1) / ZC;
    const int64_t items = tx * ty * tz;
    if (items > INT32_MAX - 64) return hipErrorInvalidValue;
    const dim3 grid(plane_grid(items));
    hipLaunchKernelGGL((k_plane3d2f<V, H, ZC>), grid, dim3(256), 0, s, S, x, xo, b, w_dev,
                       (int)tx, (int)ty, (int)tz);
    return hipGetLastError();
}

// (written rows per tile, planes per chunk) of the two-sweep plane plans
// (kind 11): binary64 sweeps, and the inner sweeps of the refinement modes
#define SRJ_PLANE2_VARIANTS(X) X(2, 16) X(4, 8) X(4, 16) X(6, 16)
#define SRJ_INNER_PLANE2_VARIANTS(X) X(4, 16) X(6, 16) X(8, 8) X(8, 16)
// (written rows per tile, planes per chunk) of the per-face two-sweep plans
// (kind 12)
#define SRJ_PLANE2F_VARIANTS(X) X(2, 8) X(2, 16) X(4, 8) X(4, 16)
#define SRJ_INNER_PLANE2F_VARIANTS(X) X(2, 16) X(4, 8) X(4, 16) X(6, 16)

}  // namespace srj
