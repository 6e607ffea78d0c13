// 3D relaxed Jacobi sweep: register plane tiles streamed along axis 2.
//
// One sweep (Islam & Wang, arXiv 2011.06636, section 2, Eq. 3 in residual
// form) of a 7-point stencil with constant or per-face couplings and a
// constant or per-point diagonal, in the fixed order
//   s = D u - c0lo u_{-e0} - c0hi u_{+e0} - c1lo u_{-e1} - c1hi u_{+e1}
//           - c2lo u_{-e2} - c2hi u_{+e2},   u' = u + w (Dinv (f - s)),
// without fused multiply-add (bit-identical to the other kernels).  A ghost
// neighbour is loaded as zero with a zero coupling, which leaves s unchanged.
//
// A wave owns 64 columns along axis 0 (lane = column; the outer lane on each
// side is a halo, 62 columns are written) and H rows along axis 1 (in
// registers), and walks ZC planes along axis 2.  It keeps the previous,
// current and next plane of u in registers, plus the rows just above and
// below its H rows; neighbours along axis 0 come from DPP wave shifts.  Each
// value of u, f, D and each coupling is loaded once per plane (rows and
// lanes of the halo aside); in binary64 a per-point 1/D is computed, not
// loaded.  Value policy V as in tile2d.h; FACE selects
// per-face couplings (all three axes) and DIAG a per-point diagonal.
#pragma once

#include "internal.h"
#include "stream3d.h"
#include "tile2d.h"

#pragma clang fp contract(off)

namespace srj {

// W: written columns per tile, 62 (one halo lane on each side) or 60 (two,
// the tiling of the two-sweep kernel, which batches mixing both use)
template <class V, int H, int ZC, bool FACE, bool DIAG, int W = 62>
__device__ __forceinline__ void plane3d_run(const Stencil3<typename V::A> &S,
                                            const typename V::T *__restrict__ x,
                                            typename V::T *__restrict__ xo,
                                            const typename V::T *__restrict__ b,
                                            typename V::A w, int tx, int ty, int tz, int lane)
{
    using A = typename V::A;
    constexpr bool kRecipInPlace = sizeof(A) == sizeof(double);
    const int64_t n0 = S.n0, n1 = S.n1, n2 = S.n2;
    const int64_t s1 = n0, s2 = n0 * n1;
    static_assert(W == 62 || W == 60, "tile width");
    constexpr int kLo = (64 - W) / 2;  // first written lane
    const int64_t gx = (int64_t)tx * W - kLo + lane;
    const int64_t gy0 = (int64_t)ty * H;
    const int64_t z0 = (int64_t)tz * ZC;
    const int64_t z1 = z0 + ZC < n2 ? z0 + ZC : n2;
    const bool col_in = gx >= 0 && gx < n0;
    auto row_ok = [&](int64_t gy) { return col_in && gy >= 0 && gy < n1; };
    // 16-bit storage: addresses are a wave-uniform row offset (rows clamped
    // into the grid, formed once per tile) plus a plane offset (clamped) plus
    // a 32-bit lane offset (lanes outside the grid read column 0), so every
    // load is unconditional, and values outside the grid are then replaced by
    // zero through per-lane selects (a wave-uniform condition would let the
    // compiler branch around each load and wait for it on its own).  Measured
    // 1.8-1.9x faster for 16-bit storage; binary32 and binary64 keep per-lane
    // addresses and predicated loads, which measured faster for them.
    constexpr bool kLean = sizeof(typename V::T) == 2;
    const int64_t colp = gx;  // column part of the flat index
    const uint32_t off = col_in ? (uint32_t)gx : 0u;
    int64_t yoff[H + 2];  // rows gy0 - 1 .. gy0 + H
    uint32_t rows_in = 0;
#pragma unroll
    for (int i = 0; i < H + 2; ++i) {
        const int64_t gy = gy0 - 1 + i;
        yoff[i] = (gy < 0 ? 0 : (gy >= n1 ? n1 - 1 : gy)) * s1;
        if (gy >= 0 && gy < n1) rows_in |= 1u << i;
    }
    auto zoff = [&](int64_t z) { return (z < 0 ? 0 : (z >= n2 ? n2 - 1 : z)) * s2; };
    auto lane_rows = [&](int64_t z) -> uint32_t {
        return (col_in && z >= 0 && z < n2) ? rows_in : 0u;
    };
    auto ldu = [&](int64_t z, int64_t gy) -> A {
        if constexpr (!kLean)
            return (z >= 0 && z < n2 && row_ok(gy)) ? V::load(x[colp + gy * s1 + z * s2]) : A(0);
        const int i = (int)(gy - gy0) + 1;
        const A v = V::load(x[zoff(z) + yoff[i] + off]);
        return ((lane_rows(z) >> i) & 1) ? v : A(0);
    };
    auto ldc = [&](const A *arr, A cst, int64_t z, int64_t gy) -> A {  // coupling / D / 1/D
        if constexpr (!kLean) {
            if (!(z >= 0 && z < n2 && row_ok(gy))) return A(0);
            return arr ? arr[colp + gy * s1 + z * s2] : cst;
        }
        const int i = (int)(gy - gy0) + 1;
        const bool in = (lane_rows(z) >> i) & 1;
        if (!arr) return in ? cst : A(0);
        const A v = arr[zoff(z) + yoff[i] + off];
        return in ? v : A(0);
    };
    // Products are formed once and moved or kept, not recomputed: c0lo u_{-e0}
    // is lane p-1's (c0 u) shifted one lane; with constant couplings, c1 u of
    // a row serves the rows on both sides, and c2 u of a plane serves the
    // planes before and after it.  A product does not depend on where it is
    // formed, so the terms are bit-identical to forming each one in place.
    A um[H], uc[H], up[H];
    A f2m[H];
    A pm[H], pc[H];  // constant couplings: c2 * plane z - 1 and c2 * plane z
#pragma unroll
    for (int r = 0; r < H; ++r) {
        um[r] = ldu(z0 - 1, gy0 + r);
        uc[r] = ldu(z0, gy0 + r);
        f2m[r] = FACE ? ldc(S.face[2], S.c[2], z0 - 1, gy0 + r) : S.c[2];
        if (!FACE) {
            pm[r] = S.c[2] * um[r];
            pc[r] = S.c[2] * uc[r];
        }
    }
    for (int64_t z = z0; z < z1; ++z) {
        A bz[H], f0[H], f1[H], f2c[H], dd[H], di[H];
#pragma unroll
        for (int r = 0; r < H; ++r) {
            const int64_t gy = gy0 + r;
            up[r] = ldu(z + 1, gy);
            if constexpr (kLean) {
                const A v = V::load(b[zoff(z) + yoff[r + 1] + off]);
                bz[r] = row_ok(gy) ? v : A(0);
            } else {
                bz[r] = row_ok(gy) ? V::load(b[colp + gy * s1 + z * s2]) : A(0);
            }
            // couplings stored towards a point outside the grid (last column,
            // row or plane) are never used: taken as zero, as the ghost term
            // they would multiply is left out by the one-sweep kernel
            f0[r] = FACE ? ldc(S.face[0], S.c[0], z, gy) : S.c[0];
            f1[r] = FACE ? ldc(S.face[1], S.c[1], z, gy) : S.c[1];
            f2c[r] = FACE ? ldc(S.face[2], S.c[2], z, gy) : S.c[2];
            if (FACE) {  // per-lane selects (col_in is per lane)
                f0[r] = (col_in && gx == n0 - 1) ? A(0) : f0[r];
                f1[r] = (col_in && gy == n1 - 1) ? A(0) : f1[r];
                f2c[r] = (col_in && z == n2 - 1) ? A(0) : f2c[r];
            }
            dd[r] = DIAG ? ldc(S.diag, S.dconst, z, gy) : S.dconst;
            // binary64: 1/D is formed here (a correctly rounded division, as
            // the stored array holds) instead of being read, 8 bytes less per
            // point; binary32 keeps the stored binary64 reciprocal rounded to
            // binary32, which a binary32 division would not reproduce
            if (DIAG && kRecipInPlace)
                di[r] = row_ok(gy) ? A(1) / dd[r] : A(0);
            else
                di[r] = DIAG ? ldc(S.dinv, S.dinvconst, z, gy) : S.dinvconst;
        }
        const A u_above = ldu(z, gy0 - 1);   // row gy0 - 1 of this plane
        const A u_below = ldu(z, gy0 + H);   // row gy0 + H of this plane
        const A f1_above = FACE ? ldc(S.face[1], S.c[1], z, gy0 - 1) : S.c[1];
        // constant couplings: c1 * row, for the H rows and the two outside
        A py[H + 2];
        A pp[H];
        if (!FACE) {
            py[0] = S.c[1] * u_above;
#pragma unroll
            for (int r = 0; r < H; ++r) py[r + 1] = S.c[1] * uc[r];
            py[H + 1] = S.c[1] * u_below;
#pragma unroll
            for (int r = 0; r < H; ++r) pp[r] = S.c[2] * up[r];
        }
#pragma unroll
        for (int r = 0; r < H; ++r) {
            const A xc = uc[r];
            A s = dd[r] * xc;
            if (FACE) {
                const A yu = r > 0 ? uc[r - 1] : u_above;
                const A yd = r + 1 < H ? uc[r + 1] : u_below;
                const A cl1 = r > 0 ? f1[r - 1] : f1_above;
                s = s - dpp_prev(f0[r] * xc);
                s = s - f0[r] * dpp_next(xc);
                s = s - cl1 * yu;
                s = s - f1[r] * yd;
                s = s - f2m[r] * um[r];
                s = s - f2c[r] * up[r];
            } else {
                const A p0 = S.c[0] * xc;
                s = s - dpp_prev(p0);
                s = s - dpp_next(p0);
                s = s - py[r];
                s = s - py[r + 2];
                s = s - pm[r];
                s = s - pp[r];
            }
            const A rr = bz[r] - s;
            const A t = di[r] * rr;
            const int64_t gy = gy0 + r;
            if (lane >= kLo && lane < kLo + W && row_ok(gy))
                xo[zoff(z) + yoff[r + 1] + off] = V::store(xc + w * t);
        }
#pragma unroll
        for (int r = 0; r < H; ++r) {
            um[r] = uc[r];
            uc[r] = up[r];
            f2m[r] = f2c[r];
            if (!FACE) {
                pm[r] = pc[r];
                pc[r] = pp[r];
            }
        }
    }
}

// Wave item of a plane kernel (four waves per workgroup).  Hardware places
// workgroup i on XCD i % 8; each XCD takes a contiguous range of items, so a
// tile's neighbours in y (tiles_x items away) run on the same XCD at about the
// same time and its halo rows come from that XCD's L2.  Returns -1 for the
// workgroups beyond the items (the grid is a multiple of 8 workgroups).
__device__ __forceinline__ int plane_item(int64_t items)
{
    const int nwg = (int)((items + 3) / 4);
    const int per_xcd = (nwg + 7) / 8;
    const int logical = (int)(blockIdx.x % 8) * per_xcd + (int)(blockIdx.x / 8);
    if (logical >= nwg) return -1;
    return logical * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
}

// Workgroups to launch for `items` wave items: a multiple of 8.
inline unsigned plane_grid(int64_t items)
{
    const int64_t nwg = (items + 3) / 4;
    return (unsigned)((nwg + 7) / 8 * 8);
}

template <class V, int H, int ZC, bool FACE, bool DIAG>
__global__ __launch_bounds__(256) void k_plane3d(Stencil3<typename V::A> S,
                                                 const typename V::T *__restrict__ x,
                                                 typename V::T *__restrict__ xo,
                                                 const typename V::T *__restrict__ b,
                                                 const typename V::A *__restrict__ wp, int tiles_x,
                                                 int tiles_y, int tiles_z)
{
    const int item = plane_item((int64_t)tiles_x * tiles_y * tiles_z);
    if (item < 0 || item >= tiles_x * tiles_y * tiles_z) return;  // whole wave leaves
    const int tx = item % tiles_x, ty = (item / tiles_x) % tiles_y, tz = item / (tiles_x * tiles_y);
    plane3d_run<V, H, ZC, FACE, DIAG>(S, x, xo, b, wp[0], tx, ty, tz, threadIdx.x & 63);
}

template <class V, int H, int ZC>
hipError_t launch_plane3d(const Stencil3<typename V::A> &S, const typename V::T *x,
                          typename V::T *xo, const typename V::T *b, const typename V::A *w_dev,
                          hipStream_t s)
{
    const int tx = (int)((S.n0 + 61) / 62), ty = (int)((S.n1 + H - 1) / H),
              tz = (int)((S.n2 + ZC - 1) / ZC);
    const int64_t items = (int64_t)tx * ty * tz;
    if (items > INT32_MAX - 64) return hipErrorInvalidValue;
    const dim3 grid(plane_grid(items));
    const bool face = S.face[0] && S.face[1] && S.face[2];
    const bool diag = S.diag != nullptr;
    if (face && diag)
        hipLaunchKernelGGL((k_plane3d<V, H, ZC, true, true>), grid, dim3(256), 0, s, S, x, xo, b, w_dev, tx, ty, tz);
    else if (!face && !S.face[0] && !S.face[1] && !S.face[2] && !diag)
        hipLaunchKernelGGL((k_plane3d<V, H, ZC, false, false>), grid, dim3(256), 0, s, S, x, xo, b, w_dev, tx, ty, tz);
    else
        return hipErrorInvalidValue;  // mixed coefficient kinds: use another plan
    return hipGetLastError();
}

// Coefficient layouts the plane kernel takes: all faces and a per-point
// diagonal, or constant couplings and diagonal.
inline bool plane3d_fits(int ndim, const void *f0, const void *f1, const void *f2, const void *diag)
{
    if (ndim != 3) return false;
    const bool all = f0 && f1 && f2 && diag;
    const bool none = !f0 && !f1 && !f2 && !diag;
    return all || none;
}

// (rows per tile, planes per chunk) of the plane plans (kind 6)
#define SRJ_PLANE_VARIANTS(X) X(2, 16) X(4, 8) X(4, 16) X(4, 32) X(8, 16)

}  // namespace srj
