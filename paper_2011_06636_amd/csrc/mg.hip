// SRJ cycles as the smoother of a geometric multigrid V-cycle.
//
// Islam & Wang (arXiv 2011.06636) name SRJ as a candidate multigrid smoother
// in section 5 without a design; this file's design is the library's reading:
//   * vertex-centred coarsening of odd grids: every active axis halves,
//     n' = (n - 1) / 2, while all active sizes are odd and >= 3;
//   * coarse operators rediscretised on the doubled spacing: couplings and
//     diagonal divided by 4 (constant-coefficient stencils only);
//   * full-weighting restriction of the residual and multilinear
//     interpolation of the correction, each a fixed-order sum;
//   * pre- and post-smoothing by whole SRJ cycles of one scheme (section 2,
//     Eqs. 3 and 7), the scheme chosen from one V-cycle to the next by
//     Algorithm 1 of section 3 on the V-cycle residual ratios (or fixed);
//   * the coarsest grid solved by SRJ with Algorithm 1 from zero to a
//     relative tolerance (srj_solve on that level's context).
// Every level is an ordinary context, so smoothing and the coarsest solve use
// the library's sweep, residual and resident kernels; the transfers are the
// two kernels below.  Each value is formed by the same operations in the same
// order as the CPU reference, so iterates are bit-identical to it.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <vector>

#include "internal.h"
#include "rowband.h"
#include "resident_run.h"
#include "rowsum.h"
#include "tile2d.h"
#include "wave2d.h"

#pragma clang fp contract(off)

namespace srj {

namespace {

constexpr int kMgBlock = 256;
static_assert(kMgBlock == kRowUnit, "one transfer workgroup per row unit");
constexpr int kMgMaxLevels = 32;

__device__ __forceinline__ double full_weight(int a) { return a == 0 ? 0.5 : 0.25; }

// Rows per unit of the interpolation: in 3D four, whose loads a thread has
// in flight together (255^3: 25.7 -> 21.8 us per launch on average over the
// levels); in 2D one, since four left the coarser levels too few workgroups
// (the residual and the restriction, tried the same way, gained nothing).
__host__ __device__ constexpr int prolong_rows(int nd) { return nd == 3 ? 4 : 1; }

// Fine residual r = b - A x at every point, the sweep's expression: D x,
// then the axis-0, axis-1, axis-2 neighbours below and above, each
// subtracted only where it lies in the grid.  Neighbour loads are
// unconditional at clamped indices (a select drops the value), so that the
// loads of a point are in flight together.  The restriction weights these
// values; forming them once per fine point instead of once per coarse
// point that uses them (up to 8 in 3D) leaves every value unchanged.
template <int ND>
__global__ __launch_bounds__(kMgBlock) void k_mg_residual(DevProblem P, const double *__restrict__ x,
                                                          double *__restrict__ r)
{
    const int64_t n0 = P.n0, n1 = P.n1, n2 = P.n2;
    int64_t xb, i1, i2;
    if (!row_unit(blockIdx.x, n0, n1, n2, xb, i1, i2)) return;
    const int64_t i0 = xb * kRowUnit + threadIdx.x;
    if (i0 >= n0) return;
    const int64_t t = i0 + n0 * (i1 + n1 * i2);
    const int64_t s1 = n0, s2 = n0 * n1;
    const bool h0 = i0 > 0, h1 = i0 < n0 - 1;
    const bool h2 = ND > 1 && i1 > 0, h3 = ND > 1 && i1 < n1 - 1;
    const bool h4 = ND > 2 && i2 > 0, h5 = ND > 2 && i2 < n2 - 1;
    const double xc = x[t];
    const double v0 = x[h0 ? t - 1 : t], v1 = x[h1 ? t + 1 : t];
    double v2 = 0.0, v3 = 0.0, v4 = 0.0, v5 = 0.0;
    if (ND > 1) {
        v2 = x[h2 ? t - s1 : t];
        v3 = x[h3 ? t + s1 : t];
    }
    if (ND > 2) {
        v4 = x[h4 ? t - s2 : t];
        v5 = x[h5 ? t + s2 : t];
    }
    double s = P.dconst * xc;
    s = h0 ? s - P.c[0] * v0 : s;
    s = h1 ? s - P.c[0] * v1 : s;
    if (ND > 1) {
        s = h2 ? s - P.c[1] * v2 : s;
        s = h3 ? s - P.c[1] * v3 : s;
    }
    if (ND > 2) {
        s = h4 ? s - P.c[2] * v4 : s;
        s = h5 ? s - P.c[2] * v5 : s;
    }
    r[t] = P.b[t] - s;
}

// Coarse right-hand side bc = R r (and, unless xc is null, xc = 0): one
// thread per coarse point; the fine
// residuals of points 2 I + 1 + a (a in {-1, 0, 1} per active axis; all lie
// in the grid, whose active sizes are 2 m + 1) are weighted by the product
// of the per-axis full weights and summed with axis 2 outermost and axis 0
// innermost.
template <int ND>
__global__ __launch_bounds__(kMgBlock) void k_mg_restrict(const double *__restrict__ r,
                                                          double *__restrict__ bc,
                                                          double *__restrict__ xc, int64_t n0,
                                                          int64_t n1, int64_t m0, int64_t m1,
                                                          int64_t m2)
{
    int64_t xb, I1, I2;
    if (!row_unit(blockIdx.x, m0, m1, m2, xb, I1, I2)) return;
    const int64_t I0 = xb * kRowUnit + threadIdx.x;
    if (I0 >= m0) return;
    const int64_t t = I0 + m0 * (I1 + m1 * I2);
    const int64_t s1 = n0, s2 = n0 * n1;
    const int64_t c = (2 * I0 + 1) + (ND > 1 ? s1 * (2 * I1 + 1) : 0) +
                      (ND > 2 ? s2 * (2 * I2 + 1) : 0);
    double s = 0.0;
#pragma unroll
    for (int a2 = (ND > 2 ? -1 : 0); a2 <= (ND > 2 ? 1 : 0); ++a2)
#pragma unroll
        for (int a1 = (ND > 1 ? -1 : 0); a1 <= (ND > 1 ? 1 : 0); ++a1)
#pragma unroll
            for (int a0 = -1; a0 <= 1; ++a0) {
                double wt = full_weight(a0);
                if (ND > 1) wt = wt * full_weight(a1);
                if (ND > 2) wt = wt * full_weight(a2);
                s = s + wt * r[c + a0 + s1 * a1 + s2 * a2];
            }
    bc[t] = s;
    if (xc) xc[t] = 0.0;  // the coarse correction starts from zero
}

// x += P ec.  Per axis a fine index 2 J + 1 takes coarse J with weight 1, a
// fine index 2 J takes coarse J - 1 and J with weight 1/2 (indices outside
// the coarse grid are the zero boundary and give no term); the terms of a
// fine point are summed with axis 2 outermost, axis 0 innermost, candidates
// in increasing order.  One thread per pair of fine points 2 J, 2 J + 1 in
// each of a unit's prolong_rows(ND) rows (rowband.h): both take their coarse
// values from axis-0 columns J - 1 and J of the same rows and planes, so each
// of those is loaded once for the pair.
// Missing terms are skipped by selects (their loads read coarse point 0), so
// each sum is the same as over its present terms alone.  I: the index type
// (32-bit when the fine grid has fewer than 2^31 points).
template <int ND, class I>
__global__ __launch_bounds__(kMgBlock) void k_prolong_add(const double *__restrict__ ec,
                                                          double *__restrict__ x, int64_t n0,
                                                          int64_t n1, int64_t n2, int64_t m0,
                                                          int64_t m1, int64_t m2)
{
    constexpr int R = prolong_rows(ND);
    const int64_t pairs = m0 + 1;  // fine columns 2 J, 2 J + 1 for J = 0 .. m0 (n0 = 2 m0 + 1)
    int64_t xb, y0, z;
    int ny;
    if (!row_unit(blockIdx.x, pairs, n1, n2, R, xb, y0, ny, z)) return;
    const I J = (I)(xb * kRowUnit + threadIdx.x);
    if (J > (I)m0) return;
    const I mm[3] = {(I)m0, (I)m1, (I)m2};
    const I stride[3] = {1, (I)m0, (I)m0 * (I)m1};
    // axis 0: the even point 2 J takes J - 1 and J, the odd point 2 J + 1 takes J
    const bool hm = J - 1 >= 0, h0 = J < mm[0];
    const bool odd_in = J < mm[0];  // 2 J + 1 <= n0 - 1
    double ue[R], uo[R];  // the updated even and odd points of each row
#pragma unroll
    for (int j = 0; j < R; ++j) {
        // rows past the unit's last repeat its first row and are not stored
        const int64_t y = y0 + (j < ny ? j : 0);
        const I ii[3] = {0, (I)y, (I)z};
        // axes 1 and 2: candidate slots, their share of the coarse index, weights
        I off[3][2];
        double cw[3][2];
        bool has[3][2];
#pragma unroll
        for (int d = 1; d < 3; ++d) {
            if (d >= ND) {
                off[d][0] = off[d][1] = 0;
                cw[d][0] = 1.0;
                cw[d][1] = 0.0;
                has[d][0] = true;
                has[d][1] = false;
            } else if (ii[d] & 1) {
                off[d][0] = stride[d] * ((ii[d] - 1) / 2);
                off[d][1] = 0;
                cw[d][0] = 1.0;
                cw[d][1] = 0.0;
                has[d][0] = true;
                has[d][1] = false;
            } else {
                const I K = ii[d] / 2;
                off[d][0] = stride[d] * (K - 1);
                off[d][1] = stride[d] * K;
                cw[d][0] = cw[d][1] = 0.5;
                has[d][0] = K - 1 >= 0;
                has[d][1] = K < mm[d];
            }
        }
        double ve = 0.0, vo = 0.0;
#pragma unroll
        for (int k2 = 0; k2 < (ND > 2 ? 2 : 1); ++k2)
#pragma unroll
            for (int k1 = 0; k1 < (ND > 1 ? 2 : 1); ++k1) {
                const bool on12 = has[1][k1] && has[2][k2];
                const I base = off[1][k1] + off[2][k2];
                const double em = ec[on12 && hm ? base + J - 1 : 0];
                const double e0 = ec[on12 && h0 ? base + J : 0];
                // even point: candidates J - 1 then J, weight 1/2 on axis 0
                {
                    double wt = 0.5;
                    if (ND > 1) wt = wt * cw[1][k1];
                    if (ND > 2) wt = wt * cw[2][k2];
                    ve = (on12 && hm) ? ve + wt * em : ve;
                    ve = (on12 && h0) ? ve + wt * e0 : ve;
                }
                // odd point: candidate J, weight 1 on axis 0
                {
                    double wt = 1.0;
                    if (ND > 1) wt = wt * cw[1][k1];
                    if (ND > 2) wt = wt * cw[2][k2];
                    vo = (on12 && h0) ? vo + wt * e0 : vo;
                }
            }
        const I row = (I)n0 * ((I)y + (I)n1 * (I)z);
        ue[j] = x[row + 2 * J] + ve;
        uo[j] = x[row + 2 * J + (odd_in ? 1 : 0)] + vo;
    }
    // stores after every load: the compiler cannot tell that the stores of
    // one row leave the loads of the next unchanged
#pragma unroll
    for (int j = 0; j < R; ++j) {
        if (j >= ny) break;
        const I row = (I)n0 * ((I)(y0 + j) + (I)n1 * (I)z);
        x[row + 2 * J] = ue[j];
        if (odd_in) x[row + 2 * J + 1] = uo[j];
    }
}

// The last pre-smoothing cycle of a 2D level (T <= 2 sweeps), the fine
// residual of its result and the restriction of that residual, in one pass:
// the wavefront strips of k_wave2d with a halo of T + 2 rows and columns.
// One stage behind the last sweep forms r = b - A x (D x, then the axis-0
// neighbours' c0 u moved by DPP, then the axis-1 neighbours: the fine
// residual's order; ghost values are zero, so an absent neighbour's term
// subtracts +0 and changes no bit) for the written points and one more row
// and column around them; a stage behind that forms, at every written point
// of odd row and column, the full-weighting sum of the coarse point it
// centres (rows -1, 0, 1 outer, columns -1, 0, 1 inner, the restriction's
// order) and writes it to the coarse right-hand side, and zero to the coarse
// correction unless that is null.  The residual itself is never stored.
// Written: x of the strip's 64 - 2 (T + 2) centre columns and OH centre rows
// (both even, so each coarse point belongs to exactly one strip and chunk).
constexpr int kResOH = 8;

template <int T>
__device__ __forceinline__ void wave2d_rr_run(int64_t n0, int64_t n1, const double *__restrict__ x,
                                              double *__restrict__ xo, double *__restrict__ bc,
                                              double *__restrict__ xc0,
                                              const double *__restrict__ b,
                                              const double *__restrict__ wlist, Coef2D<double> k2,
                                              int tx, int ty, int lane)
{
    using A = double;
    constexpr int H = T + 2;  // halo: T sweeps, the residual, the restriction
    constexpr int R = kResOH + 2 * H;
    constexpr int OW = 64 - 2 * H;
    constexpr int PF = kWavePrefetch;
    static_assert(OW % 2 == 0 && kResOH % 2 == 0, "strips and chunks start at even fine indices");
    const int64_t m0 = (n0 - 1) / 2;
    const int64_t gx = (int64_t)tx * OW - H + lane;
    const int64_t gy0 = (int64_t)ty * kResOH - H;
    const bool col_in = gx >= 0 && gx < n0;
    const bool interior = (int64_t)tx * OW - H >= 0 && (int64_t)tx * OW - H + 64 <= n0 &&
                          gy0 >= 0 && gy0 + R <= n1;
    A w[T];
#pragma unroll
    for (int k = 0; k < T; ++k) w[k] = wlist[k];
    // W[j]: the three latest rows of sweep level j (0: input), WT those of
    // the last sweep, RW those of the residual, Bw[m]: b of row i - m
    A W[T][3], WT[3], RW[3], Bw[2 * T + 2];
#pragma unroll
    for (int j = 0; j < T; ++j) W[j][0] = W[j][1] = W[j][2] = A(0);
    WT[0] = WT[1] = WT[2] = A(0);
    RW[0] = RW[1] = RW[2] = A(0);
#pragma unroll
    for (int j = 0; j < 2 * T + 2; ++j) Bw[j] = A(0);
    const int64_t cx = gx < 0 ? 0 : (gx >= n0 ? n0 - 1 : gx);
    auto load_row = [&](int i, double &xv, double &bv) {
        const int64_t gy = gy0 + i;
        const int64_t cy = gy < 0 ? 0 : (gy >= n1 ? n1 - 1 : gy);
        const int64_t p = cy * n0 + cx;
        xv = x[p];
        bv = b[p];
    };
    auto in_grid = [&](int i) {
        const int64_t gy = gy0 + i;
        return interior || (col_in && gy >= 0 && gy < n1);
    };
    double xq[PF], bq[PF];  // raw rows i .. i + PF - 1
#pragma unroll
    for (int j = 0; j < PF; ++j) load_row(j, xq[j], bq[j]);
    const bool lane_out = lane >= H && lane < 64 - H && col_in;
    // a coarse point centred at this lane's column: odd column, not the last
    const bool coarse_col = lane_out && (gx & 1) && gx < n0 - 1;
#pragma unroll
    for (int i = 0; i < R + T; ++i) {
#pragma unroll
        for (int j = 2 * T + 1; j > 0; --j) Bw[j] = Bw[j - 1];
        const bool ok = i < R && in_grid(i);
        const A xin = ok ? xq[0] : A(0);
        Bw[0] = ok ? bq[0] : A(0);
#pragma unroll
        for (int j = 0; j + 1 < PF; ++j) {
            xq[j] = xq[j + 1];
            bq[j] = bq[j + 1];
        }
        load_row(i + PF, xq[PF - 1], bq[PF - 1]);
        A nxt[T + 1];
#pragma unroll
        for (int k = 1; k <= T; ++k) {
            const int r = i - 2 * k;  // row of sweep level k made at this step
            const A xc = W[k - 1][1];
            const A p0 = k2.c0 * xc;
            A s = k2.D * xc;
            s = s - dpp_prev(p0);
            s = s - dpp_next(p0);
            s = s - k2.c1 * W[k - 1][0];
            s = s - k2.c1 * W[k - 1][2];
            const A rr = Bw[2 * k] - s;
            const A t = k2.Dinv * rr;
            A nx = xc + w[k - 1] * t;
            if (!(r >= 0 && r < R && in_grid(r))) nx = A(0);  // ghosts stay zero
            nxt[k] = nx;
            if (k == T && r >= H && r < R - H && lane_out && gy0 + r < n1)
                xo[(gy0 + r) * n0 + gx] = nx;
        }
        W[0][0] = W[0][1];
        W[0][1] = W[0][2];
        W[0][2] = xin;
#pragma unroll
        for (int k = 1; k < T; ++k) {
            W[k][0] = W[k][1];
            W[k][1] = W[k][2];
            W[k][2] = nxt[k];
        }
        WT[0] = WT[1];
        WT[1] = WT[2];
        WT[2] = nxt[T];
        // the residual of row i - 2 T - 1 of the last sweep's iterate
        {
            const A xc = WT[1];
            const A p0 = k2.c0 * xc;
            A s = k2.D * xc;
            s = s - dpp_prev(p0);
            s = s - dpp_next(p0);
            s = s - k2.c1 * WT[0];
            s = s - k2.c1 * WT[2];
            RW[0] = RW[1];
            RW[1] = RW[2];
            RW[2] = Bw[2 * T + 1] - s;
        }
        // full weighting centred at row q = i - 2 T - 2 (residual rows q - 1,
        // q, q + 1 are RW[0 .. 2])
        const int q = i - 2 * T - 2;
        if (q >= H && q < R - H) {
            A sum = 0.0;
#pragma unroll
            for (int a1 = 0; a1 < 3; ++a1) {
                const A row = RW[a1];
                const A v[3] = {dpp_prev(row), row, dpp_next(row)};
#pragma unroll
                for (int a0 = 0; a0 < 3; ++a0) {
                    const A wt = full_weight(a0 - 1) * full_weight(a1 - 1);
                    sum = sum + wt * v[a0];
                }
            }
            const int64_t gy = gy0 + q;
            if (coarse_col && (gy & 1) && gy < n1 - 1) {
                const int64_t t = (gx - 1) / 2 + m0 * ((gy - 1) / 2);
                bc[t] = sum;
                if (xc0) xc0[t] = 0.0;  // the coarse correction starts from zero
            }
        }
    }
}

template <int T>
__global__ __launch_bounds__(256) void k_wave2d_rr(int64_t n0, int64_t n1,
                                                   const double *__restrict__ x,
                                                   double *__restrict__ xo, double *__restrict__ bc,
                                                   double *__restrict__ xc0,
                                                   const double *__restrict__ b,
                                                   const double *__restrict__ wlist,
                                                   Coef2D<double> k2, int strips_x, int chunks_y,
                                                   int nblocks)
{
    // XCD-aware order as in k_wave2d: each XCD a contiguous range of strips
    const int per_xcd = (nblocks + 7) / 8;
    const int logical = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
    const int item = logical * 4 + (threadIdx.x >> 6);
    if (logical >= nblocks || item >= strips_x * chunks_y) return;  // whole wave leaves
    wave2d_rr_run<T>(n0, n1, x, xo, bc, xc0, b, wlist, k2, item % strips_x, item / strips_x,
                     threadIdx.x & 63);
}

// T (1 or 2) sweeps of a 2D constant-coefficient level from x to xo with
// factors w_dev[0 .. T), then bc = R (b - A xo) on the coarse grid and xc = 0
// unless xc is null.
hipError_t launch_wave2d_rr(const DevProblem &P, int T, const double *x, double *xo, double *bc,
                            double *xc, const double *w_dev, hipStream_t s)
{
    if (P.ndim != 2 || P.face[0] || P.face[1] || P.diag || T < 1 || T > 2 || P.n0 % 2 == 0 ||
        P.n1 % 2 == 0)
        return hipErrorInvalidValue;
    const Coef2D<double> k2{P.dconst, P.dinvconst, P.c[0], P.c[1]};
    const int OW = 64 - 2 * (T + 2);
    const int strips_x = (int)((P.n0 + OW - 1) / OW);
    const int chunks_y = (int)((P.n1 + kResOH - 1) / kResOH);
    const int64_t items = (int64_t)strips_x * chunks_y;
    const int nblocks = (int)((items + 3) / 4);
    const int grid = (nblocks + 7) / 8 * 8;
    if (T == 1)
        hipLaunchKernelGGL(k_wave2d_rr<1>, dim3(grid), dim3(256), 0, s, P.n0, P.n1, x, xo, bc, xc,
                           P.b, w_dev, k2, strips_x, chunks_y, nblocks);
    else
        hipLaunchKernelGGL(k_wave2d_rr<2>, dim3(grid), dim3(256), 0, s, P.n0, P.n1, x, xo, bc, xc,
                           P.b, w_dev, k2, strips_x, chunks_y, nblocks);
    return hipGetLastError();
}

// The interpolation of the coarse correction and the first post-smoothing
// cycle of a 2D level (T <= 2 sweeps) in one pass: the wavefront strips of
// k_wave2d (halo T + 1) whose input rows are x + P e, formed as the
// interpolation kernel forms them (axis-1 candidates outer, axis-0 inner,
// each in increasing order, absent candidates skipped).  Each lane loads,
// per coarse row it needs, the coarse value of column floor(gx / 2); an even
// column's other candidate, floor(gx / 2) - 1, is its left lane's value,
// moved by DPP.  The halo is odd (T + 1 rounded up to odd) and strips are an
// even number of columns wide, so lane 0 sits on an odd column and needs no
// left lane.  With part non-null the pass also sums the squares of
// r = b - A x of its written points (the residual norm's expression order)
// into one partial per strip chunk.
template <int T, bool NORM>
__device__ __forceinline__ void wave2d_pp_run(int64_t n0, int64_t n1, const double *__restrict__ x,
                                              double *__restrict__ xo,
                                              const double *__restrict__ ec,
                                              const double *__restrict__ b,
                                              const double *__restrict__ wlist, Coef2D<double> k2,
                                              int tx, int ty, int lane, double *__restrict__ part,
                                              int item)
{
    using A = double;
    constexpr int H = (T + 1) | 1;  // odd: lane 0 on an odd column
    static_assert(H % 2 == 1 && H >= T + 1, "an odd halo of at least T + 1");
    constexpr int R = kResOH + 2 * H;
    constexpr int OW = 64 - 2 * H;
    constexpr int PF = 4;  // rows loaded ahead: four rings of them
    const int64_t m0 = (n0 - 1) / 2, m1 = (n1 - 1) / 2;
    const int64_t gx = (int64_t)tx * OW - H + lane;
    const int64_t gy0 = (int64_t)ty * kResOH - H;
    const bool col_in = gx >= 0 && gx < n0;
    const bool interior = (int64_t)tx * OW - H >= 0 && (int64_t)tx * OW - H + 64 <= n0 &&
                          gy0 >= 0 && gy0 + R <= n1;
    A w[T];
#pragma unroll
    for (int k = 0; k < T; ++k) w[k] = wlist[k];
    // W[j]: the three latest rows of sweep level j (0: input), WT those of
    // the last sweep (NORM), Bw[m]: b of row i - m
    A W[T][3], WT[3], Bw[2 * T + 2];
#pragma unroll
    for (int j = 0; j < T; ++j) W[j][0] = W[j][1] = W[j][2] = A(0);
    WT[0] = WT[1] = WT[2] = A(0);
#pragma unroll
    for (int j = 0; j < 2 * T + 2; ++j) Bw[j] = A(0);
    double acc = 0.0;  // NORM: this lane's squared residuals, in row order
    const int64_t cx = gx < 0 ? 0 : (gx >= n0 ? n0 - 1 : gx);
    // axis 0: this lane's coarse column and the candidates' weights
    const int64_t I = gx >> 1;  // floor(gx / 2), gx >= -H
    const int64_t ci = I < 0 ? 0 : (I >= m0 ? m0 - 1 : I);
    const bool odd = (gx & 1) != 0;
    const bool has_lo = !odd && I - 1 >= 0;  // even column: candidate I - 1
    const bool has_hi = odd || I < m0;       // candidate I (the odd column's only one)
    const A cw0 = odd ? 1.0 : 0.5;
    // coarse rows of fine row gy: J0 (weight cw1), and for even rows J0 + 1
    auto crow = [&](int64_t gy, int64_t &j0, int64_t &j1, bool &h0, bool &h1, A &cw1) {
        if (gy & 1) {
            j0 = (gy - 1) / 2;
            j1 = j0;
            h0 = true;
            h1 = false;
            cw1 = 1.0;
        } else {
            const int64_t J = gy / 2;
            j0 = J - 1;
            j1 = J;
            h0 = J - 1 >= 0;
            h1 = J < m1;
            cw1 = 0.5;
        }
    };
    auto load_row = [&](int i, double &xv, double &bv, double &e0, double &e1) {
        const int64_t gy = gy0 + i;
        const int64_t cy = gy < 0 ? 0 : (gy >= n1 ? n1 - 1 : gy);
        const int64_t p = cy * n0 + cx;
        xv = x[p];
        bv = b[p];
        int64_t j0, j1;
        bool h0, h1;
        A cw1;
        crow(cy, j0, j1, h0, h1, cw1);
        const int64_t r0 = j0 < 0 ? 0 : (j0 >= m1 ? m1 - 1 : j0);
        const int64_t r1 = j1 < 0 ? 0 : (j1 >= m1 ? m1 - 1 : j1);
        e0 = ec[r0 * m0 + ci];
        e1 = ec[r1 * m0 + ci];
    };
    auto in_grid = [&](int i) {
        const int64_t gy = gy0 + i;
        return interior || (col_in && gy >= 0 && gy < n1);
    };
    double xq[PF], bq[PF], eq0[PF], eq1[PF];  // raw rows i .. i + PF - 1
#pragma unroll
    for (int j = 0; j < PF; ++j) load_row(j, xq[j], bq[j], eq0[j], eq1[j]);
    const bool lane_out = lane >= H && lane < 64 - H && col_in;
#pragma unroll
    for (int i = 0; i < R + T; ++i) {
#pragma unroll
        for (int j = 2 * T + 1; j > 0; --j) Bw[j] = Bw[j - 1];
        const bool ok = i < R && in_grid(i);
        // x + P e of row i
        A xin;
        {
            const int64_t gy = gy0 + i;
            const int64_t cy = gy < 0 ? 0 : (gy >= n1 ? n1 - 1 : gy);
            int64_t j0, j1;
            bool h0, h1;
            A cw1;
            crow(cy, j0, j1, h0, h1, cw1);
            const A lo0 = dpp_prev(eq0[0]), lo1 = dpp_prev(eq1[0]);  // column I - 1
            const A wt = cw0 * cw1;
            A v = 0.0;
            v = (h0 && has_lo) ? v + wt * lo0 : v;
            v = (h0 && has_hi) ? v + wt * eq0[0] : v;
            v = (h1 && has_lo) ? v + wt * lo1 : v;
            v = (h1 && has_hi) ? v + wt * eq1[0] : v;
            xin = ok ? xq[0] + v : A(0);
        }
        Bw[0] = ok ? bq[0] : A(0);
#pragma unroll
        for (int j = 0; j + 1 < PF; ++j) {
            xq[j] = xq[j + 1];
            bq[j] = bq[j + 1];
            eq0[j] = eq0[j + 1];
            eq1[j] = eq1[j + 1];
        }
        load_row(i + PF, xq[PF - 1], bq[PF - 1], eq0[PF - 1], eq1[PF - 1]);
        A nxt[T + 1];
#pragma unroll
        for (int k = 1; k <= T; ++k) {
            const int r = i - 2 * k;
            const A xc = W[k - 1][1];
            const A p0 = k2.c0 * xc;
            A s = k2.D * xc;
            s = s - dpp_prev(p0);
            s = s - dpp_next(p0);
            s = s - k2.c1 * W[k - 1][0];
            s = s - k2.c1 * W[k - 1][2];
            const A rr = Bw[2 * k] - s;
            const A t = k2.Dinv * rr;
            A nx = xc + w[k - 1] * t;
            if (!(r >= 0 && r < R && in_grid(r))) nx = A(0);  // ghosts stay zero
            nxt[k] = nx;
            if (k == T && r >= H && r < R - H && lane_out && gy0 + r < n1)
                xo[(gy0 + r) * n0 + gx] = nx;
        }
        W[0][0] = W[0][1];
        W[0][1] = W[0][2];
        W[0][2] = xin;
#pragma unroll
        for (int k = 1; k < T; ++k) {
            W[k][0] = W[k][1];
            W[k][1] = W[k][2];
            W[k][2] = nxt[k];
        }
        if constexpr (NORM) {
            // r = b - A x of written row q = i - 2 T - 1 of the last sweep's
            // iterate, in the residual norm's expression order
            WT[0] = WT[1];
            WT[1] = WT[2];
            WT[2] = nxt[T];
            const int q = i - 2 * T - 1;
            if (q >= H && q < R - H) {
                const A xc = WT[1];
                const A p0 = k2.c0 * xc;
                A s = k2.D * xc;
                s = s - dpp_prev(p0);
                s = s - dpp_next(p0);
                s = s - k2.c1 * WT[0];
                s = s - k2.c1 * WT[2];
                const A v = Bw[2 * T + 1] - s;
                acc = (lane_out && gy0 + q < n1) ? acc + v * v : acc;
            }
        }
    }
    if constexpr (NORM) {
        // fixed-order sum over the wave, one partial per strip chunk
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
        if (lane == 0) part[item] = acc;
    }
}

template <int T, bool NORM>
__global__ __launch_bounds__(256) void k_wave2d_pp(int64_t n0, int64_t n1,
                                                   const double *__restrict__ x,
                                                   double *__restrict__ xo,
                                                   const double *__restrict__ ec,
                                                   const double *__restrict__ b,
                                                   const double *__restrict__ wlist,
                                                   Coef2D<double> k2, int strips_x, int chunks_y,
                                                   int nblocks, double *__restrict__ part)
{
    const int per_xcd = (nblocks + 7) / 8;
    const int logical = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
    const int item = logical * 4 + (threadIdx.x >> 6);
    if (logical >= nblocks || item >= strips_x * chunks_y) return;  // whole wave leaves
    wave2d_pp_run<T, NORM>(n0, n1, x, xo, ec, b, wlist, k2, item % strips_x, item / strips_x,
                           threadIdx.x & 63, part, item);
}

// Strip chunks of the interpolating pass with T sweeps: one residual-norm
// partial each when it forms the norm.
int64_t pp_items(const DevProblem &P, int T)
{
    const int64_t OW = 64 - 2 * ((T + 1) | 1);
    return ((P.n0 + OW - 1) / OW) * ((P.n1 + kResOH - 1) / kResOH);
}

// x + P ec, then T (1 or 2) sweeps of a 2D constant-coefficient level into
// xo with factors w_dev[0 .. T); with part non-null also the sums of squares
// of b - A xo, one per strip chunk (pp_items(P, T) of them).
hipError_t launch_wave2d_pp(const DevProblem &P, int T, const double *x, double *xo,
                            const double *ec, const double *w_dev, hipStream_t s,
                            double *part = nullptr)
{
    if (P.ndim != 2 || P.face[0] || P.face[1] || P.diag || T < 1 || T > 2 || P.n0 % 2 == 0 ||
        P.n1 % 2 == 0 || P.n0 < 3 || P.n1 < 3)
        return hipErrorInvalidValue;
    const Coef2D<double> k2{P.dconst, P.dinvconst, P.c[0], P.c[1]};
    const int OW = 64 - 2 * ((T + 1) | 1);
    const int strips_x = (int)((P.n0 + OW - 1) / OW);
    const int chunks_y = (int)((P.n1 + kResOH - 1) / kResOH);
    const int64_t items = (int64_t)strips_x * chunks_y;
    const int nblocks = (int)((items + 3) / 4);
    const int grid = (nblocks + 7) / 8 * 8;
#define SRJ_PP(TT, NN)                                                                          \
    hipLaunchKernelGGL((k_wave2d_pp<TT, NN>), dim3(grid), dim3(256), 0, s, P.n0, P.n1, x, xo, ec, \
                       P.b, w_dev, k2, strips_x, chunks_y, nblocks, part)
    if (T == 1) {
        if (part) SRJ_PP(1, true);
        else SRJ_PP(1, false);
    } else {
        if (part) SRJ_PP(2, true);
        else SRJ_PP(2, false);
    }
#undef SRJ_PP
    return hipGetLastError();
}

// The coarse end of the V-cycle in three launches: every level from the
// first one of at most kTailMaxPoints points down to the coarsest is held in
// one workgroup's LDS (per level x, its ping-pong partner and b) by
// k_mg_tail<kTailDown> (pre-smoothing, fine residual and restriction level
// by level down), the coarsest grid is solved by the resident solver, and
// k_mg_tail<kTailUp> interpolates and post-smooths level by level up; a
// one-point coarsest grid is solved inside a single launch instead
// (k_mg_tail<kTailWhole>).  The operations are those of the kernels above,
// of the sweep kernels and of the resident solver, in their order, so the
// values are the same bits.  Thread p takes points p,
// p + kThreads, ... of a level (every tail grid has at most kTailPerThread
// kThreads points); the workgroup synchronises after every pass.
constexpr int kTailMaxLevels = 12;
constexpr int kTailPerThread = 4;
constexpr int64_t kTailMaxPoints = (int64_t)kTailPerThread * kThreads;
constexpr size_t kTailLdsDoubles = 19968;  // 156 KiB of the 160 KiB per workgroup

// Largest first tail level: in 3D four points per thread (the 15^3 level
// joins the tail: 255^3 to 1e-10 10.95 -> 10.71 ms); in 1D and 2D one, since
// taking the 63^2 level into the tail cost more than its six launches
// (2047^2 to 2e-9 3.90 -> 4.01 ms).
int64_t tail_max_points(int ndim) { return ndim == 3 ? kTailMaxPoints : kThreads; }

struct TailLevel {
    DevProblem P;       // the level's sizes and constants (b lives in LDS)
    const double *w;    // this V-cycle's smoothing factors for the level
    int32_t M;          // their number
    int32_t off;        // LDS offset of x; its partner at off + N, b at off + 2 N
};

struct TailArgs {
    int32_t count, pre, post, pad;
    TailLevel lv[kTailMaxLevels];
    double *xg[kTailMaxLevels];  // each level's correction in global memory
    double *bg[kTailMaxLevels];  // and its right-hand side
    // kTailWhole: the coarsest grid's solve (one point) inside the launch
    ResidentArgs ra;             // its options
    const double *omega;         // the factor table
    const int32_t *level_m, *offsets;
    ResidentRecord rec;          // where its sweep count goes
};

// What a tail launch runs: down to the coarsest grid, back up from it, or
// both around a one-point coarsest grid solved in the launch.
constexpr int kTailDown = 0, kTailUp = 1, kTailWhole = 2;

// Per-level values of the tail, copied into LDS once: every pass reads its
// level's sizes and constants from there.
struct TailTab {
    int32_t n0, n1, n2, nd, N, off, M, pad;
    double c0, c1, c2, D, Dinv;
    const double *w;
};

// The solve of a one-point coarsest grid, A u = b with A = D, as the
// single-wave resident kernel runs it for that grid: from u, cycles of the
// scheme Algorithm 1 picks (section 3) with the factors of Eq. (17) in the
// library's order, u <- u + w (1/D) (b - D u), the norm |b - D u| (the
// square root of the one square) after each cycle, the same stop tests and
// the same level arithmetic, so every value and count is the same.  Returns
// the status; sweeps counts the sweeps run.
__device__ int point_solve(double &u, double bv, double D, double Dinv,
                           const double *__restrict__ omega, const int32_t *__restrict__ level_m,
                           const int32_t *__restrict__ offsets, const ResidentArgs &a,
                           int64_t &sweeps)
{
    auto norm_of = [&]() {
        const double r = bv - D * u;
        return sqrt(r * r);
    };
    const double norm0 = norm_of();
    const double r0 = a.r0_given > 0.0 ? a.r0_given : norm0;
    const double target = a.tol_mode == SRJ_TOL_RELATIVE ? a.tol * r0 : a.tol;
    int status = SRJ_ERR_NOT_CONVERGED, level = a.start_level;
    double prev = norm0;
    sweeps = 0;
    if (!isfinite(norm0)) return SRJ_ERR_NONFINITE;
    if (norm0 == 0.0 || norm0 < target) return SRJ_OK;
    for (int cycle = 0; cycle < a.max_cycles; ++cycle) {
        const int lv = a.rule == SRJ_RULE_FIXED ? a.fixed_level : level;
        const int M = level_m[lv];
        if (sweeps + M > a.max_sweeps) break;
        const double *w = omega + offsets[lv];
        for (int j = 0; j < M; ++j) {
            const double r = bv - D * u;
            const double tt = Dinv * r;
            u = u + w[j] * tt;
        }
        sweeps += M;
        const double norm = norm_of();
        if (!isfinite(norm)) return SRJ_ERR_NONFINITE;
        if (norm < target) return SRJ_OK;
        const double ratio = norm / prev;
        prev = norm;
        int nl = level;
        if (a.rule == SRJ_RULE_HEURISTIC) {
            if (ratio > 0.4)
                nl = level + 1;
            else if (ratio < 0.4 && ratio > 0.2)
                nl = level - 1;
        } else if (a.rule == SRJ_RULE_INCREASING) {
            nl = level + 1;
        }
        level = nl < 0 ? 0 : (nl > a.max_level ? a.max_level : nl);
    }
    return status;
}

// kTailDown: from the first tail level's b (in bg[0]) down to the coarsest
// grid's b, leaving every level's pre-smoothed correction and b in xg / bg
// (the coarsest correction zero); kTailUp: from those and the coarsest
// solution back up, the first level's correction to xg[0]; kTailWhole: both
// without the round trip through xg / bg, around the solve of a one-point
// coarsest grid (point_solve).
template <int MODE>
__global__ __launch_bounds__(kThreads) void k_mg_tail(TailArgs t)
{
    extern __shared__ double lds[];
    __shared__ TailTab tab[kTailMaxLevels];
    const int p = threadIdx.x;
    if (p < t.count) {
        const TailLevel &L = t.lv[p];
        TailTab e;
        e.n0 = (int32_t)L.P.n0;
        e.n1 = (int32_t)L.P.n1;
        e.n2 = (int32_t)L.P.n2;
        e.nd = L.P.ndim;
        e.N = e.n0 * e.n1 * e.n2;
        e.off = L.off;
        e.M = L.M;
        e.pad = 0;
        e.c0 = L.P.c[0];
        e.c1 = L.P.c[1];
        e.c2 = L.P.c[2];
        e.D = L.P.dconst;
        e.Dinv = L.P.dinvconst;
        e.w = L.w;
        tab[p] = e;
    }
    __syncthreads();
    // which of a level's two buffers holds its iterate: bit l of par
    uint32_t par = 0;
    auto xbuf = [&](int l) { return lds + tab[l].off + (((par >> l) & 1) ? tab[l].N : 0); };
    auto spare = [&](int l) { return lds + tab[l].off + (((par >> l) & 1) ? 0 : tab[l].N); };
    auto bbuf = [&](int l) { return lds + tab[l].off + 2 * tab[l].N; };
    auto coords = [&](const TailTab &e, int q, int &i0, int &i1, int &i2) {
        const int a0 = q / e.n0;
        i0 = q - a0 * e.n0;
        i1 = a0 % e.n1;
        i2 = a0 / e.n1;
    };
    // (A u)_p in the library's order: D u_p, then per axis the lower and the
    // upper neighbour, terms of ghost neighbours omitted
    auto rows = [&](const TailTab &e, const double *u, int q, int i0, int i1, int i2) {
        double s = e.D * u[q];
        if (i0 > 0) s = s - e.c0 * u[q - 1];
        if (i0 < e.n0 - 1) s = s - e.c0 * u[q + 1];
        if (e.nd >= 2) {
            if (i1 > 0) s = s - e.c1 * u[q - e.n0];
            if (i1 < e.n1 - 1) s = s - e.c1 * u[q + e.n0];
        }
        if (e.nd >= 3) {
            const int s2 = e.n0 * e.n1;
            if (i2 > 0) s = s - e.c2 * u[q - s2];
            if (i2 < e.n2 - 1) s = s - e.c2 * u[q + s2];
        }
        return s;
    };
    // nu whole cycles of the level's scheme, as the sweep kernels form them
    auto smooth = [&](int l, int nu) {
        const TailTab e = tab[l];
        const double *b = bbuf(l);
        for (int k = 0; k < nu; ++k) {
            double wnext = e.w[0];
            for (int j = 0; j < e.M; ++j) {
                const double wj = wnext;
                if (j + 1 < e.M) wnext = e.w[j + 1];  // in flight during this sweep
                const double *cur = xbuf(l);
                double *nxt = spare(l);
                for (int q = p; q < e.N; q += kThreads) {
                    int i0, i1, i2;
                    coords(e, q, i0, i1, i2);
                    const double s = rows(e, cur, q, i0, i1, i2);
                    const double r = b[q] - s;
                    const double tt = e.Dinv * r;
                    nxt[q] = cur[q] + wj * tt;
                }
                __syncthreads();
                par ^= 1u << l;
            }
        }
    };
    if constexpr (MODE != kTailUp) {
        for (int q = p; q < tab[0].N; q += kThreads) {
            bbuf(0)[q] = t.bg[0][q];
            xbuf(0)[q] = 0.0;
        }
        __syncthreads();
        for (int l = 0; l + 1 < t.count; ++l) {
            smooth(l, t.pre);
            // fine residual into the level's spare buffer, then full weighting
            const TailTab e = tab[l], ec = tab[l + 1];
            double *r = spare(l);
            for (int q = p; q < e.N; q += kThreads) {
                int i0, i1, i2;
                coords(e, q, i0, i1, i2);
                r[q] = bbuf(l)[q] - rows(e, xbuf(l), q, i0, i1, i2);
            }
            __syncthreads();
            for (int q = p; q < ec.N; q += kThreads) {
                int I0, I1, I2;
                coords(ec, q, I0, I1, I2);
                const int s1 = e.n0, s2 = e.n0 * e.n1;
                const int c = (2 * I0 + 1) + (e.nd > 1 ? s1 * (2 * I1 + 1) : 0) +
                              (e.nd > 2 ? s2 * (2 * I2 + 1) : 0);
                double sum = 0.0;
                for (int a2 = (e.nd > 2 ? -1 : 0); a2 <= (e.nd > 2 ? 1 : 0); ++a2)
                    for (int a1 = (e.nd > 1 ? -1 : 0); a1 <= (e.nd > 1 ? 1 : 0); ++a1)
#pragma unroll
                        for (int a0 = -1; a0 <= 1; ++a0) {
                            double wt = full_weight(a0);
                            if (e.nd > 1) wt = wt * full_weight(a1);
                            if (e.nd > 2) wt = wt * full_weight(a2);
                            sum = sum + wt * r[c + a0 + s1 * a1 + s2 * a2];
                        }
                bbuf(l + 1)[q] = sum;
                xbuf(l + 1)[q] = 0.0;
            }
            __syncthreads();
        }
        if constexpr (MODE == kTailDown)
            for (int l = 0; l < t.count; ++l)
                for (int q = p; q < tab[l].N; q += kThreads) {
                    t.xg[l][q] = xbuf(l)[q];
                    if (l > 0) t.bg[l][q] = bbuf(l)[q];
                }
    }
    if constexpr (MODE == kTailWhole) {
        // every thread runs the same scalar solve on the same LDS values
        const int lc = t.count - 1;
        const TailTab e = tab[lc];
        double u = xbuf(lc)[0];
        const double bv = bbuf(lc)[0];
        int64_t sweeps = 0;
        const int status = point_solve(u, bv, e.D, e.Dinv, t.omega, t.level_m, t.offsets, t.ra,
                                       sweeps);
        __syncthreads();  // every thread has read the coarsest values
        if (p == 0) {
            xbuf(lc)[0] = u;
            const int32_t i = *t.rec.count;
            if (i < t.rec.cap) t.rec.sweeps[i] = sweeps;
            *t.rec.count = i + 1;
            if (status != SRJ_OK && status != SRJ_ERR_NOT_CONVERGED) *t.rec.bad = status;
        }
        __syncthreads();
    }
    if constexpr (MODE != kTailDown) {
        if constexpr (MODE == kTailUp) {
            for (int l = 0; l < t.count; ++l)
                for (int q = p; q < tab[l].N; q += kThreads) {
                    xbuf(l)[q] = t.xg[l][q];
                    if (l + 1 < t.count) bbuf(l)[q] = t.bg[l][q];
                }
            __syncthreads();
        }
        for (int l = t.count - 2; l >= 0; --l) {
            // x += P e: per axis the candidates in increasing order
            const TailTab e = tab[l], ec = tab[l + 1];
            const double *ev = xbuf(l + 1);
            double *x = xbuf(l);
            for (int q = p; q < e.N; q += kThreads) {
                int ii[3];
                coords(e, q, ii[0], ii[1], ii[2]);
                const int mm[3] = {ec.n0, ec.n1, ec.n2};
                int cj[3][2];
                double cw[3][2];
                bool has[3][2];
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    if (d >= e.nd) {
                        cj[d][0] = cj[d][1] = 0;
                        cw[d][0] = 1.0;
                        cw[d][1] = 0.0;
                        has[d][0] = true;
                        has[d][1] = false;
                    } else if (ii[d] & 1) {
                        cj[d][0] = (ii[d] - 1) / 2;
                        cj[d][1] = 0;
                        cw[d][0] = 1.0;
                        cw[d][1] = 0.0;
                        has[d][0] = true;
                        has[d][1] = false;
                    } else {
                        const int J = ii[d] / 2;
                        cj[d][0] = J - 1;
                        cj[d][1] = J;
                        cw[d][0] = cw[d][1] = 0.5;
                        has[d][0] = J - 1 >= 0;
                        has[d][1] = J < mm[d];
                    }
                }
                double v = 0.0;
#pragma unroll
                for (int k2 = 0; k2 < 2; ++k2)
#pragma unroll
                    for (int k1 = 0; k1 < 2; ++k1)
#pragma unroll
                        for (int k0 = 0; k0 < 2; ++k0) {
                            const bool on = has[0][k0] && has[1][k1] && has[2][k2];
                            double wt = cw[0][k0];
                            if (e.nd > 1) wt = wt * cw[1][k1];
                            if (e.nd > 2) wt = wt * cw[2][k2];
                            const int qc = cj[0][k0] + mm[0] * (cj[1][k1] + mm[1] * cj[2][k2]);
                            const double val = ev[on ? qc : 0];
                            v = on ? v + wt * val : v;
                        }
                x[q] = x[q] + v;
            }
            __syncthreads();
            smooth(l, t.post);
        }
        for (int q = p; q < tab[0].N; q += kThreads) t.xg[0][q] = xbuf(0)[q];
    }
}

__global__ void k_mg_zero(double *__restrict__ x, int64_t n)
{
    const int64_t t = (int64_t)blockIdx.x * kMgBlock + threadIdx.x;
    if (t < n) x[t] = 0.0;
}

unsigned blocks_for(int64_t n) { return (unsigned)((n + kMgBlock - 1) / kMgBlock); }

}  // namespace

}  // namespace srj

using namespace srj;

// Levels: contexts (level 0 borrows the caller's b), per-level correction
// and right-hand-side buffers for levels >= 1.
struct srj_mg {
    int L = 0;
    int ndim = 1;
    hipStream_t stream = nullptr;   // every level's context launches here
    hipStream_t own = nullptr;      // made when the caller passes no stream
    hipEvent_t ready = nullptr;     // the caller's null-stream work -> own
    std::vector<srj_ctx *> ctx;
    std::vector<double *> xb, bb;   // index 0 unused
    double *np = nullptr;           // 2D: residual-norm partials of the finest level's last launch
    int64_t np_cap = 0;
    std::vector<int64_t> npts;
    // V-cycles replayed from graphs: one per smoothing level, starting
    // buffer of the finest level and the options the cycle depends on
    struct Graph {
        int level, pre, post, Lc, coarse_max_cycles;
        double coarse_tol;
        const double *x, *start;  // caller's x, finest iterate at the start
        double *end;              // finest iterate at the end
        hipGraphExec_t exec;
    };
    std::vector<Graph> graphs;
    // device record of the coarsest solves: count, bad status, sweeps[rec_cap]
    void *rec = nullptr;
    int32_t rec_cap = 0;
    // pinned host mirror of the record, filled by one launch after a solve
    // (rec_host_dev: its device mapping)
    void *rec_host = nullptr, *rec_host_dev = nullptr;
    std::vector<int> prepared;      // per level: resident buffers made for this many cycles
    // per level: the plan for smoothing cycles of at most two sweeps (2D
    // grids whose default plan fuses many sweeps per launch), kind 0 if none
    std::vector<SweepPlan> short_plan;
};

namespace {

// words 8-byte words of the device record into its pinned host mirror
__global__ __launch_bounds__(256) void k_mg_publish(const int64_t *__restrict__ rec,
                                                    int64_t *__restrict__ mirror, int64_t words)
{
    for (int64_t k = threadIdx.x; k < words; k += blockDim.x) mirror[k] = rec[k];
}

srj_status mg_free(srj_mg *g)
{
    if (!g) return SRJ_OK;
    if (g->stream) (void)hipStreamSynchronize(g->stream);
    else (void)hipDeviceSynchronize();
    for (srj_ctx *c : g->ctx) srj_destroy(c);
    for (double *p : g->xb) (void)hipFree(p);
    for (double *p : g->bb) (void)hipFree(p);
    (void)hipFree(g->np);
    for (auto &e : g->graphs) (void)hipGraphExecDestroy(e.exec);
    (void)hipFree(g->rec);
    (void)hipHostFree(g->rec_host);
    if (g->ready) (void)hipEventDestroy(g->ready);
    if (g->own) (void)hipStreamDestroy(g->own);
    delete g;
    return SRJ_OK;
}

struct MgRun {
    srj_mg *g;
    const srj_mg_opts *o;
    int Lc;                 // coarsest level used
    std::vector<double *> cur;
    srj_mg_result *res;
    bool graph = false;     // launches only: captured, the counters kept on the device
    int tail = -1;          // first level of the one-workgroup tail (graph mode), or -1
};

// Options of the coarsest solve: SRJ with Algorithm 1 from zero to a
// relative tolerance, clamped to the context's scheme family as srj_solve
// clamps them.
srj_solve_opts coarse_opts(const srj_ctx *c, const srj_mg_opts *o)
{
    srj_solve_opts so;
    srj_default_opts(&so);
    so.rule = SRJ_RULE_HEURISTIC;
    so.tol_mode = SRJ_TOL_RELATIVE;
    so.tol = o->coarse_tol;
    so.max_cycles = o->coarse_max_cycles;
    so.max_sweeps = 50000000;
    so.max_level = std::min(SRJ_NUM_LEVELS - 1, c->nlevels - 1);
    return so;
}

// bc = R (b - A x), through the fine residual in r (a free buffer of the
// fine level's size); xc = 0 unless xc is null
srj_status launch_restrict(const srj_ctx *c, const double *x, double *r, double *bc, double *xc,
                           hipStream_t s)
{
    const DevProblem &P = c->P;
    const int64_t m0 = P.ndim > 0 ? (P.n0 - 1) / 2 : 1, m1 = P.ndim > 1 ? (P.n1 - 1) / 2 : 1,
                  m2 = P.ndim > 2 ? (P.n2 - 1) / 2 : 1;
    const unsigned nf = (unsigned)row_grid(P.n0, P.n1, P.n2), nb = (unsigned)row_grid(m0, m1, m2);
    switch (P.ndim) {
    case 1:
        hipLaunchKernelGGL(k_mg_residual<1>, dim3(nf), dim3(kMgBlock), 0, s, P, x, r);
        hipLaunchKernelGGL(k_mg_restrict<1>, dim3(nb), dim3(kMgBlock), 0, s, r, bc, xc, P.n0, P.n1, m0, m1, m2);
        break;
    case 2:
        hipLaunchKernelGGL(k_mg_residual<2>, dim3(nf), dim3(kMgBlock), 0, s, P, x, r);
        hipLaunchKernelGGL(k_mg_restrict<2>, dim3(nb), dim3(kMgBlock), 0, s, r, bc, xc, P.n0, P.n1, m0, m1, m2);
        break;
    default:
        hipLaunchKernelGGL(k_mg_residual<3>, dim3(nf), dim3(kMgBlock), 0, s, P, x, r);
        hipLaunchKernelGGL(k_mg_restrict<3>, dim3(nb), dim3(kMgBlock), 0, s, r, bc, xc, P.n0, P.n1, m0, m1, m2);
        break;
    }
    SRJ_HIP_CHECK(hipGetLastError());
    return SRJ_OK;
}


srj_status launch_prolong(const srj_ctx *c, const double *ec, double *x, hipStream_t s)
{
    const DevProblem &P = c->P;
    const int64_t m0 = (P.n0 - 1) / 2, m1 = P.ndim > 1 ? (P.n1 - 1) / 2 : 1,
                  m2 = P.ndim > 2 ? (P.n2 - 1) / 2 : 1;
    const unsigned nb = (unsigned)row_grid(m0 + 1, P.n1, P.n2, prolong_rows(P.ndim));  // pairs
    const bool small = P.n0 * P.n1 * P.n2 < ((int64_t)1 << 31);
#define SRJ_PROLONG(ND, I)                                                                        \
    hipLaunchKernelGGL((k_prolong_add<ND, I>), dim3(nb), dim3(kMgBlock), 0, s, ec, x, P.n0, P.n1, \
                       P.n2, m0, m1, m2)
    switch (P.ndim) {
    case 1: if (small) SRJ_PROLONG(1, int32_t); else SRJ_PROLONG(1, int64_t); break;
    case 2: if (small) SRJ_PROLONG(2, int32_t); else SRJ_PROLONG(2, int64_t); break;
    default: if (small) SRJ_PROLONG(3, int32_t); else SRJ_PROLONG(3, int64_t); break;
    }
#undef SRJ_PROLONG
    SRJ_HIP_CHECK(hipGetLastError());
    return SRJ_OK;
}

// The levels from run.tail down in one launch of k_mg_tail: b of the first
// one is g->bb[run.tail], its correction goes to g->xb[run.tail].
srj_status launch_tail(MgRun &run, int level)
{
    srj_mg *g = run.g;
    const int Ls = run.tail, K = run.Lc - Ls + 1;
    TailArgs t{};
    t.count = K;
    t.pre = run.o->pre;
    t.post = run.o->post;
    int32_t off = 0;
    for (int k = 0; k < K; ++k) {
        srj_ctx *c = g->ctx[Ls + k];
        t.lv[k].P = c->P;
        t.lv[k].w = c->omega_dev + c->offsets[level];
        t.lv[k].M = (int32_t)c->factors[level].size();
        t.lv[k].off = off;
        t.xg[k] = g->xb[Ls + k];
        t.bg[k] = g->bb[Ls + k];
        off += (int32_t)(3 * g->npts[Ls + k]);
    }
    const size_t shmem = sizeof(double) * (size_t)off;
    ResidentRecord rec;
    char *base = static_cast<char *>(g->rec);
    rec.count = reinterpret_cast<int32_t *>(base);
    rec.bad = reinterpret_cast<int32_t *>(base) + 1;
    rec.sweeps = reinterpret_cast<int64_t *>(base + 8);
    rec.cap = g->rec_cap;
    srj_ctx *cc = g->ctx[run.Lc];
    const srj_solve_opts so = coarse_opts(cc, run.o);
    srj_status st = SRJ_OK;
    if (g->npts[run.Lc] == 1) {
        // a one-point coarsest grid is solved inside the one launch
        if ((st = resident_tables(cc, &so, &t.ra, &t.level_m, &t.offsets)) != SRJ_OK) return st;
        t.omega = cc->omega_dev;
        t.rec = rec;
        hipLaunchKernelGGL(k_mg_tail<kTailWhole>, dim3(1), dim3(kThreads), shmem, g->stream, t);
        SRJ_HIP_CHECK(hipGetLastError());
    } else {
        hipLaunchKernelGGL(k_mg_tail<kTailDown>, dim3(1), dim3(kThreads), shmem, g->stream, t);
        SRJ_HIP_CHECK(hipGetLastError());
        // the coarsest grid, from the zero correction the first launch left
        if ((st = resident_launch_recorded(cc, g->xb[run.Lc], &so, rec)) != SRJ_OK) return st;
        hipLaunchKernelGGL(k_mg_tail<kTailUp>, dim3(1), dim3(kThreads), shmem, g->stream, t);
        SRJ_HIP_CHECK(hipGetLastError());
    }
    run.cur[Ls] = g->xb[Ls];
    return SRJ_OK;
}

// First level of the one-workgroup tail: the finest level of at most
// tail_max_points(ndim) points below the finest grid and above the coarsest one,
// whose levels down to the coarsest fit the tail's LDS and level count; -1
// if there is none.
int tail_start(const srj_mg *g, int Lc)
{
    for (int l = 1; l < Lc; ++l) {
        if (g->npts[l] > tail_max_points(g->ndim)) continue;
        int64_t doubles = 0;
        for (int k = l; k <= Lc; ++k) doubles += 3 * g->npts[k];
        if (doubles <= (int64_t)kTailLdsDoubles && Lc - l + 1 <= kTailMaxLevels) return l;
        return -1;
    }
    return -1;
}

// The V-cycle's closing norm is formed by its last launch (the finest 2D
// level's interpolation with its only post-smoothing cycle) instead of a
// pass of its own.
bool fused_norm(const srj_mg *g, const srj_mg_opts *o, int level)
{
    const srj_ctx *c = g->ctx[0];
    return g->ndim == 2 && g->np && o->post == 1 && c->factors[level].size() <= 2 &&
           !c->profiling;
}

srj_status vcycle(MgRun &run, int l, int level, double *x0)
{
    srj_mg *g = run.g;
    if (run.graph && l == run.tail) return launch_tail(run, level);
    srj_ctx *c = g->ctx[l];
    const double frac = (double)g->npts[l] / (double)g->npts[0];
    if (l == run.Lc) {
        // coarsest grid: SRJ with Algorithm 1 from zero to coarse_tol
        double *x = g->xb[l];
        hipLaunchKernelGGL(k_mg_zero, dim3(blocks_for(g->npts[l])), dim3(kMgBlock), 0, g->stream, x,
                           g->npts[l]);
        SRJ_HIP_CHECK(hipGetLastError());
        const srj_solve_opts so = coarse_opts(c, run.o);
        if (run.graph) {
            ResidentRecord rec;
            char *base = static_cast<char *>(g->rec);
            rec.count = reinterpret_cast<int32_t *>(base);
            rec.bad = reinterpret_cast<int32_t *>(base) + 1;
            rec.sweeps = reinterpret_cast<int64_t *>(base + 8);
            rec.cap = g->rec_cap;
            run.cur[l] = x;
            return resident_launch_recorded(c, x, &so, rec);
        }
        srj_solve_result r;
        srj_status st = srj_solve(c, x, &so, &r, nullptr, nullptr);
        if (st != SRJ_OK && st != SRJ_ERR_NOT_CONVERGED) return st;
        run.cur[l] = x;
        run.res->coarse_sweeps += r.sweeps;
        run.res->work += (double)r.sweeps * frac;
        return SRJ_OK;
    }
    // the level's two buffers: level 0 the caller's x and the context's
    // ping-pong buffer, other levels their correction buffer and theirs
    int64_t sw = 0;
    auto pair_smooth = [&](int nu) -> srj_status {
        double *a = l == 0 ? x0 : g->xb[l];
        double *cur = run.cur[l];
        double *nxt = cur == a ? c->ws : a;
        // cycles of one or two sweeps run as single-sweep strips (one launch
        // per cycle either way, bit-identical), not as blocks built to fuse ten
        const SweepPlan keep = c->plan;
        if (g->short_plan[l].kind != 0 && c->factors[level].size() <= 2) c->plan = g->short_plan[l];
        srj_status st = SRJ_OK;
        for (int k = 0; k < nu && st == SRJ_OK; ++k) {
            st = run_sweeps(c, &cur, &nxt, level);
            sw += (int64_t)c->factors[level].size();
        }
        c->plan = keep;
        if (st != SRJ_OK) return st;
        run.cur[l] = cur;
        return SRJ_OK;
    };
    // 2D levels whose cycles have at most two sweeps: the last pre-smoothing
    // cycle, the fine residual of its result and its restriction in one launch
    const int M = (int)c->factors[level].size();
    const bool fuse = g->ndim == 2 && run.o->pre > 0 && M <= 2 && !c->profiling;
    srj_status st = pair_smooth(fuse ? run.o->pre - 1 : run.o->pre);
    if (st != SRJ_OK) return st;
    // the coarse correction starts from zero (the tail starts its own)
    double *xz = run.graph && l + 1 == run.tail ? nullptr : g->xb[l + 1];
    if (fuse) {
        double *a = l == 0 ? x0 : g->xb[l];
        double *cur = run.cur[l];
        double *nxt = cur == a ? c->ws : a;
        SRJ_HIP_CHECK(launch_wave2d_rr(c->P, M, cur, nxt, g->bb[l + 1], xz,
                                       c->omega_dev + c->offsets[level], g->stream));
        run.cur[l] = nxt;
        sw += M;
    } else {
        // the level's other buffer holds nothing live until the post-smoothing
        double *a = l == 0 ? x0 : g->xb[l];
        double *spare = run.cur[l] == a ? c->ws : a;
        if ((st = launch_restrict(c, run.cur[l], spare, g->bb[l + 1], xz, g->stream)) != SRJ_OK)
            return st;
    }
    double *xc = g->xb[l + 1];
    run.cur[l + 1] = xc;
    if ((st = vcycle(run, l + 1, level, x0)) != SRJ_OK) return st;
    if (g->ndim == 2 && run.o->post > 0 && M <= 2 && !c->profiling) {
        // the interpolation and the first post-smoothing cycle in one launch
        double *a = l == 0 ? x0 : g->xb[l];
        double *cur = run.cur[l];
        double *nxt = cur == a ? c->ws : a;
        double *part = l == 0 && fused_norm(g, run.o, level) ? g->np : nullptr;
        SRJ_HIP_CHECK(launch_wave2d_pp(c->P, M, cur, nxt, run.cur[l + 1],
                                       c->omega_dev + c->offsets[level], g->stream, part));
        run.cur[l] = nxt;
        sw += M;
        if ((st = pair_smooth(run.o->post - 1)) != SRJ_OK) return st;
    } else {
        if ((st = launch_prolong(c, run.cur[l + 1], run.cur[l], g->stream)) != SRJ_OK) return st;
        if ((st = pair_smooth(run.o->post)) != SRJ_OK) return st;
    }
    if (!run.graph) {
        if (l == 0) run.res->sweeps += sw;
        run.res->work += (double)sw * frac;
    }
    return SRJ_OK;
}

// Most V-cycle graphs kept per multigrid context: 25 smoothing levels times
// two starting buffers for one x and one set of options.
constexpr size_t kMaxGraphs = 64;

// V-cycles can be replayed from graphs when the coarsest grid is solved in
// one workgroup and nothing times the launches.
bool graphable(const srj_mg *g, int Lc)
{
    const srj_ctx *c = g->ctx[Lc];
    if (!c->resident || !resident_fits(c->P)) return false;
    for (int l = 0; l <= Lc; ++l)
        if (g->ctx[l]->profiling) return false;
    return true;
}

// The V-cycle at smoothing level `level` from the finest iterate run.cur[0],
// captured once per (level, starting buffer, options) and replayed; leaves
// run.cur[0] at the finest iterate it ends on.
srj_status vcycle_graph(MgRun &run, int level, double *x)
{
    srj_mg *g = run.g;
    const srj_mg_opts *o = run.o;
    double *start = run.cur[0];
    for (const auto &e : g->graphs)
        if (e.level == level && e.pre == o->pre && e.post == o->post && e.Lc == run.Lc &&
            e.coarse_max_cycles == o->coarse_max_cycles && e.coarse_tol == o->coarse_tol &&
            e.x == x && e.start == start) {
            SRJ_HIP_CHECK(hipGraphLaunch(e.exec, g->stream));
            run.cur[0] = e.end;
            return SRJ_OK;
        }
    SRJ_HIP_CHECK(hipStreamBeginCapture(g->stream, hipStreamCaptureModeThreadLocal));
    const srj_status st = vcycle(run, 0, level, x);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(g->stream, &graph);
    if (st != SRJ_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return st;
    }
    if (e != hipSuccess) return fail(SRJ_ERR_HIP, std::string("V-cycle capture: ") + hipGetErrorString(e));
    hipGraphExec_t exec = nullptr;
    const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ei != hipSuccess) return fail(SRJ_ERR_HIP, std::string("V-cycle graph: ") + hipGetErrorString(ei));
    if (g->graphs.size() >= kMaxGraphs) {
        // a bounded cache (callers that pass a new x on every solve would
        // otherwise grow it without end): the oldest entry goes, once the
        // stream has finished every replay of it
        SRJ_HIP_CHECK(hipStreamSynchronize(g->stream));
        (void)hipGraphExecDestroy(g->graphs.front().exec);
        g->graphs.erase(g->graphs.begin());
    }
    g->graphs.push_back({level, o->pre, o->post, run.Lc, o->coarse_max_cycles, o->coarse_tol, x,
                         start, run.cur[0], exec});
    SRJ_HIP_CHECK(hipGraphLaunch(exec, g->stream));
    return SRJ_OK;
}

// Device record and coarsest-context buffers for V-cycles replayed from
// graphs; drops the graphs when the record moves.
srj_status prepare_graphs(srj_mg *g, const srj_mg_opts *o, int Lc)
{
    if (g->rec_cap < o->max_vcycles) {
        for (auto &e : g->graphs) (void)hipGraphExecDestroy(e.exec);
        g->graphs.clear();
        (void)hipFree(g->rec);
        (void)hipHostFree(g->rec_host);
        g->rec = g->rec_host = g->rec_host_dev = nullptr;
        g->rec_cap = 0;
        const size_t bytes = 8 + sizeof(int64_t) * (size_t)o->max_vcycles;
        if (hipMalloc(&g->rec, bytes) != hipSuccess || hipHostMalloc(&g->rec_host, bytes, 0) != hipSuccess ||
            hipHostGetDevicePointer(&g->rec_host_dev, g->rec_host, 0) != hipSuccess) {
            (void)hipFree(g->rec);
            (void)hipHostFree(g->rec_host);
            g->rec = g->rec_host = g->rec_host_dev = nullptr;
            return fail(SRJ_ERR_NOMEM, "allocation failed for the multigrid record");
        }
        g->rec_cap = o->max_vcycles;
    }
    if (g->prepared[Lc] < o->coarse_max_cycles) {
        // the graphs hold the buffers' addresses: reallocation drops them
        for (auto &e : g->graphs) (void)hipGraphExecDestroy(e.exec);
        g->graphs.clear();
        srj_status st = resident_prepare(g->ctx[Lc], o->coarse_max_cycles);
        if (st != SRJ_OK) return st;
        g->prepared[Lc] = o->coarse_max_cycles;
    }
    // hipMemsetAsync stays outside the captured graphs
    SRJ_HIP_CHECK(hipMemsetAsync(g->rec, 0, 8, g->stream));
    return SRJ_OK;
}

srj_status validate_mg_opts(const srj_mg_opts *o)
{
    if (!o) return fail(SRJ_ERR_INVALID, "opts is NULL");
    if (o->rule != SRJ_RULE_HEURISTIC && o->rule != SRJ_RULE_FIXED)
        return fail(SRJ_ERR_INVALID, "rule must be SRJ_RULE_HEURISTIC or SRJ_RULE_FIXED");
    if (o->max_level < 0 || o->max_level >= SRJ_NUM_LEVELS)
        return fail(SRJ_ERR_INVALID, "max_level outside 0..24");
    if (o->start_level < 0 || o->start_level > o->max_level)
        return fail(SRJ_ERR_INVALID, "start_level outside 0..max_level");
    if (o->pre < 0 || o->post < 0 || o->pre > 1000 || o->post > 1000)
        return fail(SRJ_ERR_INVALID, "pre and post must be 0..1000");
    if (o->max_levels < 2) return fail(SRJ_ERR_INVALID, "max_levels must be >= 2");
    if (!(o->coarse_tol > 0.0)) return fail(SRJ_ERR_INVALID, "coarse_tol must be > 0");
    if (o->coarse_max_cycles < 1) return fail(SRJ_ERR_INVALID, "coarse_max_cycles must be >= 1");
    if (o->tol_mode != SRJ_TOL_RELATIVE && o->tol_mode != SRJ_TOL_ABSOLUTE)
        return fail(SRJ_ERR_INVALID, "tol_mode must be relative or absolute");
    if (!(o->tol > 0.0)) return fail(SRJ_ERR_INVALID, "tol must be > 0");
    if (o->max_vcycles < 1) return fail(SRJ_ERR_INVALID, "max_vcycles must be >= 1");
    return SRJ_OK;
}

}  // namespace

extern "C" {

void srj_mg_default_opts(srj_mg_opts *o)
{
    if (!o) return;
    memset(o, 0, sizeof(*o));
    o->rule = SRJ_RULE_HEURISTIC;
    o->start_level = 0;
    o->max_level = SRJ_NUM_LEVELS - 1;
    o->pre = 1;
    o->post = 1;
    o->max_levels = kMgMaxLevels;
    o->coarse_tol = 1e-8;
    o->coarse_max_cycles = 1000;
    o->tol_mode = SRJ_TOL_RELATIVE;
    o->tol = 1e-10;
    o->max_vcycles = 200;
}

srj_status srj_mg_setup(const srj_problem *p, void *hip_stream, srj_mg **out)
{
    if (!out) return fail(SRJ_ERR_INVALID, "out is NULL");
    *out = nullptr;
    srj_status st = validate_problem(p);
    if (st != SRJ_OK) return st;
    if (p->diag || p->face[0] || p->face[1] || p->face[2])
        return fail(SRJ_ERR_UNSUPPORTED, "multigrid takes constant-coefficient stencils");
    int64_t n[3] = {p->n[0], p->n[1], p->n[2]};
    std::vector<std::array<int64_t, 3>> dims;
    for (;;) {
        dims.push_back({n[0], n[1], n[2]});
        if ((int)dims.size() >= kMgMaxLevels) break;
        bool can = true;
        for (int d = 0; d < p->ndim; ++d)
            if (n[d] < 3 || n[d] % 2 == 0) can = false;
        if (!can) break;
        for (int d = 0; d < p->ndim; ++d) n[d] = (n[d] - 1) / 2;
    }
    if (dims.size() < 2)
        return fail(SRJ_ERR_UNSUPPORTED, "grid cannot be coarsened (every active size must be odd and >= 3)");
    srj_mg *g = new srj_mg();
    g->L = (int)dims.size();
    g->ndim = p->ndim;
    g->stream = static_cast<hipStream_t>(hip_stream);
    if (!g->stream) {
        // V-cycles are captured into graphs, which the null stream cannot
        // do: the levels run on a stream of their own, ordered after the
        // caller's null-stream work at the start of every solve
        if (hipStreamCreateWithFlags(&g->own, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&g->ready, hipEventDisableTiming) != hipSuccess) {
            mg_free(g);
            return fail(SRJ_ERR_HIP, "multigrid stream");
        }
        g->stream = g->own;
    }
    g->prepared.assign(g->L, 0);
    g->short_plan.assign(g->L, SweepPlan{});
    g->ctx.assign(g->L, nullptr);
    g->xb.assign(g->L, nullptr);
    g->bb.assign(g->L, nullptr);
    g->npts.assign(g->L, 0);
    srj_problem q = *p;
    for (int l = 0; l < g->L; ++l) {
        for (int d = 0; d < 3; ++d) q.n[d] = dims[l][d];
        g->npts[l] = q.n[0] * q.n[1] * q.n[2];
        if (l > 0) {
            // rediscretisation on the doubled spacing: couplings and diagonal / 4
            for (int d = 0; d < 3; ++d) q.cconst[d] = q.cconst[d] / 4.0;
            q.dconst = q.dconst / 4.0;
            const size_t bytes = sizeof(double) * (size_t)g->npts[l];
            if (hipMalloc(&g->xb[l], bytes) != hipSuccess || hipMalloc(&g->bb[l], bytes) != hipSuccess) {
                mg_free(g);
                return fail(SRJ_ERR_NOMEM, "hipMalloc failed for a multigrid level");
            }
            q.b = g->bb[l];
        }
        srj_ctx *c = nullptr;
        st = srj_setup(&q, g->stream, &c);
        if (st != SRJ_OK) {
            const std::string msg = srj_last_error();
            mg_free(g);
            return fail(st, "multigrid level " + std::to_string(l) + ": " + msg);
        }
        g->ctx[l] = c;
        if (c->P.ndim == 2 && c->plan.kind != 0 && c->plan.T > 2) {
            SweepPlan sp;
            sp.kind = 5;  // wavefront strips of 8 rows, up to two sweeps per launch
            sp.by = 8;
            sp.T = 2;
            sp.occ = 1;
            if (fused_supported(c->P, sp)) g->short_plan[l] = sp;
        }
    }
    if (g->ndim == 2) {
        const DevProblem &P0 = g->ctx[0]->P;
        g->np_cap = std::max(pp_items(P0, 1), pp_items(P0, 2));
        if (hipMalloc(&g->np, sizeof(double) * (size_t)g->np_cap) != hipSuccess) {
            g->np = nullptr;
            mg_free(g);
            return fail(SRJ_ERR_NOMEM, "hipMalloc failed for the multigrid norm partials");
        }
    }
    // the tail launches take up to kTailLdsDoubles doubles of dynamic LDS
    const void *tails[3] = {reinterpret_cast<const void *>(&k_mg_tail<kTailDown>),
                            reinterpret_cast<const void *>(&k_mg_tail<kTailUp>),
                            reinterpret_cast<const void *>(&k_mg_tail<kTailWhole>)};
    for (const void *f : tails) {
        const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize,
                                                 (int)(sizeof(double) * kTailLdsDoubles));
        if (e != hipSuccess) {
            mg_free(g);
            return fail(SRJ_ERR_HIP, std::string("multigrid tail LDS: ") + hipGetErrorString(e));
        }
    }
    *out = g;
    return SRJ_OK;
}

static srj_status mg_solve_run(srj_mg *g, double *x, const srj_mg_opts *o, srj_mg_result *res,
                               int32_t *levels_out, double *norms_out);

srj_status srj_mg_solve(srj_mg *g, double *x, const srj_mg_opts *o, srj_mg_result *res,
                        int32_t *levels_out, double *norms_out)
{
    // the per-V-cycle log (SRJ_LOG) needs the histories: the solve then
    // fills arrays of its own where the caller passes none
    if (!log_enabled() || !g || !x || !o || !res || o->max_vcycles < 1 ||
        o->max_vcycles > (1 << 24))
        return mg_solve_run(g, x, o, res, levels_out, norms_out);
    std::vector<int32_t> lv;
    std::vector<double> nv;
    if (!levels_out) {
        lv.resize((size_t)o->max_vcycles);
        levels_out = lv.data();
    }
    if (!norms_out) {
        nv.resize((size_t)o->max_vcycles + 1);
        norms_out = nv.data();
    }
    const srj_status st = mg_solve_run(g, x, o, res, levels_out, norms_out);
    if (st == SRJ_OK || st == SRJ_ERR_NOT_CONVERGED || st == SRJ_ERR_NONFINITE) {
        // finest-grid smoothing sweeps of a V-cycle at each smoothing level
        const std::vector<int32_t> &lm = g->ctx[0]->levelM;
        std::vector<int32_t> per(lm.size());
        for (size_t l = 0; l < lm.size(); ++l) per[l] = (o->pre + o->post) * lm[l];
        log_cycles("mg", st, res->vcycles, levels_out, per.data(), (int)per.size(), norms_out,
                   res->sweeps, res->r0, res->r_final);
    }
    return st;
}

static srj_status mg_solve_run(srj_mg *g, double *x, const srj_mg_opts *o, srj_mg_result *res,
                               int32_t *levels_out, double *norms_out)
{
    if (!g || !x || !res) return fail(SRJ_ERR_INVALID, "NULL argument");
    srj_status st = validate_mg_opts(o);
    if (st != SRJ_OK) return st;
    srj_ctx *c0 = g->ctx[0];
    st = check_device_array(x, sizeof(double) * (size_t)g->npts[0], c0->device, "x");
    if (st != SRJ_OK) return st;
    memset(res, 0, sizeof(*res));
    MgRun run{g, o, std::min(g->L, o->max_levels) - 1, std::vector<double *>(g->L, nullptr), res};
    res->levels = run.Lc + 1;
    run.cur[0] = x;
    if (g->own) {
        SRJ_HIP_CHECK(hipEventRecord(g->ready, nullptr));
        SRJ_HIP_CHECK(hipStreamWaitEvent(g->own, g->ready, 0));
    }
    run.graph = graphable(g, run.Lc);
    if (run.graph && (st = prepare_graphs(g, o, run.Lc)) != SRJ_OK) return st;
    if (run.graph) run.tail = tail_start(g, run.Lc);
    std::vector<int> vlevels;

    double norm0 = 0.0;
    if ((st = residual_norm(c0, x, &norm0)) != SRJ_OK) return st;
    res->r0 = norm0;
    res->r_final = norm0;
    if (norms_out) norms_out[0] = norm0;
    const double target = o->tol_mode == SRJ_TOL_RELATIVE ? o->tol * norm0 : o->tol;
    srj_status status = SRJ_ERR_NOT_CONVERGED;
    int level = o->start_level;
    double prev = norm0;
    if (!std::isfinite(norm0)) {
        status = SRJ_ERR_NONFINITE;
    } else if (norm0 == 0.0 || norm0 < target) {
        res->converged = 1;
        status = SRJ_OK;
    } else {
        for (int v = 0; v < o->max_vcycles; ++v) {
            const int lv = o->rule == SRJ_RULE_FIXED ? o->start_level : level;
            st = run.graph ? vcycle_graph(run, lv, x) : vcycle(run, 0, lv, x);
            if (st != SRJ_OK) return st;
            vlevels.push_back(lv);
            double norm = 0.0;
            if (fused_norm(g, o, lv)) {
                const int64_t n = pp_items(c0->P, (int)c0->factors[lv].size());
                if ((st = fold_norm(c0, g->np, n, &norm)) != SRJ_OK) return st;
            } else if ((st = residual_norm(c0, run.cur[0], &norm)) != SRJ_OK) {
                return st;
            }
            if (levels_out) levels_out[v] = lv;
            if (norms_out) norms_out[v + 1] = norm;
            res->vcycles = v + 1;
            res->final_level = lv;
            res->r_final = norm;
            if (!std::isfinite(norm)) {
                status = SRJ_ERR_NONFINITE;
                break;
            }
            if (norm < target) {
                res->converged = 1;
                status = SRJ_OK;
                break;
            }
            // Algorithm 1 on the V-cycle ratios picks the next smoothing scheme
            const double ratio = norm / prev;
            prev = norm;
            if (o->rule == SRJ_RULE_HEURISTIC) level = next_level(o->rule, level, ratio, o->max_level);
        }
    }
    if (run.cur[0] != x)
        SRJ_HIP_CHECK(hipMemcpyAsync(x, run.cur[0], sizeof(double) * (size_t)g->npts[0],
                                     hipMemcpyDeviceToDevice, g->stream));
    const bool recorded = run.graph && !vlevels.empty();
    if (recorded) {
        // the record's head and one count per V-cycle into the pinned mirror
        const int64_t words = 1 + (int64_t)std::min<size_t>(vlevels.size(), (size_t)g->rec_cap);
        hipLaunchKernelGGL(k_mg_publish, dim3(1), dim3(256), 0, g->stream,
                           static_cast<const int64_t *>(g->rec),
                           static_cast<int64_t *>(g->rec_host_dev), words);
        SRJ_HIP_CHECK(hipGetLastError());
    }
    SRJ_HIP_CHECK(hipStreamSynchronize(g->stream));
    if (recorded) {
        // the counters in the order the launches made them: per V-cycle the
        // coarsest solve, then the levels from the coarsest up
        int32_t head[2] = {0, 0};
        memcpy(head, g->rec_host, sizeof(head));
        if (head[0] != (int32_t)vlevels.size())
            return fail(SRJ_ERR_HIP, "multigrid record holds a different number of coarsest solves");
        std::vector<int64_t> cs(vlevels.size());
        memcpy(cs.data(), static_cast<const char *>(g->rec_host) + 8, sizeof(int64_t) * cs.size());
        for (size_t v = 0; v < vlevels.size(); ++v) {
            res->coarse_sweeps += cs[v];
            res->work += (double)cs[v] * ((double)g->npts[run.Lc] / (double)g->npts[0]);
            for (int l = run.Lc - 1; l >= 0; --l) {
                const int64_t sw = (int64_t)(o->pre + o->post) *
                                   (int64_t)g->ctx[l]->factors[vlevels[v]].size();
                if (l == 0) res->sweeps += sw;
                res->work += (double)sw * ((double)g->npts[l] / (double)g->npts[0]);
            }
        }
        if (head[1] != 0) return fail((srj_status)head[1], "coarsest-grid solve failed");
    }
    if (status == SRJ_ERR_NONFINITE) return fail(status, "non-finite residual norm");
    if (status == SRJ_ERR_NOT_CONVERGED) return fail(status, "V-cycle cap reached");
    return SRJ_OK;
}

srj_status srj_mg_destroy(srj_mg *g) { return mg_free(g); }

}  // extern "C"
