// Cycle-end residual r = b - A x and its squared L2 norm (Islam & Wang,
// arXiv 2011.06636: the L2 residual norm drives the scheme choice of
// section 3 and the stopping tests of section 4, e.g. Eq. (27)).
//
// The per-point residual uses the same expression order as the sweeps.  The
// sum of squares is deterministic: each thread adds its column's rows of a
// unit in row order, then wave shuffles and an LDS tree inside the
// workgroup give one partial per workgroup, and one workgroup folds the
// partials in a fixed order.  No floating-point atomics.
#include "internal.h"
#include "rowband.h"

#pragma clang fp contract(off)

namespace srj {

namespace {

constexpr int kBlock = 256;
static_assert(kBlock == kRowUnit, "one residual workgroup per row unit");
constexpr int kFinal = 1024;

// Fixed-order sum over the 64 lanes of a wave, result in lane 0.
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

template <int NW>
__device__ __forceinline__ double block_sum(double v, double *lds)
{
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) lds[wave] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0) {
        t = lds[0];
#pragma unroll
        for (int i = 1; i < NW; ++i) t += lds[i];
    }
    return t;
}

// One unit (256 columns of kNormRows rows, rowband.h) per workgroup: each
// thread forms the residuals of its column's rows, all loads of all rows in
// flight together, and sums their squares in row order; the workgroup's sum
// goes to slot blockIdx.x (zero for a workgroup without a unit), so the fold
// adds the same partials in the same order for a given grid.  Neighbour
// values and couplings are loaded from clamped indices unconditionally and a
// select drops the terms of ghost neighbours, leaving the expression's
// operations and order unchanged: with a branch around each neighbour's load
// the compiler waited for every load in turn.
template <int ND>
__global__ __launch_bounds__(kBlock) void k_residual_sumsq(DevProblem P,
                                                           const double *__restrict__ x,
                                                           double *__restrict__ partials)
{
    __shared__ double lds[kBlock / 64];
    int64_t xb, y, i2;
    int ny;
    if (!row_unit(blockIdx.x, P.n0, P.n1, P.n2, kNormRows, xb, y, ny, i2)) {
        if (threadIdx.x == 0) partials[blockIdx.x] = 0.0;
        return;  // whole workgroup
    }
    const int64_t i0 = xb * kBlock + threadIdx.x;
    const bool in = i0 < P.n0;
    const int64_t n0 = P.n0, n1 = P.n1, n2 = P.n2;
    const int64_t s1 = n0, s2 = n0 * n1;
    const int64_t c0 = in ? i0 : n0 - 1;
    const bool h0 = c0 > 0, h1 = c0 < n0 - 1;
    const bool h4 = ND >= 3 && i2 > 0, h5 = ND >= 3 && i2 < n2 - 1;
    double rr[kNormRows];
#pragma unroll
    for (int j = 0; j < kNormRows; ++j) {
        // rows past the unit's last repeat its first row and are not summed
        const int64_t i1 = y + (j < ny ? j : 0);
        const int64_t p = c0 + s1 * i1 + s2 * i2;
        const bool h2 = ND >= 2 && i1 > 0, h3 = ND >= 2 && i1 < n1 - 1;
        const int64_t q0 = h0 ? p - 1 : p, q1 = h1 ? p + 1 : p;
        const int64_t q2 = h2 ? p - s1 : p, q3 = h3 ? p + s1 : p;
        const int64_t q4 = h4 ? p - s2 : p, q5 = h5 ? p + s2 : p;
        const double xc = x[p];
        double s = (P.diag ? P.diag[p] : P.dconst) * xc;
        {
            const double v0 = x[q0], v1 = x[q1];
            const double f0 = P.face[0] ? P.face[0][q0] : P.c[0];
            const double f1 = P.face[0] ? P.face[0][p] : P.c[0];
            s = h0 ? s - f0 * v0 : s;
            s = h1 ? s - f1 * v1 : s;
        }
        if (ND >= 2) {
            const double v2 = x[q2], v3 = x[q3];
            const double f2 = P.face[1] ? P.face[1][q2] : P.c[1];
            const double f3 = P.face[1] ? P.face[1][p] : P.c[1];
            s = h2 ? s - f2 * v2 : s;
            s = h3 ? s - f3 * v3 : s;
        }
        if (ND >= 3) {
            const double v4 = x[q4], v5 = x[q5];
            const double f4 = P.face[2] ? P.face[2][q4] : P.c[2];
            const double f5 = P.face[2] ? P.face[2][p] : P.c[2];
            s = h4 ? s - f4 * v4 : s;
            s = h5 ? s - f5 * v5 : s;
        }
        const double r = P.b[p] - s;
        rr[j] = (in && j < ny) ? r * r : 0.0;
    }
    double acc = rr[0];
#pragma unroll
    for (int j = 1; j < kNormRows; ++j) acc += rr[j];
    const double t = block_sum<kBlock / 64>(acc, lds);
    if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

// General sparse matrix: the same per-row expression as k_sweep_ell.
__global__ __launch_bounds__(kBlock) void k_residual_ell(DevProblem P, const double *__restrict__ x,
                                                         double *__restrict__ partials)
{
    __shared__ double lds[kBlock / 64];
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    double rr = 0.0;
    if (p < P.n0) {
        double s = P.diag[p] * x[p];
        const int len = P.ell_len[p];
        for (int j = 0; j < len; ++j)
            s = s + P.ell_val[(int64_t)j * P.n0 + p] * x[P.ell_col[(int64_t)j * P.n0 + p]];
        const double r = P.b[p] - s;
        rr = r * r;
    }
    const double t = block_sum<kBlock / 64>(rr, lds);
    if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

// One block: thread i sums partials i, i + 1024, ... in order, then a fixed
// tree; ROOT writes the square root of the sum instead of the sum.
template <bool ROOT>
__global__ __launch_bounds__(kFinal) void k_fold(const double *__restrict__ partials, int64_t n,
                                                 double *__restrict__ out)
{
    __shared__ double lds[kFinal / 64];
    double v = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += kFinal) v += partials[i];
    const double t = block_sum<kFinal / 64>(v, lds);
    if (threadIdx.x == 0) *out = ROOT ? sqrt(t) : t;
}

template <int ND>
void launch_stencil_residual(const DevProblem &P, const double *x, double *partials, dim3 grid,
                             hipStream_t s)
{
    hipLaunchKernelGGL(k_residual_sumsq<ND>, grid, dim3(kBlock), 0, s, P, x, partials);
}

dim3 residual_grid(const DevProblem &P)
{
    return dim3((unsigned)row_grid(P.n0, P.n1, P.n2, kNormRows));
}

}  // namespace

hipError_t launch_fold(ReduceScratch &rs, int64_t nblocks, hipStream_t s)
{
    if (nblocks > rs.capacity) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_fold<false>, dim3(1), dim3(kFinal), 0, s, rs.partials, nblocks, rs.sum);
    return hipGetLastError();
}

int64_t residual_blocks(const DevProblem &P)
{
    return row_grid(P.n0, P.n1, P.n2, kNormRows);  // one partial per workgroup
}

hipError_t launch_residual_sumsq(const DevProblem &P, const double *x, ReduceScratch &rs,
                                 hipStream_t s)
{
    const dim3 grid = residual_grid(P);
    const int64_t nb = residual_blocks(P);  // partials: one per workgroup
    if (nb > rs.capacity) return hipErrorInvalidValue;
    if (P.ell_len) {
        hipLaunchKernelGGL(k_residual_ell, grid, dim3(kBlock), 0, s, P, x, rs.partials);
    } else {
    switch (P.ndim) {
    case 1: launch_stencil_residual<1>(P, x, rs.partials, grid, s); break;
    case 2: launch_stencil_residual<2>(P, x, rs.partials, grid, s); break;
    default: launch_stencil_residual<3>(P, x, rs.partials, grid, s); break;
    }
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_fold<false>, dim3(1), dim3(kFinal), 0, s, rs.partials, nb, rs.sum);
    return hipGetLastError();
}

hipError_t launch_residual_norm_into(const DevProblem &P, const double *x, double *partials,
                                     int64_t capacity, double *norm_out, hipStream_t s)
{
    const dim3 grid = residual_grid(P);
    const int64_t nb = residual_blocks(P);  // partials: one per workgroup
    if (nb > capacity || P.ell_len) return hipErrorInvalidValue;
    switch (P.ndim) {
    case 1: launch_stencil_residual<1>(P, x, partials, grid, s); break;
    case 2: launch_stencil_residual<2>(P, x, partials, grid, s); break;
    default: launch_stencil_residual<3>(P, x, partials, grid, s); break;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_fold<true>, dim3(1), dim3(kFinal), 0, s, partials, nb, norm_out);
    return hipGetLastError();
}

}  // namespace srj
