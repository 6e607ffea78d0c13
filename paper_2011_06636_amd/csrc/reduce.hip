// Cycle-end residual r = b - A x and its squared L2 norm (Islam & Wang,
// arXiv 2011.06636: the L2 residual norm drives the scheme choice of
// section 3 and the stopping tests of section 4, e.g. Eq. (27)).
//
// The per-point residual uses the same expression order as the sweeps.  The
// sum of squares is deterministic: wave shuffles and an LDS tree inside each
// block, one partial per block, then one block folds the partials in a fixed
// order.  No floating-point atomics.
#include "internal.h"

#pragma clang fp contract(off)

namespace srj {

namespace {

constexpr int kBlock = 256;
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

template <int ND>
__global__ __launch_bounds__(kBlock) void k_residual_sumsq(DevProblem P,
                                                           const double *__restrict__ x,
                                                           double *__restrict__ partials)
{
    __shared__ double lds[kBlock / 64];
    const int64_t i0 = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t i1 = blockIdx.y, i2 = blockIdx.z;
    double rr = 0.0;
    if (i0 < P.n0) {
        const int64_t s1 = P.n0, s2 = P.n0 * P.n1;
        const int64_t p = i0 + s1 * i1 + s2 * i2;
        double s = (P.diag ? P.diag[p] : P.dconst) * x[p];
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
        rr = r * r;
    }
    const double t = block_sum<kBlock / 64>(rr, lds);
    if (threadIdx.x == 0)
        partials[blockIdx.x + (int64_t)gridDim.x * (blockIdx.y + (int64_t)gridDim.y * blockIdx.z)] = t;
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
    return dim3((unsigned)((P.n0 + kBlock - 1) / kBlock), (unsigned)P.n1, (unsigned)P.n2);
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
    return ((P.n0 + kBlock - 1) / kBlock) * P.n1 * P.n2;
}

hipError_t launch_residual_sumsq(const DevProblem &P, const double *x, ReduceScratch &rs,
                                 hipStream_t s)
{
    const dim3 grid = residual_grid(P);
    const int64_t nb = (int64_t)grid.x * grid.y * grid.z;
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
    const int64_t nb = (int64_t)grid.x * grid.y * grid.z;
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
