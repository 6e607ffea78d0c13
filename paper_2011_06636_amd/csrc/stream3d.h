// 3D relaxed Jacobi sweep streamed along the slowest axis.
//
// One sweep of Islam & Wang (arXiv 2011.06636) section 2, Eq. 3 in residual
// form on a 7-point stencil with constant or per-face couplings and a
// constant or per-point diagonal, in the fixed order
//     s = D_p u_p - c0lo u_{p-e0} - c0hi u_{p+e0} - c1lo u_{p-e1} - c1hi u_{p+e1}
//                 - c2lo u_{p-e2} - c2hi u_{p+e2}
//     u'_p = u_p + w (Dinv_p (f_p - s))
// with no fused multiply-add (bit-identical to the one-sweep kernels).
//
// A block covers 64 x 4 points of a plane and walks ZC planes along axis 2:
// the lower/centre/upper values along axis 2 and the lower axis-2 coupling
// stay in registers from one plane to the next, so each value of u, f, D,
// 1/D and each coupling is loaded once per point; in-plane neighbours are
// re-read through the caches.  Value policy V as in tile2d.h.
#pragma once

#include "internal.h"

#pragma clang fp contract(off)

namespace srj {

template <class A>
struct Stencil3 {
    int64_t n0, n1, n2;
    A c[3];
    const A *face[3];  // nullptr: constant coupling c[d]
    A dconst, dinvconst;
    const A *diag;     // nullptr: constant diagonal
    const A *dinv;
};

// One thread: column (i0, i1), planes z0 .. z0 + ZC - 1.
template <class V, int ZC>
__device__ __forceinline__ void stream3d_run(const Stencil3<typename V::A> &S,
                                             const typename V::T *__restrict__ x,
                                             typename V::T *__restrict__ xo,
                                             const typename V::T *__restrict__ b,
                                             typename V::A w, int64_t i0, int64_t i1, int64_t z0)
{
    using A = typename V::A;
    const int64_t zend = z0 + ZC < S.n2 ? z0 + ZC : S.n2;
    const int64_t s1 = S.n0, s2 = S.n0 * S.n1;
    int64_t p = i0 + s1 * i1 + s2 * z0;
    const bool has_l0 = i0 > 0, has_h0 = i0 < S.n0 - 1;
    const bool has_l1 = i1 > 0, has_h1 = i1 < S.n1 - 1;
    A xm = z0 > 0 ? V::load(x[p - s2]) : A(0);
    A xc = V::load(x[p]);
    A f2m = z0 > 0 ? (S.face[2] ? S.face[2][p - s2] : S.c[2]) : A(0);
    for (int64_t z = z0; z < zend; ++z, p += s2) {
        const A xp = z + 1 < S.n2 ? V::load(x[p + s2]) : A(0);
        A s = (S.diag ? S.diag[p] : S.dconst) * xc;
        if (has_l0) s = s - (S.face[0] ? S.face[0][p - 1] : S.c[0]) * V::load(x[p - 1]);
        if (has_h0) s = s - (S.face[0] ? S.face[0][p] : S.c[0]) * V::load(x[p + 1]);
        if (has_l1) s = s - (S.face[1] ? S.face[1][p - s1] : S.c[1]) * V::load(x[p - s1]);
        if (has_h1) s = s - (S.face[1] ? S.face[1][p] : S.c[1]) * V::load(x[p + s1]);
        if (z > 0) s = s - f2m * xm;
        const A f2c = S.face[2] ? S.face[2][p] : S.c[2];
        if (z + 1 < S.n2) s = s - f2c * xp;
        const A r = V::load(b[p]) - s;
        const A t = (S.diag ? S.dinv[p] : S.dinvconst) * r;
        xo[p] = V::store(xc + w * t);
        xm = xc;
        xc = xp;
        f2m = f2c;
    }
}

template <class V, int ZC>
__global__ __launch_bounds__(256) void k_stream3d(Stencil3<typename V::A> S,
                                                  const typename V::T *__restrict__ x,
                                                  typename V::T *__restrict__ xo,
                                                  const typename V::T *__restrict__ b,
                                                  const typename V::A *__restrict__ wp)
{
    const int64_t i0 = (int64_t)blockIdx.x * 64 + threadIdx.x;
    const int64_t i1 = (int64_t)blockIdx.y * 4 + threadIdx.y;
    if (i0 >= S.n0 || i1 >= S.n1) return;  // no barriers below
    stream3d_run<V, ZC>(S, x, xo, b, wp[0], i0, i1, (int64_t)blockIdx.z * ZC);
}

template <class V, int ZC>
hipError_t launch_stream3d(const Stencil3<typename V::A> &S, const typename V::T *x,
                           typename V::T *xo, const typename V::T *b,
                           const typename V::A *w_dev, hipStream_t s)
{
    const dim3 grid((unsigned)((S.n0 + 63) / 64), (unsigned)((S.n1 + 3) / 4),
                    (unsigned)((S.n2 + ZC - 1) / ZC));
    hipLaunchKernelGGL((k_stream3d<V, ZC>), grid, dim3(64, 4), 0, s, S, x, xo, b, w_dev);
    return hipGetLastError();
}

// z-chunk lengths available to plans (kind 3)
#define SRJ_3D_CHUNKS(X) X(8) X(16) X(32) X(64)

}  // namespace srj
