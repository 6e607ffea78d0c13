// (A u)_p for the kernels that keep a whole small grid in LDS.
#pragma once

#include "internal.h"

#pragma clang fp contract(off)

namespace srj {

// The library's fixed order (Islam & Wang, arXiv 2011.06636, section 2,
// Eq. 1): D_p u_p first, then for each axis the lower and the upper
// neighbour; terms of Dirichlet ghost neighbours are omitted (they are zero).
// A general sparse matrix adds its off-diagonal entries A_pq u_q in the row's
// storage order (for a stencil written as such a matrix, with A_pq = -c, the
// bits are the same: (-c) u = -(c u)).
__device__ __forceinline__ double row_s(const DevProblem &P, const double *u, int64_t p,
                                        int64_t i0, int64_t i1, int64_t i2)
{
    if (P.ell_len) {  // general sparse matrix: the diagonal, then the row in storage order
        double s = P.diag[p] * u[p];
        for (int j = 0; j < P.ell_len[p]; ++j)
            s = s + P.ell_val[(int64_t)j * P.n0 + p] * u[P.ell_col[(int64_t)j * P.n0 + p]];
        return s;
    }
    const int64_t s1 = P.n0, s2 = P.n0 * P.n1;
    double s = (P.diag ? P.diag[p] : P.dconst) * u[p];
    if (i0 > 0) s = s - (P.face[0] ? P.face[0][p - 1] : P.c[0]) * u[p - 1];
    if (i0 < P.n0 - 1) s = s - (P.face[0] ? P.face[0][p] : P.c[0]) * u[p + 1];
    if (P.ndim >= 2) {
        if (i1 > 0) s = s - (P.face[1] ? P.face[1][p - s1] : P.c[1]) * u[p - s1];
        if (i1 < P.n1 - 1) s = s - (P.face[1] ? P.face[1][p] : P.c[1]) * u[p + s1];
    }
    if (P.ndim >= 3) {
        if (i2 > 0) s = s - (P.face[2] ? P.face[2][p - s2] : P.c[2]) * u[p - s2];
        if (i2 < P.n2 - 1) s = s - (P.face[2] ? P.face[2][p] : P.c[2]) * u[p + s2];
    }
    return s;
}

}  // namespace srj
