// Work units of the one-thread-per-point kernels (residual norm, multigrid
// transfers): a unit is 256 consecutive points of one grid row (axis 0),
// unit (xb, y, z) the xb-th of row y of plane z.  Hardware places workgroup
// b on XCD b % 8, and each XCD has its own L2; dealing the units out in
// launch order would put the rows above, below, before and behind a row on
// other XCDs, each fetching them again.  Grids of at least kBandMinRows rows
// per plane are therefore dealt in bands instead: XCD k takes the rows
// y in [k n1 / 8, (k + 1) n1 / 8) of every plane, plane by plane, so a row's
// neighbours in y and z are read through the same L2.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace srj {

constexpr int kRowUnit = 256;
constexpr int64_t kBandMinRows = 64;

__host__ __device__ inline int64_t row_units_x(int64_t n0) { return (n0 + kRowUnit - 1) / kRowUnit; }

__host__ __device__ inline bool row_banded(int64_t n1) { return n1 >= kBandMinRows; }

// Workgroups to launch for the units of an n0 x n1 x n2 grid (a multiple of
// 8 when banded: every XCD covers its largest band).
inline int64_t row_grid(int64_t n0, int64_t n1, int64_t n2)
{
    const int64_t xb = row_units_x(n0);
    if (!row_banded(n1)) return xb * n1 * n2;
    return 8 * xb * ((n1 + 7) / 8) * n2;
}

// Unit of workgroup b (wave-uniform); false if b has none.
__device__ __forceinline__ bool row_unit(int64_t b, int64_t n0, int64_t n1, int64_t n2,
                                         int64_t &xb, int64_t &y, int64_t &z)
{
    const int64_t nx = row_units_x(n0);
    if (!row_banded(n1)) {
        xb = b % nx;
        y = (b / nx) % n1;
        z = b / (nx * n1);
        return z < n2;
    }
    const int64_t k = b % 8, j = b / 8;
    const int64_t y0 = n1 * k / 8, band = n1 * (k + 1) / 8 - y0;
    const int64_t per_plane = nx * band;
    if (j >= per_plane * n2) return false;
    z = j / per_plane;
    const int64_t rem = j - z * per_plane;
    y = y0 + rem / nx;
    xb = rem - (rem / nx) * nx;
    return true;
}

}  // namespace srj
