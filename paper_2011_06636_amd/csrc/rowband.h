// Work units of the one-thread-per-column kernels (residual norm, multigrid
// transfers): a unit is 256 consecutive columns (axis 0) of R consecutive
// rows of one plane, each thread taking one column of the unit's rows.
// Hardware places workgroup b on XCD b % 8, and each XCD has its own L2;
// dealing the units out in launch order would put the rows above, below,
// before and behind a row on other XCDs, each fetching them again.  Grids of
// at least kBandMinRows rows per plane are therefore dealt in bands instead:
// XCD k takes the rows y in [k n1 / 8, (k + 1) n1 / 8) of every plane, plane
// by plane, in units of R rows from the band's first row (the band's last
// unit may hold fewer), so a row's neighbours in y and z are read through
// the same L2.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace srj {

constexpr int kRowUnit = 256;
constexpr int64_t kBandMinRows = 64;
// Rows per unit of the kernels that leave one partial sum of the residual
// norm per workgroup (the norm, the refinement's outer pass): each thread has
// the loads of that many points in flight, and there are that many times
// fewer partials to fold.
constexpr int kNormRows = 4;

__host__ __device__ inline int64_t row_units_x(int64_t n0) { return (n0 + kRowUnit - 1) / kRowUnit; }

__host__ __device__ inline bool row_banded(int64_t n1) { return n1 >= kBandMinRows; }

// Units of R rows over `rows` rows.
__host__ __device__ inline int64_t row_groups(int64_t rows, int R) { return (rows + R - 1) / R; }

// Workgroups to launch for the units of R rows of an n0 x n1 x n2 grid (a
// multiple of 8 when banded: every XCD covers its largest band, of at most
// ceil(n1 / 8) rows).
inline int64_t row_grid(int64_t n0, int64_t n1, int64_t n2, int R = 1)
{
    const int64_t xb = row_units_x(n0);
    if (!row_banded(n1)) return xb * row_groups(n1, R) * n2;
    return 8 * xb * row_groups((n1 + 7) / 8, R) * n2;
}

// Unit of workgroup b (wave-uniform): columns from 256 xb, rows y .. y + ny
// - 1 (1 <= ny <= R) of plane z; false if b has none.
__device__ __forceinline__ bool row_unit(int64_t b, int64_t n0, int64_t n1, int64_t n2, int R,
                                         int64_t &xb, int64_t &y, int &ny, int64_t &z)
{
    const int64_t nx = row_units_x(n0);
    int64_t y0 = 0, band = n1, j = b;
    if (row_banded(n1)) {
        const int64_t k = b % 8;
        j = b / 8;
        y0 = n1 * k / 8;
        band = n1 * (k + 1) / 8 - y0;
    }
    const int64_t per_plane = nx * row_groups(band, R);
    if (j >= per_plane * n2) return false;
    z = j / per_plane;
    const int64_t rem = j - z * per_plane;
    const int64_t g = rem / nx;
    xb = rem - g * nx;
    y = y0 + g * R;
    const int64_t left = band - g * R;
    ny = (int)(left < R ? left : R);
    return true;
}

// Single-row units (R = 1).
__device__ __forceinline__ bool row_unit(int64_t b, int64_t n0, int64_t n1, int64_t n2,
                                         int64_t &xb, int64_t &y, int64_t &z)
{
    int ny;
    return row_unit(b, n0, n1, n2, 1, xb, y, ny, z);
}

}  // namespace srj
