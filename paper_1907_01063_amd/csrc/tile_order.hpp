// Order in which the workgroups of a product launch take its output tiles.
//
// Plain orders enumerate the tiles row by row.  The grouped orders take bands
// of G tile rows one after another and walk each band column by column, so
// the workgroups that run at the same time on one XCD (about 64) cover a
// G x (64 / G) block of tiles: they share G row panels, which stay in that
// XCD's L2 for the whole band, and a few column panels, each fetched once for
// G tiles.  Row-by-row order instead streams every column panel once per tile
// row.  Host and device code (the host side is checked by a unit test).
#pragma once

#include <math.h>
#include <stdint.h>

#ifdef __HIPCC__
#include <hip/hip_runtime.h>
#else
#define __host__
#define __device__
#endif

namespace gpc {

// Tile (ti, tj), tj <= ti, of index b in the row-by-row enumeration of the
// lower triangle of tiles.
__host__ __device__ inline void lower_tile(int64_t b, int64_t& ti, int64_t& tj)
{
    int64_t t = (int64_t)((sqrt(8.0 * (double)b + 1.0) - 1.0) * 0.5);
    while (t * (t + 1) / 2 > b) --t;
    while ((t + 1) * (t + 2) / 2 <= b) ++t;
    ti = t;
    tj = b - t * (t + 1) / 2;
}

// Work item of dispatch index w of a launch of nwg workgroups.  Workgroups
// are dealt to the 8 XCDs round-robin (dispatch index mod 8); the item of w
// is numbered so that XCD x takes the x-th contiguous range of items (a tail
// past the last multiple of 8 keeps its own index).
__host__ __device__ inline int xcd_item(int w, int nwg)
{
    const int per = nwg / 8;
    return w < per * 8 ? (w % 8) * per + w / 8 : w;
}

// Tile (tm, tn) of index t of a tilesM x tilesN grid in the grouped order
// (bands of G rows; a last, shorter band takes the remaining rows).
__host__ __device__ inline void grouped_tile(int64_t t, int64_t tilesM, int64_t tilesN, int64_t G, int64_t& tm,
                                             int64_t& tn)
{
    const int64_t full = (tilesM / G) * G;   // rows in complete bands
    if (t < full * tilesN) {
        const int64_t band = G * tilesN, b = t / band, r = t - b * band;
        tm = b * G + r % G;
        tn = r / G;
    } else {
        const int64_t gl = tilesM - full, r = t - full * tilesN;
        tm = full + r % gl;
        tn = r / gl;
    }
}

// Tile (tm, tn), tn <= tm, of index t of the lower triangle of a
// tilesM x tilesM grid in the grouped order: band g holds tile rows
// [gG, gG + G); its tiles left of the band's diagonal block come column by
// column, then the diagonal block's lower triangle, column by column.
// Band g starts at index gG (gG + 1) / 2, as in the row-by-row order.
__host__ __device__ inline void grouped_lower_tile(int64_t t, int64_t tilesM, int64_t G, int64_t& tm, int64_t& tn)
{
    int64_t row, col;
    lower_tile(t, row, col);                 // row of t in the row-by-row order
    const int64_t r0 = (row / G) * G;        // first row of its band
    const int64_t gl = tilesM - r0 < G ? tilesM - r0 : G;
    int64_t r = t - r0 * (r0 + 1) / 2;
    if (r < r0 * gl) {
        tn = r / gl;
        tm = r0 + r % gl;
        return;
    }
    r -= r0 * gl;
    int64_t c = 0;
    while (r >= gl - c) {
        r -= gl - c;
        ++c;
    }
    tn = r0 + c;
    tm = r0 + c + r;
}

}  // namespace gpc
