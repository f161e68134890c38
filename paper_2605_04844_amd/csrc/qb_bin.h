// QPass helpers shared by the intersect translation unit: packed tile rects of
// a Gaussian -> QPass runs.
#pragma once

#include "qb_radix.h"

namespace qbb {

__device__ __forceinline__ QRect unpack_rect(int lohi_x, int lohi_y)
{
    QRect r;
    r.x0 = (int)(int16_t)(lohi_x & 0xFFFF);
    r.x1 = lohi_x >> 16;
    r.y0 = (int)(int16_t)(lohi_y & 0xFFFF);
    r.y1 = lohi_y >> 16;
    return r;
}

// QPass runs of Gaussian gi from its packed rects.
__device__ __forceinline__ void gaussian_runs(const int4* __restrict__ rects, uint32_t gi, QRuns& q)
{
    int4 p0 = rects[2 * (int64_t)gi], p1 = rects[2 * (int64_t)gi + 1];
    QRect r[4] = {unpack_rect(p0.x, p0.y), unpack_rect(p0.z, p0.w), unpack_rect(p1.x, p1.y),
                  unpack_rect(p1.z, p1.w)};
    qpass_runs(r, q);
}

}  // namespace qbb
