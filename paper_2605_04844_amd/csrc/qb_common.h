// Internal helpers shared by the HIP translation units of libquadbox.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/quadbox.h"

#define QB_TILE 16
#define QB_BLOCK 256

// Launch helper: checks the launch and maps failures to QB_ERR_HIP.
#define QB_LAUNCH(kernel, grid, block, shmem, stream, ...)                                 \
    do {                                                                                   \
        hipLaunchKernelGGL(kernel, dim3(grid), dim3(block), shmem, stream, __VA_ARGS__);   \
        if (hipGetLastError() != hipSuccess) return QB_ERR_HIP;                            \
    } while (0)

#define QB_CHECK(expr)                                                                     \
    do {                                                                                   \
        qb_status _s = (expr);                                                             \
        if (_s != QB_OK) return _s;                                                        \
    } while (0)

static inline hipStream_t qb_hip_stream(qb_stream_t s) { return reinterpret_cast<hipStream_t>(s); }

static inline int64_t qb_div_up(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Bump allocator over a caller workspace; every slice is 256-byte aligned.
struct QbArena {
    char* base;
    size_t cap;
    size_t used;
    template <typename T>
    T* take(int64_t count) {
        size_t bytes = (size_t)(count > 0 ? count : 1) * sizeof(T);
        size_t off = (used + 255) & ~(size_t)255;
        used = off + bytes;
        return base ? reinterpret_cast<T*>(base + off) : nullptr;
    }
    bool ok() const { return used <= cap; }
};

// Tile rect of a sub-box: inclusive tile bounds; empty when x0 > x1.
struct QRect {
    int x0, x1, y0, y1;
};

// Run of scanlines with one tile span (the QPass per-scanline result is
// constant between two consecutive sub-box ends along the scan axis).
struct QSeg {
    int s0;   // first scanline
    int n;    // number of scanlines
    int lo;   // first tile along the other axis
    int len;  // tiles per scanline
};

#define QB_MAX_SEG 7

// QPass (Sec. 3.2): global tile range of the non-empty sub-boxes, scan along
// its shorter axis; per scanline, the sub-boxes whose range on the scan axis
// holds it (interval overlap test) give the span [min lo, max hi] on the other
// axis.  Scanlines are grouped into runs whose active set is the same, which
// makes each pair addressable in O(1).  Returns the number of runs; *axis = 0
// scans columns (scanline = tx), 1 rows; *total = tiles in the set.
__host__ __device__ __forceinline__ int qpass_segments(const QRect r[4], QSeg seg[QB_MAX_SEG], int* axis,
                                              int* total)
{
    int a[4], b[4], c[4], d[4];
    int m = 0;
    int gx0 = 1 << 30, gx1 = -(1 << 30), gy0 = 1 << 30, gy1 = -(1 << 30);
    for (int k = 0; k < 4; ++k) {
        if (r[k].x0 > r[k].x1 || r[k].y0 > r[k].y1) continue;
        gx0 = r[k].x0 < gx0 ? r[k].x0 : gx0;
        gx1 = r[k].x1 > gx1 ? r[k].x1 : gx1;
        gy0 = r[k].y0 < gy0 ? r[k].y0 : gy0;
        gy1 = r[k].y1 > gy1 ? r[k].y1 : gy1;
        a[m] = r[k].x0; b[m] = r[k].x1; c[m] = r[k].y0; d[m] = r[k].y1;
        ++m;
    }
    *total = 0;
    *axis = 0;
    if (m == 0) return 0;
    if (gx1 - gx0 > gy1 - gy0) {  // rows are the shorter axis: swap roles
        *axis = 1;
        for (int k = 0; k < m; ++k) {
            int t0 = a[k], t1 = b[k];
            a[k] = c[k]; b[k] = d[k]; c[k] = t0; d[k] = t1;
        }
    }
    // breakpoints along the scan axis: every start and every end + 1
    int e[8];
    int ne = 0;
    for (int k = 0; k < m; ++k) {
        e[ne++] = a[k];
        e[ne++] = b[k] + 1;
    }
    for (int i = 1; i < ne; ++i) {  // insertion sort, at most 8 values
        int v = e[i], j = i - 1;
        while (j >= 0 && e[j] > v) { e[j + 1] = e[j]; --j; }
        e[j + 1] = v;
    }
    int ns = 0, tot = 0;
    for (int i = 0; i + 1 < ne; ++i) {
        int s0 = e[i], s1 = e[i + 1];
        if (s1 <= s0) continue;
        int lo = 1 << 30, hi = -(1 << 30);
        for (int k = 0; k < m; ++k)
            if (a[k] <= s0 && b[k] >= s0) {  // interval overlap with this run
                lo = c[k] < lo ? c[k] : lo;
                hi = d[k] > hi ? d[k] : hi;
            }
        if (hi < lo) continue;
        seg[ns].s0 = s0;
        seg[ns].n = s1 - s0;
        seg[ns].lo = lo;
        seg[ns].len = hi - lo + 1;
        tot += seg[ns].n * seg[ns].len;
        ++ns;
    }
    *total = tot;
    return ns;
}
