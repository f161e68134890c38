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

// A qb_box_mode, optionally with QB_CLIP_3SIGMA on an opacity-aware mode.
static inline bool qb_valid_mode(int32_t mode)
{
    int32_t base = mode & ~QB_CLIP_3SIGMA;
    if (base < QB_BOX_3SIGMA || base > QB_BOX_QUADBOX_NAIVE) return false;
    return !((mode & QB_CLIP_3SIGMA) && base == QB_BOX_3SIGMA);
}

// A usable camera: positive image size within the tile-id range, positive
// focal lengths, a positive near plane (depth keys are the binary32 bits of
// the view depth, which order correctly only for positive depths), and
// finite intrinsics, pose and centre.
static inline bool qb_valid_camera(const qb_camera& c)
{
    if (c.width <= 0 || c.height <= 0 || c.width > 32767 * QB_TILE || c.height > 32767 * QB_TILE) return false;
    if (!(c.fx > 0.0f) || !(c.fy > 0.0f) || !(c.near_plane > 0.0f)) return false;
    float all[7 + 9 + 3 + 3] = {c.fx, c.fy, c.cx, c.cy, c.near_plane};
    for (int k = 0; k < 9; ++k) all[7 + k] = c.R[k];
    for (int k = 0; k < 3; ++k) all[16 + k] = c.t[k], all[19 + k] = c.campos[k];
    for (float x : all)
        if (!(x - x == 0.0f)) return false;   // NaN or infinite
    return true;
}

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

// Tile-local rows [r0, r1] (packed r0 | r1 << 16, clamped to [-1, 16]) that
// can hold a pixel passing the cutoff of a Gaussian with mean row v, conic
// (a, b, c) and gamma: the ellipse power >= -gamma/2 spans v +- sqrt(gamma
// Sigma_yy) with Sigma_yy = a / (a c - b^2).  Widened by 1% + 0.5 px so that
// binary32 rounding of the power can never pass a pixel outside the range.
__host__ __device__ __forceinline__ int entry_rows(float v, float a, float b, float c, float gamma, int ty)
{
    // a c - b^2 of a needle's conic cancels: binary64 (the products are exact)
    double det = (double)a * (double)c - (double)b * (double)b;
    float h = det > 0.0 && gamma > 0.0f && a > 0.0f ? (float)sqrt((double)gamma * (double)a / det) : 3.0e4f;
    h = h * 1.01f + 0.5f;
    float y0 = v - h - (float)(ty * QB_TILE), y1 = v + h - (float)(ty * QB_TILE);
    int r0 = y0 < -1.0f ? -1 : (y0 > 16.0f ? 16 : (int)floorf(y0));
    int r1 = y1 < -1.0f ? -1 : (y1 > 16.0f ? 16 : (int)ceilf(y1));
    return (r0 & 0xFFFF) | (r1 << 16);
}

// Per-view table of a batched call, passed by value as a kernel argument
// (about 2.6 KB at QB_MAX_VIEWS views).  tile_start[v] is the first global
// tile of view v; tile_start[num] is the total.
struct QbViewTable {
    int num;
    int tile_start[QB_MAX_VIEWS + 1];
    int tiles_x[QB_MAX_VIEWS];
    qb_view view[QB_MAX_VIEWS];
};

// View of global tile b (b < tile_start[num]).
__device__ __forceinline__ int qb_view_of(const QbViewTable& vt, int b)
{
    int v = 0;
    while (v + 1 < vt.num && b >= vt.tile_start[v + 1]) ++v;
    return v;
}

// Validates the views of a batched render (backward: also the gradient
// buffers) and fills the table.
static inline qb_status qb_make_view_table(int32_t num_views, const qb_view* views, bool backward,
                                           QbViewTable* vt)
{
    if (num_views < 1 || num_views > QB_MAX_VIEWS || !views) return QB_ERR_INVALID_ARG;
    vt->num = num_views;
    int64_t total = 0;
    for (int v = 0; v < num_views; ++v) {
        const qb_view& w = views[v];
        if (w.width <= 0 || w.height <= 0 || w.width > 32767 * QB_TILE || w.height > 32767 * QB_TILE ||
            !w.ranges || !w.ids || !w.splats || !w.final_T || !w.n_contrib)
            return QB_ERR_INVALID_ARG;
        if (!backward && !w.image) return QB_ERR_INVALID_ARG;
        if (backward && (!w.dL_dimage || !w.grad2d)) return QB_ERR_INVALID_ARG;
        int64_t tx = qb_div_up(w.width, QB_TILE);
        vt->tile_start[v] = (int)total;
        vt->tiles_x[v] = (int)tx;
        vt->view[v] = w;
        total += tx * qb_div_up(w.height, QB_TILE);
        if (total > (1 << 30)) return QB_ERR_INVALID_ARG;
    }
    vt->tile_start[num_views] = (int)total;
    return QB_OK;
}

__host__ __device__ __forceinline__ bool qrect_holds(const QRect& r, int tx, int ty)
{
    return tx >= r.x0 && tx <= r.x1 && ty >= r.y0 && ty <= r.y1;
}

// Naive QuadBox traversal, the ablation without QPass (Sec. 3.2): each
// sub-box's tile rect is walked with nested loops, and a tile that an earlier
// sub-box's rect holds was visited already and is skipped.  visit(tx, ty, c)
// sees the c-th new tile; returns the number of tiles.
template <class Visit>
__host__ __device__ __forceinline__ int naive_walk(const QRect r[4], Visit visit)
{
    int cnt = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k)
        for (int ty = r[k].y0; ty <= r[k].y1; ++ty)
            for (int tx = r[k].x0; tx <= r[k].x1; ++tx) {
                bool seen = false;
#pragma unroll
                for (int j = 0; j < k; ++j) seen = seen || qrect_holds(r[j], tx, ty);
                if (!seen) {
                    visit(tx, ty, cnt);
                    ++cnt;
                }
            }
    return cnt;
}

// QPass runs of one Gaussian (Sec. 3.2).  A run is a block of consecutive
// scanlines whose QPass interval is the same: n scanlines from s0, each with
// the len tiles from lo on the other axis.  Every run slot is filled (empty
// ones have n = 0 or len = 0), so the arrays stay in registers.
#define QB_MAX_SEG 7
#define QB_BIG (1 << 30)

struct QRuns {
    int s0[QB_MAX_SEG], n[QB_MAX_SEG], lo[QB_MAX_SEG], len[QB_MAX_SEG];
    int axis;   // 0: scanlines are tile columns, 1: tile rows
    int total;  // tiles in the set
};

__host__ __device__ __forceinline__ void qb_cswap(int& x, int& y)
{
    int lo = x < y ? x : y, hi = x < y ? y : x;
    x = lo;
    y = hi;
}

// QPass: the global tile range of the non-empty sub-boxes, scanned along its
// shorter axis; on each scanline, the sub-boxes whose range on the scan axis
// holds it (interval overlap test) give the span [min lo, max hi] on the other
// axis.  The active set only changes at a sub-box start or end + 1, so the
// scanlines between two consecutive such breakpoints form one run.
__host__ __device__ __forceinline__ void qpass_runs(const QRect r[4], QRuns& q)
{
    bool act[4];
    int gx0 = QB_BIG, gx1 = -QB_BIG, gy0 = QB_BIG, gy1 = -QB_BIG;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        act[k] = r[k].x0 <= r[k].x1 && r[k].y0 <= r[k].y1;
        if (act[k]) {
            gx0 = r[k].x0 < gx0 ? r[k].x0 : gx0;
            gx1 = r[k].x1 > gx1 ? r[k].x1 : gx1;
            gy0 = r[k].y0 < gy0 ? r[k].y0 : gy0;
            gy1 = r[k].y1 > gy1 ? r[k].y1 : gy1;
        }
    }
    q.axis = (gx1 - gx0 > gy1 - gy0) ? 1 : 0;  // scan the shorter axis
    int a[4], b[4], c[4], d[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        int sa = q.axis ? r[k].y0 : r[k].x0, sb = q.axis ? r[k].y1 : r[k].x1;
        int oa = q.axis ? r[k].x0 : r[k].y0, ob = q.axis ? r[k].x1 : r[k].y1;
        a[k] = act[k] ? sa : QB_BIG;
        b[k] = act[k] ? sb : QB_BIG - 1;
        c[k] = oa;
        d[k] = ob;
    }
    int e[8] = {a[0], b[0] + 1, a[1], b[1] + 1, a[2], b[2] + 1, a[3], b[3] + 1};
    // Batcher's odd-even merge network for 8 keys (19 comparators)
    qb_cswap(e[0], e[1]); qb_cswap(e[2], e[3]); qb_cswap(e[4], e[5]); qb_cswap(e[6], e[7]);
    qb_cswap(e[0], e[2]); qb_cswap(e[1], e[3]); qb_cswap(e[4], e[6]); qb_cswap(e[5], e[7]);
    qb_cswap(e[1], e[2]); qb_cswap(e[5], e[6]); qb_cswap(e[0], e[4]); qb_cswap(e[3], e[7]);
    qb_cswap(e[1], e[5]); qb_cswap(e[2], e[6]);
    qb_cswap(e[1], e[4]); qb_cswap(e[3], e[6]);
    qb_cswap(e[2], e[4]); qb_cswap(e[3], e[5]);
    qb_cswap(e[3], e[4]);
    int tot = 0;
#pragma unroll
    for (int i = 0; i < QB_MAX_SEG; ++i) {
        int s0 = e[i], s1 = e[i + 1];
        int lo = QB_BIG, hi = -QB_BIG;
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (a[k] <= s0 && b[k] >= s0) {  // interval overlap with this run
                lo = c[k] < lo ? c[k] : lo;
                hi = d[k] > hi ? d[k] : hi;
            }
        bool valid = s1 > s0 && s0 < QB_BIG && hi >= lo;
        q.s0[i] = s0;
        q.n[i] = valid ? s1 - s0 : 0;
        q.lo[i] = lo;
        q.len[i] = valid ? hi - lo + 1 : 0;
        tot += q.n[i] * q.len[i];
    }
    q.total = tot;
}
