// qb_render: per-tile front-to-back alpha compositing, Eq. (2).
//
// One 128-lane workgroup (two wave64) per 16x16 tile; each lane owns the two
// pixels (x, y) and (x + 8, y) of one row, so the row-dependent terms of the
// quadratic form and every LDS read are shared by two pixels.  The tile's
// depth-sorted list is walked in batches of 128: each lane gathers one
// Gaussian record into LDS (the 48-byte records of all Gaussians fit the
// 256 MB Infinity Cache, so these gathers rarely reach HBM), then every lane
// composites the batch for its pixels from LDS broadcasts.  A pixel stops
// before the Gaussian that would take its transmittance below 1e-4; the
// workgroup leaves the list as soon as all 256 pixels have stopped.
//
// The 1/255 cutoff is Eq. (4) in log form: skip where power < -gamma/2, with
// power evaluated in the fixed binary32 order
//   power = fma(fma(-a/2, dx, (-b) dy), dx, ((-c/2) dy) dy),  dx = u - x, dy = v - y
// so the decision is reproducible bit for bit.
#include "qb_common.h"

namespace {

constexpr int kRenderThreads = 128;  // two wave64; each lane owns two pixels of one row

// Tiles go to workgroups in row-major order.  The dispatcher deals
// workgroups round-robin to the 8 XCDs, so each XCD receives every 8th tile of
// every row band: the heavy tiles of a dense region are spread over all XCDs
// (measured faster than giving each XCD a contiguous band of tiles, which
// keeps shared Gaussians in one L2 but leaves the XCDs unevenly loaded).
// Composites one tile of one image (the workgroup's 128 lanes).
__device__ __forceinline__ void render_tile(int tile, int W, int H, int tiles_x, const uint2* __restrict__ ranges,
                                            const uint32_t* __restrict__ ids, const float4* __restrict__ splats,
                                            float bg0, float bg1, float bg2, float* __restrict__ image,
                                            float* __restrict__ final_T, uint32_t* __restrict__ n_contrib,
                                            uint32_t* __restrict__ n_touched)
{
    __shared__ float4 s_geo[kRenderThreads];   // u, v, -a/2, -b
    __shared__ float4 s_opa[kRenderThreads];   // -c/2, o, -gamma/2, unused
    __shared__ float4 s_col[kRenderThreads];   // r, g, b, unused

    int tx = tile % tiles_x, ty = tile / tiles_x;
    int lx = threadIdx.x & 7, ly = threadIdx.x >> 3;
    int px0 = tx * QB_TILE + lx, px1 = px0 + 8, py = ty * QB_TILE + ly;
    bool in0 = px0 < W && py < H, in1 = px1 < W && py < H;
    float fx0 = (float)px0, fx1 = (float)px1, fy = (float)py;

    uint2 rg = ranges[tile];
    int64_t start = rg.x, end = rg.y;
    bool done0 = !in0, done1 = !in1;
    float T0 = 1.0f, T1 = 1.0f;
    float a0 = 0.0f, a1 = 0.0f, a2 = 0.0f, b0c = 0.0f, b1c = 0.0f, b2c = 0.0f;
    uint32_t last0 = 0, last1 = 0, stop0 = 0, stop1 = 0;

    for (int64_t base = start; base < end; base += kRenderThreads) {
        if (__syncthreads_count(done0 && done1) == kRenderThreads) break;
        int64_t j = base + threadIdx.x;
        if (j < end) {
            uint32_t id = ids[j];
            float4 a = splats[3 * (int64_t)id + 0];   // u, v, depth, o
            float4 b = splats[3 * (int64_t)id + 1];   // a, b, c, gamma
            float4 c = splats[3 * (int64_t)id + 2];   // r, g, b, visible
            s_geo[threadIdx.x] = make_float4(a.x, a.y, -0.5f * b.x, -b.y);
            s_opa[threadIdx.x] = make_float4(-0.5f * b.z, a.w, -0.5f * b.w, 0.0f);
            s_col[threadIdx.x] = c;
        }
        __syncthreads();
        if (done0 && done1) continue;
        int cnt = (int)min((int64_t)kRenderThreads, end - base);
        uint32_t idx0 = (uint32_t)(base - start);
        for (int k = 0; k < cnt; ++k) {
            float4 g = s_geo[k];
            float4 o = s_opa[k];
            // the terms of the quadratic form that depend on the row only
            float dy = g.y - fy;
            float nbdy = g.w * dy;
            float hcdy2 = (o.x * dy) * dy;
            float dx0 = g.x - fx0, dx1 = g.x - fx1;
            float p0 = fmaf(fmaf(g.z, dx0, nbdy), dx0, hcdy2);
            float p1 = fmaf(fmaf(g.z, dx1, nbdy), dx1, hcdy2);
            bool act0 = !done0 && !(p0 > 0.0f || p0 < o.z);
            bool act1 = !done1 && !(p1 > 0.0f || p1 < o.z);
            // branch only when the whole wave agrees; per pixel, select
            if (!__any(act0 || act1)) continue;
            float4 col = s_col[k];
            uint32_t at = idx0 + (uint32_t)k + 1u;
            {
                float alpha = fminf(0.99f, o.y * __expf(p0));
                float test_T = T0 * (1.0f - alpha);
                bool stop = act0 && test_T < 1e-4f;
                bool add = act0 && !(test_T < 1e-4f);
                float w = add ? alpha * T0 : 0.0f;
                a0 = fmaf(col.x, w, a0);
                a1 = fmaf(col.y, w, a1);
                a2 = fmaf(col.z, w, a2);
                T0 = add ? test_T : T0;
                last0 = add ? at : last0;
                stop0 = stop ? at : stop0;
                done0 = done0 || stop;
            }
            {
                float alpha = fminf(0.99f, o.y * __expf(p1));
                float test_T = T1 * (1.0f - alpha);
                bool stop = act1 && test_T < 1e-4f;
                bool add = act1 && !(test_T < 1e-4f);
                float w = add ? alpha * T1 : 0.0f;
                b0c = fmaf(col.x, w, b0c);
                b1c = fmaf(col.y, w, b1c);
                b2c = fmaf(col.z, w, b2c);
                T1 = add ? test_T : T1;
                last1 = add ? at : last1;
                stop1 = stop ? at : stop1;
                done1 = done1 || stop;
            }
            if (__all(done0 && done1)) break;
        }
    }
    uint32_t len = (uint32_t)(end - start);
    int64_t plane = (int64_t)W * H;
    if (in0) {
        int64_t p = (int64_t)py * W + px0;
        image[p] = fmaf(T0, bg0, a0);
        image[plane + p] = fmaf(T0, bg1, a1);
        image[2 * plane + p] = fmaf(T0, bg2, a2);
        if (final_T) final_T[p] = T0;
        if (n_contrib) n_contrib[p] = last0;
        if (n_touched) n_touched[p] = done0 ? stop0 : len;
    }
    if (in1) {
        int64_t p = (int64_t)py * W + px1;
        image[p] = fmaf(T1, bg0, b0c);
        image[plane + p] = fmaf(T1, bg1, b1c);
        image[2 * plane + p] = fmaf(T1, bg2, b2c);
        if (final_T) final_T[p] = T1;
        if (n_contrib) n_contrib[p] = last1;
        if (n_touched) n_touched[p] = done1 ? stop1 : len;
    }
}

__global__ __launch_bounds__(kRenderThreads) void k_render(
    int W, int H, int tiles_x, const uint2* __restrict__ ranges, const uint32_t* __restrict__ ids,
    const float4* __restrict__ splats, float bg0, float bg1, float bg2, float* __restrict__ image,
    float* __restrict__ final_T, uint32_t* __restrict__ n_contrib, uint32_t* __restrict__ n_touched)
{
    render_tile((int)blockIdx.x, W, H, tiles_x, ranges, ids, splats, bg0, bg1, bg2, image, final_T, n_contrib,
                n_touched);
}

// Every tile of every view in one launch: workgroup b takes global tile b,
// whose view is found in the (at most QB_MAX_VIEWS) tile offsets.
__global__ __launch_bounds__(kRenderThreads) void k_render_views(QbViewTable vt, float bg0, float bg1, float bg2)
{
    int b = (int)blockIdx.x;
    int v = qb_view_of(vt, b);
    const qb_view& w = vt.view[v];
    render_tile(b - vt.tile_start[v], w.width, w.height, vt.tiles_x[v], reinterpret_cast<const uint2*>(w.ranges),
                w.ids, reinterpret_cast<const float4*>(w.splats), bg0, bg1, bg2, w.image, w.final_T, w.n_contrib,
                nullptr);
}

}  // namespace

extern "C" qb_status qb_render(int32_t width, int32_t height, const uint32_t* ranges, const uint32_t* ids,
                               const qb_splat* splats, const float* bg, float* image, float* final_T,
                               uint32_t* n_contrib, uint32_t* n_touched, qb_stream_t stream)
{
    if (width <= 0 || height <= 0 || width > 32767 * QB_TILE || height > 32767 * QB_TILE || !ranges ||
        !image || !bg)
        return QB_ERR_INVALID_ARG;
    int tiles_x = (int)qb_div_up(width, QB_TILE);
    int64_t tiles = (int64_t)tiles_x * qb_div_up(height, QB_TILE);
    if (tiles > (1 << 24)) return QB_ERR_INVALID_ARG;
    QB_LAUNCH(k_render, tiles, kRenderThreads, 0, qb_hip_stream(stream), (int)width, (int)height, tiles_x,
              reinterpret_cast<const uint2*>(ranges), ids, reinterpret_cast<const float4*>(splats), bg[0], bg[1],
              bg[2], image, final_T, n_contrib, n_touched);
    return QB_OK;
}

extern "C" qb_status qb_render_views(int32_t num_views, const qb_view* views, const float* bg, qb_stream_t stream)
{
    if (!bg) return QB_ERR_INVALID_ARG;
    QbViewTable vt;
    qb_status st = qb_make_view_table(num_views, views, false, &vt);
    if (st != QB_OK) return st;
    if (vt.tile_start[num_views] == 0) return QB_OK;
    QB_LAUNCH(k_render_views, vt.tile_start[num_views], kRenderThreads, 0, qb_hip_stream(stream), vt, bg[0], bg[1],
              bg[2]);
    return QB_OK;
}
