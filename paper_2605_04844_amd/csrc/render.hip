// qb_render: per-tile front-to-back alpha compositing, Eq. (2).
//
// One 256-lane workgroup (four wave64) per 16x16 tile, one pixel per lane.
// The tile's depth-sorted list is walked in batches of 256: each lane gathers
// one Gaussian record into LDS (the 48-byte records of all Gaussians fit the
// 256 MB Infinity Cache, so these gathers rarely reach HBM), then every lane
// composites the batch for its pixel from LDS broadcasts.  A pixel stops before
// the Gaussian that would take its transmittance below 1e-4; the workgroup
// leaves the list as soon as all 256 pixels have stopped.
//
// The 1/255 cutoff is Eq. (4) in log form: skip where power < -gamma/2, with
// power evaluated in the fixed binary32 order
//   power = fma(fma(-a/2, dx, (-b) dy), dx, ((-c/2) dy) dy),  dx = u - x, dy = v - y
// so the decision is reproducible bit for bit.
#include "qb_common.h"

namespace {

constexpr int kRenderThreads = QB_TILE * QB_TILE;

__global__ __launch_bounds__(kRenderThreads) void k_render(
    int W, int H, int tiles_x, const uint2* __restrict__ ranges, const uint32_t* __restrict__ ids,
    const float4* __restrict__ splats, float bg0, float bg1, float bg2, float* __restrict__ image,
    float* __restrict__ final_T, uint32_t* __restrict__ n_contrib)
{
    __shared__ float4 s_geo[kRenderThreads];   // u, v, -a/2, -b
    __shared__ float4 s_opa[kRenderThreads];   // -c/2, o, -gamma/2, unused
    __shared__ float4 s_col[kRenderThreads];   // r, g, b, unused

    int tile = blockIdx.x;
    int tx = tile % tiles_x, ty = tile / tiles_x;
    int lx = threadIdx.x & (QB_TILE - 1), ly = threadIdx.x >> 4;
    int px = tx * QB_TILE + lx, py = ty * QB_TILE + ly;
    bool inside = px < W && py < H;
    float fx = (float)px, fy = (float)py;

    uint2 rg = ranges[tile];
    int64_t start = rg.x, end = rg.y;
    bool done = !inside;
    float T = 1.0f, c0 = 0.0f, c1 = 0.0f, c2 = 0.0f;
    uint32_t seen = 0, last = 0;

    for (int64_t b0 = start; b0 < end; b0 += kRenderThreads) {
        if (__syncthreads_count(done) == kRenderThreads) break;
        int64_t j = b0 + threadIdx.x;
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
        int cnt = (int)min((int64_t)kRenderThreads, end - b0);
        if (!done) {
            for (int k = 0; k < cnt; ++k) {
                float4 g = s_geo[k];
                float4 o = s_opa[k];
                ++seen;
                float dx = g.x - fx, dy = g.y - fy;
                float power = fmaf(fmaf(g.z, dx, g.w * dy), dx, (o.x * dy) * dy);
                if (power > 0.0f || power < o.z) continue;
                float alpha = fminf(0.99f, o.y * __expf(power));
                float test_T = T * (1.0f - alpha);
                if (test_T < 1e-4f) {
                    done = true;
                    break;
                }
                float4 col = s_col[k];
                float w = alpha * T;
                c0 = fmaf(col.x, w, c0);
                c1 = fmaf(col.y, w, c1);
                c2 = fmaf(col.z, w, c2);
                T = test_T;
                last = seen;
            }
        }
    }
    if (inside) {
        int64_t p = (int64_t)py * W + px;
        int64_t plane = (int64_t)W * H;
        image[p] = fmaf(T, bg0, c0);
        image[plane + p] = fmaf(T, bg1, c1);
        image[2 * plane + p] = fmaf(T, bg2, c2);
        if (final_T) final_T[p] = T;
        if (n_contrib) n_contrib[p] = last;
    }
}

}  // namespace

extern "C" qb_status qb_render(int32_t width, int32_t height, const uint32_t* ranges, const uint32_t* ids,
                               const qb_splat* splats, const float* bg, float* image, float* final_T,
                               uint32_t* n_contrib, qb_stream_t stream)
{
    if (width <= 0 || height <= 0 || width > 32767 * QB_TILE || height > 32767 * QB_TILE || !ranges ||
        !image || !bg)
        return QB_ERR_INVALID_ARG;
    int tiles_x = (int)qb_div_up(width, QB_TILE);
    int64_t tiles = (int64_t)tiles_x * qb_div_up(height, QB_TILE);
    if (tiles > (1 << 24)) return QB_ERR_INVALID_ARG;
    QB_LAUNCH(k_render, tiles, kRenderThreads, 0, qb_hip_stream(stream), (int)width, (int)height, tiles_x,
              reinterpret_cast<const uint2*>(ranges), ids, reinterpret_cast<const float4*>(splats), bg[0], bg[1],
              bg[2], image, final_T, n_contrib);
    return QB_OK;
}
