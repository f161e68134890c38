// qb_tile_order: the order in which the render's workgroups take tiles.
//
// The render runs one workgroup per 16x16 tile, and at the frame sizes of
// interest every tile's workgroup is resident from the start (2 waves of 46
// VGPRs per tile, 8 waves per SIMD), so the work each SIMD does is fixed by
// which tiles the dispatcher deals to it.  Tile work varies by 2.5x across a
// frame and is spatially clustered; in row-major order the heavy tiles of a
// dense region share compute units and the busiest SIMDs finish long after
// the mean.  Dealing the tiles in decreasing order of work gives every
// compute unit a share of each work class.  None of this changes what a
// tile computes: the images, T, contributor counts and gradients are those
// of the row-major order.
//
// Work estimate: a tile's cost is the number of list entries its pixels
// examine before they stop (Eq. (2) with the 1e-4 transmittance stop), which
// the list length does not predict (most lists run far past the point where
// their pixels saturate).  The estimate follows the tile's centre pixel over
// the first kWorkPrefix entries of its list: one wave per tile, four
// consecutive entries per lane, the pixel's transmittance carried as a sum
// of log2(1 - alpha) (one wave prefix sum).  Where the sum drops below
// log2(1e-4) within the prefix, the estimate is the entry at which the pixel
// stops; where it does not, the stop is extrapolated at the prefix's rate of
// attenuation, kWorkPrefix * log2(1e-4) / log2(T), capped at the list
// length (the list length itself when nothing attenuates).  One step keeps
// the kernel to three dependent memory round trips (range, ids, records):
// walking up to 1024 entries exactly took twice as long for the same render
// time, and a 128-entry prefix or sampling every 2nd or 4th entry ordered
// the tiles worse (the render gave back part of its gain).
//
// Order: a counting sort of the estimates clamped to kOrderBins - 1 in one
// workgroup (LDS histogram, scan, scatter), heaviest first; tiles with
// equal estimates come in no fixed order.
#include "qb_common.h"

namespace {

constexpr int kWorkPerLane = 4;
constexpr int kWorkPrefix = 64 * kWorkPerLane;   // entries the estimate walks
constexpr float kLog2Stop = -13.28771238f;       // log2(1e-4)
constexpr int kOrderBins = 4096;
constexpr int kOrderThreads = 1024;

__device__ __forceinline__ float wave_inclusive_sum(float x, int lane)
{
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        float y = __shfl_up(x, d);
        if (lane >= d) x += y;
    }
    return x;
}

// Estimated entries the centre pixel of `tile` examines (see the file
// comment); the whole wave calls it and gets the same value.
__device__ uint32_t tile_work(int tile, int W, int H, int tiles_x, const uint2* __restrict__ ranges,
                              const uint32_t* __restrict__ ids, const float4* __restrict__ splats, int lane)
{
    int x0 = (tile % tiles_x) * QB_TILE, y0 = (tile / tiles_x) * QB_TILE;
    float px = (float)(x0 + min(QB_TILE, W - x0) / 2);
    float py = (float)(y0 + min(QB_TILE, H - y0) / 2);
    uint2 rg = ranges[tile];
    int64_t start = rg.x, end = rg.y;
    int64_t lim = min(end, start + (int64_t)kWorkPrefix);
    uint32_t id[kWorkPerLane];
#pragma unroll
    for (int j = 0; j < kWorkPerLane; ++j) {
        int64_t idx = start + lane * kWorkPerLane + j;
        id[j] = idx < lim ? ids[idx] : 0xFFFFFFFFu;
    }
    float4 ga[kWorkPerLane], gb[kWorkPerLane];
#pragma unroll
    for (int j = 0; j < kWorkPerLane; ++j)
        if (id[j] != 0xFFFFFFFFu) {
            ga[j] = splats[3 * (int64_t)id[j] + 0];   // u, v, depth, o
            gb[j] = splats[3 * (int64_t)id[j] + 1];   // a, b, c, gamma
        }
    float l[kWorkPerLane];
    float s = 0.0f;
#pragma unroll
    for (int j = 0; j < kWorkPerLane; ++j) {
        l[j] = 0.0f;
        if (id[j] != 0xFFFFFFFFu) {
            float4 a = ga[j], b = gb[j];
            float dx = a.x - px, dy = a.y - py;
            float p = fmaf(fmaf(-0.5f * b.x, dx, -b.y * dy), dx, (-0.5f * b.z * dy) * dy);
            if (!(p > 0.0f || p < -0.5f * b.w)) l[j] = __log2f(1.0f - fminf(0.99f, a.w * __expf(p)));
        }
        s += l[j];
    }
    float incl = wave_inclusive_sum(s, lane);
    uint64_t hit = __ballot(incl < kLog2Stop);
    if (hit) {
        int f = __builtin_ctzll(hit);
        uint32_t est = 0;
        if (lane == f) {
            float run = incl - s;
            int j = 0;
            for (; j < kWorkPerLane - 1; ++j) {
                run += l[j];
                if (run < kLog2Stop) break;
            }
            est = (uint32_t)min((int64_t)(f * kWorkPerLane + j + 1), lim - start);
        }
        return __shfl(est, f);
    }
    float total = __shfl(incl, 63);   // log2 T after the prefix
    if (lim < end && total < 0.0f)
        return (uint32_t)fminf((float)kWorkPrefix * (kLog2Stop / total), (float)(end - start));
    return (uint32_t)(end - start);
}

__global__ __launch_bounds__(QB_BLOCK) void k_tile_work(int W, int H, int tiles_x, int tiles,
                                                        const uint2* __restrict__ ranges,
                                                        const uint32_t* __restrict__ ids,
                                                        const float4* __restrict__ splats, uint32_t* __restrict__ work)
{
    int tile = blockIdx.x * (QB_BLOCK / 64) + (int)(threadIdx.x / 64);
    int lane = threadIdx.x & 63;
    if (tile >= tiles) return;
    uint32_t est = tile_work(tile, W, H, tiles_x, ranges, ids, splats, lane);
    if (lane == 0) work[tile] = est;
}

// Global tile b of every view (b < vt.tile_start[vt.num]).
__global__ __launch_bounds__(QB_BLOCK) void k_tile_work_views(QbViewTable vt, uint32_t* __restrict__ work)
{
    int b = blockIdx.x * (QB_BLOCK / 64) + (int)(threadIdx.x / 64);
    int lane = threadIdx.x & 63;
    if (b >= vt.tile_start[vt.num]) return;
    int v = qb_view_of(vt, b);
    const qb_view& w = vt.view[v];
    uint32_t est = tile_work(b - vt.tile_start[v], w.width, w.height, vt.tiles_x[v],
                             reinterpret_cast<const uint2*>(w.ranges), w.ids, reinterpret_cast<const float4*>(w.splats),
                             lane);
    if (lane == 0) work[b] = est;
}

__device__ __forceinline__ uint32_t order_bin(uint32_t w)
{
    return (uint32_t)(kOrderBins - 1) - min(w, (uint32_t)(kOrderBins - 1));
}

// One workgroup: histogram of the bins, exclusive scan, scatter.
__global__ __launch_bounds__(kOrderThreads) void k_tile_order(const uint32_t* __restrict__ work, int tiles,
                                                              uint32_t* __restrict__ order)
{
    __shared__ uint32_t hist[kOrderBins];
    __shared__ uint32_t wave_sum[kOrderThreads / 64];
    constexpr int kPer = kOrderBins / kOrderThreads;
    int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    for (int i = tid; i < kOrderBins; i += kOrderThreads) hist[i] = 0u;
    // up to kKeep tiles per thread keep their bins in registers between the
    // two passes; larger frames read work[] again
    constexpr int kKeep = 4;
    const bool keep = tiles <= kKeep * kOrderThreads;
    uint32_t bin[kKeep];
#pragma unroll
    for (int k = 0; k < kKeep; ++k) {
        int t = tid + k * kOrderThreads;
        bin[k] = keep && t < tiles ? order_bin(work[t]) : 0u;
    }
    __syncthreads();
    if (keep) {
#pragma unroll
        for (int k = 0; k < kKeep; ++k)
            if (tid + k * kOrderThreads < tiles) atomicAdd(&hist[bin[k]], 1u);
    } else {
        for (int t = tid; t < tiles; t += kOrderThreads) atomicAdd(&hist[order_bin(work[t])], 1u);
    }
    __syncthreads();
    uint32_t v[kPer], s = 0;
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        v[j] = hist[tid * kPer + j];
        s += v[j];
    }
    uint32_t incl = s;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t y = __shfl_up(incl, d);
        if (lane >= d) incl += y;
    }
    if (lane == 63) wave_sum[wv] = incl;
    __syncthreads();
    uint32_t ex = incl - s;
    for (int k = 0; k < wv; ++k) ex += wave_sum[k];
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        hist[tid * kPer + j] = ex;
        ex += v[j];
    }
    __syncthreads();
    if (keep) {
#pragma unroll
        for (int k = 0; k < kKeep; ++k) {
            int t = tid + k * kOrderThreads;
            if (t < tiles) order[atomicAdd(&hist[bin[k]], 1u)] = (uint32_t)t;
        }
    } else {
        for (int t = tid; t < tiles; t += kOrderThreads) order[atomicAdd(&hist[order_bin(work[t])], 1u)] = (uint32_t)t;
    }
}

}  // namespace

extern "C" qb_status qb_tile_order(int32_t width, int32_t height, const uint32_t* ranges, const uint32_t* ids,
                                   const qb_splat* splats, uint32_t* work, uint32_t* order, qb_stream_t stream)
{
    if (width <= 0 || height <= 0 || width > 32767 * QB_TILE || height > 32767 * QB_TILE || !ranges || !ids ||
        !splats || !work || !order)
        return QB_ERR_INVALID_ARG;
    int tiles_x = (int)qb_div_up(width, QB_TILE);
    int64_t tiles = (int64_t)tiles_x * qb_div_up(height, QB_TILE);
    if (tiles > (1 << 24)) return QB_ERR_INVALID_ARG;
    hipStream_t s = qb_hip_stream(stream);
    QB_LAUNCH(k_tile_work, qb_div_up(tiles, QB_BLOCK / 64), QB_BLOCK, 0, s, (int)width, (int)height, tiles_x,
              (int)tiles, reinterpret_cast<const uint2*>(ranges), ids, reinterpret_cast<const float4*>(splats), work);
    QB_LAUNCH(k_tile_order, 1, kOrderThreads, 0, s, (const uint32_t*)work, (int)tiles, order);
    return QB_OK;
}

extern "C" qb_status qb_tile_order_views(int32_t num_views, const qb_view* views, uint32_t* work, uint32_t* order,
                                         qb_stream_t stream)
{
    if (!work || !order) return QB_ERR_INVALID_ARG;
    QbViewTable vt;
    qb_status st = qb_make_view_table(num_views, views, false, &vt);
    if (st != QB_OK) return st;
    int tiles = vt.tile_start[num_views];
    if (tiles == 0) return QB_OK;
    hipStream_t s = qb_hip_stream(stream);
    QB_LAUNCH(k_tile_work_views, qb_div_up(tiles, QB_BLOCK / 64), QB_BLOCK, 0, s, vt, work);
    QB_LAUNCH(k_tile_order, 1, kOrderThreads, 0, s, (const uint32_t*)work, tiles, order);
    return QB_OK;
}
