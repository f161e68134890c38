// qb_render: per-tile front-to-back alpha compositing, Eq. (2).
//
// One workgroup per 16x16 tile; by default 128 lanes (two wave64), each lane
// owning the two pixels (x, y) and (x + 8, y) of one row, so the
// row-dependent terms of the quadratic form and every LDS read are shared by
// two pixels.  The tile's depth-sorted list is walked in batches of one
// record per lane: each lane gathers one
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

// Tiles go to workgroups in the order qb_tile_order computes (estimated
// work, heaviest first: every workgroup is resident from the start, so this
// order decides how evenly the SIMDs are loaded), or in row-major order
// without one.  Row-major was measured faster than giving each XCD a
// contiguous band of tiles (the dispatcher deals workgroups round-robin to
// the 8 XCDs, so row-major spreads a dense region over all of them).
//
// Launch shape: PPL pixels per lane, all in one row of the tile, 16/PPL
// apart (256/PPL lanes per tile).  The row terms of the quadratic form and
// every LDS read are shared by a lane's PPL pixels; the batch staged in LDS
// holds one record per lane.  qb_render_ex selects PPL (1, 2 or 4).  When a
// wave covers fewer than 16 rows (PPL 1 or 2), each staged batch also gets,
// per wave, a ballot mask of the entries whose cutoff ellipse can reach the
// wave's rows (entry_rows), and the wave walks only those entries.
// x of lane (l & AND) | j of each 32-lane half (ds_swizzle, bitmask mode):
// with AND clearing the low bits of a group of 2^m lanes, lane j of every
// group broadcast to its group.
template <int AND, int J>
__device__ __forceinline__ float bcast_lane_c(float x)
{
    return __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(x), AND | (J << 5)));
}

// the same with j known only after unrolling (0 <= j < 16); the switch folds
template <int AND>
__device__ __forceinline__ float bcast_lane(float x, int j)
{
    switch (j) {
    case 0: return bcast_lane_c<AND, 0>(x);
    case 1: return bcast_lane_c<AND, 1>(x);
    case 2: return bcast_lane_c<AND, 2>(x);
    case 3: return bcast_lane_c<AND, 3>(x);
    case 4: return bcast_lane_c<AND, 4>(x);
    case 5: return bcast_lane_c<AND, 5>(x);
    case 6: return bcast_lane_c<AND, 6>(x);
    case 7: return bcast_lane_c<AND, 7>(x);
    case 8: return bcast_lane_c<AND, 8>(x);
    case 9: return bcast_lane_c<AND, 9>(x);
    case 10: return bcast_lane_c<AND, 10>(x);
    case 11: return bcast_lane_c<AND, 11>(x);
    case 12: return bcast_lane_c<AND, 12>(x);
    case 13: return bcast_lane_c<AND, 13>(x);
    case 14: return bcast_lane_c<AND, 14>(x);
    default: return bcast_lane_c<AND, 15>(x);
    }
}

template <int PPL, bool COUNT, bool SKIP, int XROW>
__device__ __forceinline__ void render_tile(int tile, int W, int H, int tiles_x, const uint2* __restrict__ ranges,
                                            const uint32_t* __restrict__ ids, const float4* __restrict__ splats,
                                            float bg0, float bg1, float bg2, float* __restrict__ image,
                                            float* __restrict__ final_T, uint32_t* __restrict__ n_contrib,
                                            uint32_t* __restrict__ n_touched, uint32_t* __restrict__ n_composited)
{
    constexpr int NT = 256 / PPL;        // lanes per tile
    constexpr int LX = QB_TILE / PPL;    // lanes per tile row
    __shared__ float4 s_geo[NT];   // u, v, -a/2, -b
    __shared__ float4 s_opa[NT];   // -c/2, o, -gamma/2, log2(o)
    __shared__ float4 s_col[NT];   // r, g, b, unused
    __shared__ int s_rows[NT];     // tile rows that can pass the cutoff (entry_rows)

    constexpr int kRowsPerWave = 64 / LX;   // tile rows a wave covers
    constexpr bool kSkip = SKIP && kRowsPerWave < QB_TILE;
    constexpr int NM = NT / 64;             // 64-entry masks per batch
    int tx = tile % tiles_x, ty = tile / tiles_x;
    int lx = threadIdx.x % LX, ly = threadIdx.x / LX;
    int py = ty * QB_TILE + ly;
    int lane = threadIdx.x & 63;
    int wrow0 = (int)(threadIdx.x / 64) * kRowsPerWave;
    float fy = (float)py;
    // The walk reads the staged batch through bases held in a vector
    // register: a zero that the compiler cannot prove uniform, so each run of
    // entries gets its address once and every LDS read an immediate offset
    // (with the arrays' own uniform bases, the compiler copies a scalar base
    // into a vector register again before nearly every read).
    int vzero;
    asm volatile("v_mov_b32 %0, 0" : "=v"(vzero));
    // A pixel that has stopped (or lies outside the image) has its x set to
    // +inf: dx is then -inf and, the conic's a being positive, its power
    // -inf, so the cutoff test rejects it by itself (a NaN power, possible
    // only there, is rejected too).
    constexpr float kStopped = __builtin_huge_valf();
    constexpr float kLog2e = 1.44269504088896341f;
    bool in[PPL];
    float fxp[PPL], T[PPL], c0[PPL], c1[PPL], c2[PPL];
    uint32_t last[PPL], stop[PPL], comp[PPL];
#pragma unroll
    for (int q = 0; q < PPL; ++q) {
        int px = tx * QB_TILE + lx + q * LX;
        in[q] = px < W && py < H;
        fxp[q] = in[q] ? (float)px : kStopped;
        T[q] = 1.0f;
        c0[q] = c1[q] = c2[q] = 0.0f;
        last[q] = stop[q] = comp[q] = 0u;
    }
    auto all_done = [&]() {
        bool d = true;
#pragma unroll
        for (int q = 0; q < PPL; ++q) d = d && fxp[q] == kStopped;
        return d;
    };

    const float4* geo = s_geo + vzero;
    const float4* opa = s_opa + vzero;
    const float4* col = s_col + vzero;

    uint2 rg = ranges[tile];
    int64_t start = rg.x, end = rg.y;
    for (int64_t base = start; base < end; base += NT) {
        if (__syncthreads_count(all_done()) == NT) break;
        int64_t j = base + threadIdx.x;
        if (j < end) {
            uint32_t id = ids[j];
            float4 a = splats[3 * (int64_t)id + 0];   // u, v, depth, o
            float4 b = splats[3 * (int64_t)id + 1];   // a, b, c, gamma
            float4 c = splats[3 * (int64_t)id + 2];   // r, g, b, visible
            s_geo[threadIdx.x] = make_float4(a.x, a.y, -0.5f * b.x, -b.y);
            s_opa[threadIdx.x] = make_float4(-0.5f * b.z, a.w, -0.5f * b.w, __log2f(a.w));
            s_col[threadIdx.x] = c;
            if (kSkip) s_rows[threadIdx.x] = entry_rows(a.y, b.x, b.y, b.z, b.w, ty);
        }
        __syncthreads();
        int cnt = (int)min((int64_t)NT, end - base);
        uint32_t idx0 = (uint32_t)(base - start);
        // one list entry k of the batch for every pixel of the lane; returns
        // true when the whole wave has stopped
        // composites one entry (log2 of the opacity in o.w, colour col, list
        // position at) into the lane's pixels whose power p passed (act):
        //   alpha = min(0.99, o e^p) = min(0.99, 2^(p log2(e) + log2(o))), one
        //           fma ahead of the exp instead of two multiplies
        //   T'    = T - alpha T with one rounding (fma)
        //   w     = T - T', which is alpha T up to the rounding of T' (the
        //           subtraction is exact while alpha <= 1/2) and 0 where the
        //           pixel adds nothing, so the weights and the final T sum to 1
        auto composite = [&](const float4& o, const float4& col, const float* p, const bool* act, uint32_t at,
                             bool* stopped) {
#pragma unroll
            for (int q = 0; q < PPL; ++q) {
                float alpha = fminf(0.99f, __builtin_amdgcn_exp2f(fmaf(p[q], kLog2e, o.w)));
                float test_T = fmaf(-alpha, T[q], T[q]);
                // T is never NaN, so !(test_T < 1e-4) is test_T >= 1e-4; one
                // compare gives both masks
                bool add = act[q] && test_T >= 1e-4f;
                bool stp = act[q] && !add;
                float Tn = add ? test_T : T[q];
                float w = T[q] - Tn;
                c0[q] = fmaf(col.x, w, c0[q]);
                c1[q] = fmaf(col.y, w, c1[q]);
                c2[q] = fmaf(col.z, w, c2[q]);
                T[q] = Tn;
                last[q] = add ? at : last[q];
                if (COUNT) stop[q] = stp ? at : stop[q];
                if (COUNT) comp[q] += add ? 1u : 0u;
                fxp[q] = stp ? kStopped : fxp[q];
                stopped[q] = stp;
            }
        };
        // the cutoff test of entry k for the lane's pixels; returns whether any passed
        auto test = [&](int k, float4& o, float* p, bool* act) -> bool {
            float4 g = geo[k];
            o = opa[k];
            // the terms of the quadratic form that depend on the row only
            float dy = g.y - fy;
            float nbdy = g.w * dy;
            float hcdy2 = (o.x * dy) * dy;
            bool any = false;
#pragma unroll
            for (int q = 0; q < PPL; ++q) {
                float dx = g.x - fxp[q];
                p[q] = fmaf(fmaf(g.z, dx, nbdy), dx, hcdy2);
                act[q] = !(p[q] > 0.0f) && p[q] >= o.z;
                any = any || act[q];
            }
            return any;
        };
        // the cutoff test with the row terms (-b) dy and ((-c/2) dy) dy given
        auto test_rt = [&](int k, float nbdy, float hcdy2, float4& o, float* p, bool* act) -> bool {
            float4 g = geo[k];
            o = opa[k];
            bool any = false;
#pragma unroll
            for (int q = 0; q < PPL; ++q) {
                float dx = g.x - fxp[q];
                p[q] = fmaf(fmaf(g.z, dx, nbdy), dx, hcdy2);
                act[q] = !(p[q] > 0.0f) && p[q] >= o.z;
                any = any || act[q];
            }
            return any;
        };
        // entry k with its row terms given
        auto entry_rt = [&](int k, float nb, float hc) -> bool {
            float4 o;
            float p[PPL];
            bool act[PPL];
            if (!__any(test_rt(k, nb, hc, o, p, act))) return false;
            bool stopped[PPL];
            composite(o, col[k], p, act, idx0 + (uint32_t)k + 1u, stopped);
            return __all(all_done());
        };
        // entries k and k + 1 with their row terms given
        auto entry2_rt = [&](int k, float nba, float hca, float nbb, float hcb) -> bool {
            float4 oa, ob;
            float pa[PPL], pb[PPL];
            bool acta[PPL], actb[PPL];
            bool any = test_rt(k, nba, hca, oa, pa, acta);
            any = test_rt(k + 1, nbb, hcb, ob, pb, actb) || any;
            if (!__any(any)) return false;
            bool stopped[PPL];
            composite(oa, col[k], pa, acta, idx0 + (uint32_t)k + 1u, stopped);
#pragma unroll
            for (int q = 0; q < PPL; ++q) actb[q] = actb[q] && !stopped[q];   // a pixel may have stopped at k
            composite(ob, col[k + 1], pb, actb, idx0 + (uint32_t)k + 2u, stopped);
            return __all(all_done());
        };
        // one list entry k of the batch; returns true when the whole wave has stopped
        auto entry = [&](int k) -> bool {
            float4 o;
            float p[PPL];
            bool act[PPL];
            bool any = test(k, o, p, act);
            // branch only when the whole wave agrees; per pixel, select
            if (!__any(any)) return false;
            bool stopped[PPL];
            composite(o, col[k], p, act, idx0 + (uint32_t)k + 1u, stopped);
            return __all(all_done());
        };
        // entries k and k + 1: both tests first (independent), one uniform
        // branch for the pair, then the two composites in list order
        auto entry2 = [&](int k) -> bool {
            float4 oa, ob;
            float pa[PPL], pb[PPL];
            bool acta[PPL], actb[PPL];
            bool any = test(k, oa, pa, acta);
            any = test(k + 1, ob, pb, actb) || any;
            if (!__any(any)) return false;
            bool stopped[PPL];
            composite(oa, col[k], pa, acta, idx0 + (uint32_t)k + 1u, stopped);
#pragma unroll
            for (int q = 0; q < PPL; ++q) actb[q] = actb[q] && !stopped[q];   // a pixel may have stopped at k
            composite(ob, col[k + 1], pb, actb, idx0 + (uint32_t)k + 2u, stopped);
            return __all(all_done());
        };
        if (kSkip) {
            // entries of this batch whose ellipse can reach this wave's rows,
            // one bit each (uniform masks), walked in order.  Leave the batch
            // only when the whole wave is done: every lane takes part in the
            // ballots (lane l contributes entry m * 64 + l).
            if (__all(all_done())) continue;
            uint64_t mask[NM];
#pragma unroll
            for (int m = 0; m < NM; ++m) {
                int k = m * 64 + lane;
                bool rel = k < cnt;
                if (rel) {
                    int rr = s_rows[k];
                    int r0 = (int)(int16_t)(rr & 0xFFFF), r1 = rr >> 16;
                    rel = !(r1 < wrow0 || r0 > wrow0 + kRowsPerWave - 1);
                }
                mask[m] = __ballot(rel);
            }
            bool finished = false;
#pragma unroll
            for (int m = 0; m < NM; ++m) {
                uint64_t bits = finished ? 0ull : mask[m];
                while (bits) {
                    int k = m * 64 + (int)__builtin_ctzll(bits);
                    bits &= bits - 1;
                    if (entry(k)) { finished = true; break; }
                }
            }
        } else {
            // a lane whose pixels have all stopped sits the batch out, except
            // with shared row terms: there every lane of a row is a source of
            // the broadcasts, so the wave walks on until all of it has
            // stopped (a stopped pixel's test rejects every entry by itself)
            if (XROW ? __all(all_done()) : all_done()) continue;
            // whether the whole wave has stopped is asked once per 8 pairs:
            // after that, entries find no active pixel and only run the
            // tests, which is cheaper than the vote on every pair
            bool finished = false;
            int k = 0;
            constexpr int kPairsPerCheck = 8;
            for (; k + 2 * kPairsPerCheck - 1 < cnt; k += 2 * kPairsPerCheck) {
                if constexpr (XROW) {
                    // The row terms of an entry are the same for the LX lanes
                    // of one tile row: lane lx of the row computes them for
                    // entries k + c LX + lx, and a swizzle within each group of
                    // LX lanes hands entry k + c LX + j's terms from lane j to
                    // the group.  Same values, one lane computing each.
                    constexpr int kChunks = 2 * kPairsPerCheck / LX;
                    float tnb[kChunks], thc[kChunks];
#pragma unroll
                    for (int c = 0; c < kChunks; ++c) {
                        int e = k + c * LX + lx;
                        float4 gg = geo[e];
                        float ox = opa[e].x;
                        float dy = gg.y - fy;
                        tnb[c] = gg.w * dy;
                        thc[c] = (ox * dy) * dy;
                    }
                    constexpr int kAnd = 0x1F & ~(LX - 1);
                    bool fin = false;
                    if constexpr (XROW == 1) {
                        // entries in pairs: both tests, one branch
#pragma unroll
                        for (int c = 0; c < kPairsPerCheck; ++c) {
                            int e0 = 2 * c, e1 = 2 * c + 1;
                            float nba = bcast_lane<kAnd>(tnb[e0 / LX], e0 % LX);
                            float hca = bcast_lane<kAnd>(thc[e0 / LX], e0 % LX);
                            float nbb = bcast_lane<kAnd>(tnb[e1 / LX], e1 % LX);
                            float hcb = bcast_lane<kAnd>(thc[e1 / LX], e1 % LX);
                            bool done = entry2_rt(k + e0, nba, hca, nbb, hcb);
                            if (c == kPairsPerCheck - 1) fin = done;
                        }
                    } else {
                        // one branch per entry: no composite for an entry
                        // that no pixel of the wave passes
#pragma unroll
                        for (int e = 0; e < 2 * kPairsPerCheck; ++e) {
                            float nb = bcast_lane<kAnd>(tnb[e / LX], e % LX);
                            float hc = bcast_lane<kAnd>(thc[e / LX], e % LX);
                            bool done = entry_rt(k + e, nb, hc);
                            if (e == 2 * kPairsPerCheck - 1) fin = done;
                        }
                    }
                    if (fin) { finished = true; break; }
                } else {
#pragma unroll
                    for (int c = 0; c < kPairsPerCheck - 1; ++c) entry2(k + 2 * c);
                    if (entry2(k + 2 * (kPairsPerCheck - 1))) { finished = true; break; }
                }
            }
            for (; !finished && k + 1 < cnt; k += 2)
                if (entry2(k)) { finished = true; break; }
            if (!finished && k < cnt) entry(k);
        }
    }
    uint32_t len = (uint32_t)(end - start);
    int64_t plane = (int64_t)W * H;
#pragma unroll
    for (int q = 0; q < PPL; ++q) {
        if (!in[q]) continue;
        int64_t pix = (int64_t)py * W + tx * QB_TILE + lx + q * LX;
        image[pix] = fmaf(T[q], bg0, c0[q]);
        image[plane + pix] = fmaf(T[q], bg1, c1[q]);
        image[2 * plane + pix] = fmaf(T[q], bg2, c2[q]);
        if (final_T) final_T[pix] = T[q];
        if (n_contrib) n_contrib[pix] = last[q];
        if (COUNT) n_touched[pix] = fxp[q] == kStopped ? stop[q] : len;
        if (COUNT && n_composited) n_composited[pix] = comp[q];
    }
}

// COUNT: also write n_touched (entries examined per pixel) and, when given,
// n_composited (entries composited per pixel), compiled out of the launches
// that do not ask for them.  Workgroup i takes tile order[i]
// (qb_tile_order), or tile i when order is NULL; an entry past the last tile
// is skipped.
template <int PPL, bool COUNT, bool SKIP, int XROW>
__global__ __launch_bounds__(256 / PPL) void k_render(
    int W, int H, int tiles_x, const uint2* __restrict__ ranges, const uint32_t* __restrict__ ids,
    const float4* __restrict__ splats, float bg0, float bg1, float bg2, float* __restrict__ image,
    float* __restrict__ final_T, uint32_t* __restrict__ n_contrib, uint32_t* __restrict__ n_touched,
    uint32_t* __restrict__ n_composited, const uint32_t* __restrict__ order)
{
    uint32_t tile = order ? order[blockIdx.x] : blockIdx.x;
    if (tile >= gridDim.x) return;
    render_tile<PPL, COUNT, SKIP, XROW>((int)tile, W, H, tiles_x, ranges, ids, splats, bg0, bg1, bg2, image, final_T,
                                  n_contrib, n_touched, n_composited);
}

// Every tile of every view in one launch: workgroup i takes global tile
// order[i] (or i), whose view is found in the (at most QB_MAX_VIEWS) tile
// offsets.
template <int PPL, bool SKIP, int XROW>
__global__ __launch_bounds__(256 / PPL) void k_render_views(QbViewTable vt, const uint32_t* __restrict__ order,
                                                            float bg0, float bg1, float bg2)
{
    uint32_t g = order ? order[blockIdx.x] : blockIdx.x;
    if (g >= gridDim.x) return;
    int b = (int)g;
    int v = qb_view_of(vt, b);
    const qb_view& w = vt.view[v];
    render_tile<PPL, false, SKIP, XROW>(b - vt.tile_start[v], w.width, w.height, vt.tiles_x[v], reinterpret_cast<const uint2*>(w.ranges),
                     w.ids, reinterpret_cast<const float4*>(w.splats), bg0, bg1, bg2, w.image, w.final_T, w.n_contrib,
                     nullptr, nullptr);
}

}  // namespace

// Launches render variant `variant` (qb_render_variant) over `tiles` tiles.
template <bool COUNT>
static qb_status launch_render(int variant, int64_t tiles, hipStream_t s, int W, int H, int tiles_x,
                               const uint2* rg, const uint32_t* ids, const float4* sp, const float* bg, float* image,
                               float* final_T, uint32_t* n_contrib, uint32_t* n_touched, uint32_t* n_composited,
                               const uint32_t* order)
{
#define QB_RENDER_LAUNCH(P, SK, XR)                                                                      \
    QB_LAUNCH((k_render<P, COUNT, SK, XR>), tiles, 256 / P, 0, s, W, H, tiles_x, rg, ids, sp, bg[0], bg[1], bg[2], \
              image, final_T, n_contrib, n_touched, n_composited, order)
    switch (variant) {
    case QB_RENDER_2PX: QB_RENDER_LAUNCH(2, false, 0); break;
    case QB_RENDER_1PX: QB_RENDER_LAUNCH(1, false, 0); break;
    case QB_RENDER_4PX: QB_RENDER_LAUNCH(4, false, 0); break;
    case QB_RENDER_2PX_ROWS: QB_RENDER_LAUNCH(2, true, 0); break;
    case QB_RENDER_1PX_ROWS: QB_RENDER_LAUNCH(1, true, 0); break;
    case QB_RENDER_2PX_XROW: QB_RENDER_LAUNCH(2, false, 1); break;
    case QB_RENDER_4PX_XROW: QB_RENDER_LAUNCH(4, false, 1); break;
    default: QB_RENDER_LAUNCH(2, false, 2); break;
    }
#undef QB_RENDER_LAUNCH
    return QB_OK;
}

extern "C" qb_status qb_render_ex(int32_t width, int32_t height, const uint32_t* ranges, const uint32_t* ids,
                                  const qb_splat* splats, const float* bg, float* image, float* final_T,
                                  uint32_t* n_contrib, uint32_t* n_touched, int32_t variant,
                                  const uint32_t* tile_order, qb_stream_t stream)
{
    if (width <= 0 || height <= 0 || width > 32767 * QB_TILE || height > 32767 * QB_TILE || !ranges ||
        !image || !bg || variant < 0 || variant >= QB_RENDER_VARIANTS)
        return QB_ERR_INVALID_ARG;
    int tiles_x = (int)qb_div_up(width, QB_TILE);
    int64_t tiles = (int64_t)tiles_x * qb_div_up(height, QB_TILE);
    if (tiles > (1 << 24)) return QB_ERR_INVALID_ARG;
    hipStream_t s = qb_hip_stream(stream);
    const uint2* rg = reinterpret_cast<const uint2*>(ranges);
    const float4* sp = reinterpret_cast<const float4*>(splats);
    if (n_touched)
        return launch_render<true>(variant, tiles, s, (int)width, (int)height, tiles_x, rg, ids, sp, bg, image, final_T,
                                   n_contrib, n_touched, nullptr, tile_order);
    return launch_render<false>(variant, tiles, s, (int)width, (int)height, tiles_x, rg, ids, sp, bg, image, final_T,
                                n_contrib, nullptr, nullptr, tile_order);
}

extern "C" qb_status qb_render_stats(int32_t width, int32_t height, const uint32_t* ranges, const uint32_t* ids,
                                     const qb_splat* splats, const float* bg, float* image, float* final_T,
                                     uint32_t* n_contrib, uint32_t* n_touched, uint32_t* n_composited,
                                     int32_t variant, const uint32_t* tile_order, qb_stream_t stream)
{
    if (width <= 0 || height <= 0 || width > 32767 * QB_TILE || height > 32767 * QB_TILE || !ranges ||
        !image || !bg || !n_touched || !n_composited || variant < 0 || variant >= QB_RENDER_VARIANTS)
        return QB_ERR_INVALID_ARG;
    int tiles_x = (int)qb_div_up(width, QB_TILE);
    int64_t tiles = (int64_t)tiles_x * qb_div_up(height, QB_TILE);
    if (tiles > (1 << 24)) return QB_ERR_INVALID_ARG;
    return launch_render<true>(variant, tiles, qb_hip_stream(stream), (int)width, (int)height, tiles_x,
                               reinterpret_cast<const uint2*>(ranges), ids, reinterpret_cast<const float4*>(splats),
                               bg, image, final_T, n_contrib, n_touched, n_composited, tile_order);
}

extern "C" qb_status qb_render(int32_t width, int32_t height, const uint32_t* ranges, const uint32_t* ids,
                               const qb_splat* splats, const float* bg, float* image, float* final_T,
                               uint32_t* n_contrib, uint32_t* n_touched, qb_stream_t stream)
{
    return qb_render_ex(width, height, ranges, ids, splats, bg, image, final_T, n_contrib, n_touched, QB_RENDER_2PX,
                        nullptr, stream);
}

extern "C" qb_status qb_render_views_ex(int32_t num_views, const qb_view* views, const float* bg, int32_t variant,
                                        const uint32_t* tile_order, qb_stream_t stream)
{
    if (!bg || variant < 0 || variant >= QB_RENDER_VARIANTS) return QB_ERR_INVALID_ARG;
    QbViewTable vt;
    qb_status st = qb_make_view_table(num_views, views, false, &vt);
    if (st != QB_OK) return st;
    int tiles = vt.tile_start[num_views];
    if (tiles == 0) return QB_OK;
    hipStream_t s = qb_hip_stream(stream);
#define QB_RENDER_VIEWS(P, SK, XR) \
    QB_LAUNCH((k_render_views<P, SK, XR>), tiles, 256 / P, 0, s, vt, tile_order, bg[0], bg[1], bg[2])
    switch (variant) {
    case QB_RENDER_2PX: QB_RENDER_VIEWS(2, false, 0); break;
    case QB_RENDER_1PX: QB_RENDER_VIEWS(1, false, 0); break;
    case QB_RENDER_4PX: QB_RENDER_VIEWS(4, false, 0); break;
    case QB_RENDER_2PX_ROWS: QB_RENDER_VIEWS(2, true, 0); break;
    case QB_RENDER_1PX_ROWS: QB_RENDER_VIEWS(1, true, 0); break;
    case QB_RENDER_2PX_XROW: QB_RENDER_VIEWS(2, false, 1); break;
    case QB_RENDER_4PX_XROW: QB_RENDER_VIEWS(4, false, 1); break;
    default: QB_RENDER_VIEWS(2, false, 2); break;
    }
#undef QB_RENDER_VIEWS
    return QB_OK;
}

extern "C" qb_status qb_render_views(int32_t num_views, const qb_view* views, const float* bg, qb_stream_t stream)
{
    return qb_render_views_ex(num_views, views, bg, QB_RENDER_2PX, nullptr, stream);
}
