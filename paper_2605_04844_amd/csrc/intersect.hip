// qb_intersect: DuplicateWithKeys with the QPass traversal (Sec. 2, Sec. 3.2).
//
//  1. key every Gaussian by its depth bits (0xFFFFFFFF when it covers no tile)
//     and stable-radix-sort the ids: the (depth, id) order of the final list
//  2. gather the tile counts in that order and scan them (pair offsets)
//  3. emit: each 256-lane workgroup takes 256 consecutive Gaussians of that
//     order, runs QPass for each (one lane per Gaussian) into run descriptors
//     in LDS, then enumerates the workgroup's pairs pair-parallel: lane p finds
//     its Gaussian by binary search over the LDS offsets and its tile by O(1)
//     decoding of the runs, so every lane writes one pair per step and the
//     stores of a wave are contiguous (coalesced 8-byte keys and 4-byte ids).
#include "qb_radix.h"

namespace {

constexpr int kEmitThreads = 256;

__global__ __launch_bounds__(QB_BLOCK) void k_depth_keys(int64_t n, const float4* __restrict__ splats,
                                                         const int32_t* __restrict__ counts,
                                                         uint32_t* __restrict__ keys,
                                                         uint32_t* __restrict__ vals)
{
    int64_t i = (int64_t)blockIdx.x * QB_BLOCK + threadIdx.x;
    if (i >= n) return;
    float d = splats[3 * i].z;
    keys[i] = counts[i] > 0 ? __float_as_uint(d) : 0xFFFFFFFFu;
    vals[i] = (uint32_t)i;
}

__global__ __launch_bounds__(QB_BLOCK) void k_gather_counts(int64_t n, const uint32_t* __restrict__ order,
                                                            const int32_t* __restrict__ counts,
                                                            uint32_t* __restrict__ out)
{
    int64_t i = (int64_t)blockIdx.x * QB_BLOCK + threadIdx.x;
    if (i >= n) return;
    out[i] = (uint32_t)counts[order[i]];
}

__device__ __forceinline__ QRect unpack_rect(int lohi_x, int lohi_y)
{
    QRect r;
    r.x0 = (int)(int16_t)(lohi_x & 0xFFFF);
    r.x1 = lohi_x >> 16;
    r.y0 = (int)(int16_t)(lohi_y & 0xFFFF);
    r.y1 = lohi_y >> 16;
    return r;
}

__global__ __launch_bounds__(kEmitThreads) void k_emit(
    int64_t n, const uint32_t* __restrict__ order, const uint64_t* __restrict__ offs,
    const float4* __restrict__ splats, const int4* __restrict__ rects,
    const int32_t* __restrict__ counts, int tiles_x, int64_t cap, const int64_t* __restrict__ num_pairs,
    uint64_t* __restrict__ keys, uint32_t* __restrict__ ids)
{
    __shared__ int64_t s_off[kEmitThreads + 1];   // pair offsets relative to the block start
    __shared__ QSeg s_seg[kEmitThreads][QB_MAX_SEG];
    __shared__ int s_nseg[kEmitThreads];
    __shared__ int s_axis[kEmitThreads];
    __shared__ uint32_t s_id[kEmitThreads];
    __shared__ uint32_t s_depth[kEmitThreads];

    if (*num_pairs > cap) return;  // overflow: the caller re-runs with more capacity
    int64_t k0 = (int64_t)blockIdx.x * kEmitThreads;
    int t = threadIdx.x;
    int64_t k = k0 + t;
    int64_t block_start = offs[k0];
    int cnt = 0;
    if (k < n) {
        uint32_t gi = order[k];
        cnt = counts[gi];
        s_id[t] = gi;
        s_off[t] = (int64_t)offs[k] - block_start;
        if (cnt > 0) {
            int4 p0 = rects[2 * (int64_t)gi], p1 = rects[2 * (int64_t)gi + 1];
            QRect r[4] = {unpack_rect(p0.x, p0.y), unpack_rect(p0.z, p0.w), unpack_rect(p1.x, p1.y),
                          unpack_rect(p1.z, p1.w)};
            int axis, total;
            QSeg seg[QB_MAX_SEG];
            int ns = qpass_segments(r, seg, &axis, &total);
            for (int s = 0; s < ns; ++s) s_seg[t][s] = seg[s];
            s_nseg[t] = ns;
            s_axis[t] = axis;
            s_depth[t] = __float_as_uint(splats[3 * (int64_t)gi].z);
            if (total != cnt) cnt = min(cnt, total);  // never write past the slot
        } else {
            s_nseg[t] = 0;
        }
    } else {
        s_off[t] = 0x7FFFFFFFFFFFFFFFll;  // beyond every pair of the block
        s_nseg[t] = 0;
    }
    // block pair total: offset of the last valid lane plus its count
    __shared__ int64_t s_total;
    int64_t last = min((int64_t)kEmitThreads, n - k0) - 1;
    if (t == (int)last) s_total = s_off[t] + cnt;
    __syncthreads();
    int64_t total = s_total;
    int nvalid = (int)(last + 1);
    for (int64_t p = t; p < total; p += kEmitThreads) {
        // last Gaussian whose offset is <= p (zero-count ones share offsets
        // with the next one and are skipped by taking the last match)
        int lo = 0, hi = nvalid;  // invariant: s_off[lo] <= p < s_off[hi] (s_off[nvalid] = +inf)
        while (hi - lo > 1) {
            int mid = (lo + hi) >> 1;
            if (s_off[mid] <= p) lo = mid; else hi = mid;
        }
        int j = lo;
        int64_t local = p - s_off[j];
        int ns = s_nseg[j];
        int tx = -1, ty = -1;
        for (int s = 0; s < ns; ++s) {
            QSeg g = s_seg[j][s];
            int64_t sz = (int64_t)g.n * g.len;
            if (local < sz) {
                int q = (int)(local / g.len);
                int rem = (int)(local - (int64_t)q * g.len);
                int sl = g.s0 + q, ot = g.lo + rem;
                if (s_axis[j] == 0) { tx = sl; ty = ot; } else { tx = ot; ty = sl; }
                break;
            }
            local -= sz;
        }
        if (tx < 0) continue;  // unreachable when counts match the runs
        int64_t dst = block_start + p;
        if (dst >= cap) break;
        keys[dst] = ((uint64_t)(uint32_t)(ty * tiles_x + tx) << 32) | s_depth[j];
        ids[dst] = s_id[j];
    }
}

__global__ void k_store_total(const uint64_t* __restrict__ tot, int64_t* __restrict__ num_pairs)
{
    *num_pairs = (int64_t)*tot;
}

struct IsectWs {
    uint32_t *dk0, *dv0, *dk1, *dv1;  // depth sort ping-pong
    uint32_t* csorted;                // counts in sorted order
    uint64_t* offs;                   // n + 1 offsets
    uint64_t* total;
    uint64_t* scan64;
    uint32_t* radix;
};

IsectWs carve(QbArena& a, int64_t n)
{
    IsectWs w;
    w.dk0 = a.take<uint32_t>(n);
    w.dv0 = a.take<uint32_t>(n);
    w.dk1 = a.take<uint32_t>(n);
    w.dv1 = a.take<uint32_t>(n);
    w.csorted = a.take<uint32_t>(n);
    w.offs = a.take<uint64_t>(n + 1);
    w.total = a.take<uint64_t>(1);
    w.scan64 = a.take<uint64_t>(qbr::scan_scratch(n));
    w.radix = a.take<uint32_t>((int64_t)(qbr::radix_scratch_bytes(n) / sizeof(uint32_t)));
    return w;
}

}  // namespace

extern "C" size_t qb_intersect_workspace_size(int64_t n)
{
    if (n < 0) return 0;
    QbArena a{nullptr, 0, 0};
    carve(a, n);
    return a.used + 256;
}

extern "C" qb_status qb_intersect(int64_t n, const qb_splat* splats, const qb_rects* rects,
                                  const int32_t* counts, int32_t width, int32_t height,
                                  int64_t pair_capacity, uint64_t* keys, uint32_t* ids,
                                  int64_t* num_pairs, void* workspace, size_t workspace_bytes,
                                  qb_stream_t stream)
{
    if (n < 0 || n >= (int64_t)1 << 31 || width <= 0 || height <= 0 || pair_capacity < 0 ||
        pair_capacity > (int64_t)0xFFFFFFFF || !num_pairs)
        return QB_ERR_INVALID_ARG;
    if (width > 32767 * QB_TILE || height > 32767 * QB_TILE) return QB_ERR_INVALID_ARG;
    if (n > 0 && (!splats || !rects || !counts || !workspace)) return QB_ERR_INVALID_ARG;
    if (pair_capacity > 0 && (!keys || !ids)) return QB_ERR_INVALID_ARG;
    if (workspace_bytes < qb_intersect_workspace_size(n)) return QB_ERR_INVALID_ARG;
    hipStream_t s = qb_hip_stream(stream);
    if (n == 0) {
        if (hipMemsetAsync(num_pairs, 0, sizeof(int64_t), s) != hipSuccess) return QB_ERR_HIP;
        return QB_OK;
    }
    QbArena a{(char*)(((uintptr_t)workspace + 255) & ~(uintptr_t)255), workspace_bytes - 256, 0};
    IsectWs w = carve(a, n);
    if (!a.ok()) return QB_ERR_INVALID_ARG;
    int tiles_x = (int)qb_div_up(width, QB_TILE);
    int64_t grid = qb_div_up(n, QB_BLOCK);
    const float4* sp = reinterpret_cast<const float4*>(splats);
    QB_LAUNCH(k_depth_keys, grid, QB_BLOCK, 0, s, n, sp, counts, w.dk0, w.dv0);
    // four 8-bit passes: ends back in (dk0, dv0)
    QB_CHECK((qbr::radix_sort<uint32_t>(w.dk0, w.dv0, w.dk0, w.dv0, w.dk1, w.dv1, (const int64_t*)nullptr, n, n,
                                        0, 32, w.radix, s)));
    const uint32_t* order = w.dv0;
    QB_LAUNCH(k_gather_counts, grid, QB_BLOCK, 0, s, n, order, counts, w.csorted);
    QB_CHECK((qbr::exclusive_scan<uint32_t, uint64_t>(w.csorted, w.offs, n, w.scan64, w.total, s)));
    QB_LAUNCH(k_store_total, 1, 1, 0, s, (const uint64_t*)w.total, num_pairs);
    QB_LAUNCH(k_emit, qb_div_up(n, kEmitThreads), kEmitThreads, 0, s, n, order, (const uint64_t*)w.offs, sp,
              reinterpret_cast<const int4*>(rects), counts, tiles_x, pair_capacity, (const int64_t*)num_pairs,
              keys, ids);
    return QB_OK;
}
