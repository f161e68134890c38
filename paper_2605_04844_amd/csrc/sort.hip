// qb_sort: SortPairs (Sec. 2) and the per-tile ranges of the sorted list.
//
// qb_intersect emits the pairs grouped by Gaussian in ascending (depth, id)
// order, so the full (tile, depth, id) order is reached by a stable LSD radix
// sort over the tile bits of the key alone (ceil(log2 tiles) bits: one pass at
// 256 tiles, two at 3600-8160).  Ranges come from two binary searches per
// tile over the sorted keys (lower bounds of t<<32 and (t+1)<<32), which also
// places empty tiles exactly.
#include "qb_radix.h"

namespace {

__global__ __launch_bounds__(QB_BLOCK) void k_ranges(const uint64_t* __restrict__ keys,
                                                     const int64_t* __restrict__ num_pairs, int64_t cap,
                                                     int num_tiles, uint32_t* __restrict__ ranges)
{
    int t = blockIdx.x * QB_BLOCK + threadIdx.x;
    if (t >= num_tiles) return;
    int64_t n = qbr::sort_count(num_pairs, 0, cap);
    uint32_t bound[2];
#pragma unroll
    for (int e = 0; e < 2; ++e) {
        uint64_t target = (uint64_t)(uint32_t)(t + e) << 32;
        int64_t lo = 0, hi = n;
        while (lo < hi) {
            int64_t mid = lo + ((hi - lo) >> 1);
            if (keys[mid] < target) lo = mid + 1; else hi = mid;
        }
        bound[e] = (uint32_t)lo;
    }
    reinterpret_cast<uint2*>(ranges)[t] = make_uint2(bound[0], bound[1]);
}

int tile_bits(int num_tiles)
{
    int b = 0;
    while ((1ll << b) < (long long)num_tiles) ++b;
    return b;
}

struct SortWs {
    uint64_t* ktmp;
    uint32_t* vtmp;
    uint32_t* radix;
};

SortWs carve(QbArena& a, int64_t cap)
{
    SortWs w;
    w.ktmp = a.take<uint64_t>(cap);
    w.vtmp = a.take<uint32_t>(cap);
    w.radix = a.take<uint32_t>((int64_t)(qbr::radix_scratch_bytes(cap) / sizeof(uint32_t)));
    return w;
}

}  // namespace

extern "C" size_t qb_sort_workspace_size(int64_t pair_capacity, int32_t num_tiles)
{
    (void)num_tiles;
    if (pair_capacity < 0) return 0;
    QbArena a{nullptr, 0, 0};
    carve(a, pair_capacity);
    return a.used + 256;
}

extern "C" qb_status qb_sort(int64_t pair_capacity, const int64_t* num_pairs, int32_t num_tiles,
                             const uint64_t* keys_in, const uint32_t* ids_in, uint64_t* keys_out,
                             uint32_t* ids_out, uint32_t* ranges, void* workspace,
                             size_t workspace_bytes, qb_stream_t stream)
{
    if (pair_capacity < 0 || pair_capacity > (int64_t)0xFFFFFFFF || !num_pairs || num_tiles < 1 ||
        num_tiles > (1 << 24) || !ranges || !workspace)
        return QB_ERR_INVALID_ARG;
    if (pair_capacity > 0 && (!keys_in || !ids_in || !keys_out || !ids_out)) return QB_ERR_INVALID_ARG;
    if ((const void*)keys_in == (const void*)keys_out || (const void*)ids_in == (const void*)ids_out)
        return QB_ERR_INVALID_ARG;
    if (workspace_bytes < qb_sort_workspace_size(pair_capacity, num_tiles)) return QB_ERR_INVALID_ARG;
    hipStream_t s = qb_hip_stream(stream);
    QbArena a{(char*)(((uintptr_t)workspace + 255) & ~(uintptr_t)255), workspace_bytes - 256, 0};
    SortWs w = carve(a, pair_capacity);
    if (!a.ok()) return QB_ERR_INVALID_ARG;
    int tb = tile_bits(num_tiles);
    QB_CHECK((qbr::radix_sort<uint64_t>(keys_in, ids_in, keys_out, ids_out, w.ktmp, w.vtmp, num_pairs, 0,
                                        pair_capacity, 32, 32 + tb, w.radix, s)));
    QB_LAUNCH(k_ranges, qb_div_up(num_tiles, QB_BLOCK), QB_BLOCK, 0, s, (const uint64_t*)keys_out, num_pairs,
              pair_capacity, (int)num_tiles, ranges);
    return QB_OK;
}
