// qb_sort: SortPairs (Sec. 2) and the per-tile ranges of the sorted list.
//
// qb_intersect emits the pairs grouped by Gaussian in ascending (depth, id)
// order, so the full (tile, depth, id) order is reached by a stable LSD radix
// sort over the tile bits alone: ceil(log2 tiles) bits in passes of at most
// 8 (one pass at 256 tiles, two of 6-7 bits at 3600-8160).  Each pass stages
// its items in LDS by digit and writes them as contiguous runs.  Ranges come
// from two searches per tile over the sorted tiles (lower bounds of t and
// t+1), which also places empty tiles exactly.  The 64-bit keys
// tile << 32 | bits(depth) are written only when asked for.
#include "qb_radix.h"

namespace {

// Radix workgroup shapes (lanes, pairs per lane), indexed by qb_sort_variant;
// 512 x 8 (4096 pairs per workgroup) is qb_sort's.  The workspace covers the
// shape with the most workgroups (the smallest tile).
constexpr int kSortMinTile = 4096;

// One wave per tile: lanes 0-31 find the first index whose tile is >= t,
// lanes 32-63 the first whose tile is >= t + 1, each half by a 32-ary
// search.  Invariant: every index below lo holds a smaller tile, every index
// from hi on a tile >= the target.  A round probes 32 points that split
// [lo, hi) into 33 parts; the probes below the target form a prefix (the
// list is sorted), so their count c (one ballot) names the part that holds
// the bound.  Once hi - lo <= 32 the candidates themselves are probed.  At
// 10^7 - 10^8 pairs that is five rounds of one gather each, against the 25
// dependent loads of a per-thread binary search.
__global__ __launch_bounds__(QB_BLOCK) void k_ranges(const uint16_t* __restrict__ tiles,
                                                     const int64_t* __restrict__ num_pairs, int64_t cap,
                                                     int num_tiles, uint32_t* __restrict__ ranges)
{
    int t = blockIdx.x * (QB_BLOCK / 64) + (int)(threadIdx.x / 64);
    if (t >= num_tiles) return;
    int lane = threadIdx.x & 63, half = lane >> 5, k = lane & 31;
    int64_t n = qbr::sort_count(num_pairs, 0, cap);
    uint32_t target = (uint32_t)(t + half);
    int64_t lo = 0, hi = n;
    for (;;) {
        bool wide = hi - lo > 32;
        if (!__any(wide)) break;
        bool below = false;
        if (wide) below = (uint32_t)tiles[lo + ((hi - lo) * (k + 1)) / 33] < target;
        int c = __popc((uint32_t)(__ballot(below) >> (32 * half)));
        if (wide) {
            int64_t span = hi - lo;
            int64_t nlo = c == 0 ? lo : lo + (span * c) / 33 + 1;
            int64_t nhi = c == 32 ? hi : lo + (span * (c + 1)) / 33;
            lo = nlo;
            hi = nhi;
        }
    }
    bool below = lo + k < hi && (uint32_t)tiles[lo + k] < target;
    uint32_t bound = (uint32_t)(lo + __popc((uint32_t)(__ballot(below) >> (32 * half))));
    uint32_t upper = __shfl(bound, 32);
    if (lane == 0) reinterpret_cast<uint2*>(ranges)[t] = make_uint2(bound, upper);
}

__global__ __launch_bounds__(QB_BLOCK) void k_make_keys(const uint16_t* __restrict__ tiles,
                                                        const uint32_t* __restrict__ ids,
                                                        const float4* __restrict__ splats,
                                                        const int64_t* __restrict__ num_pairs, int64_t cap,
                                                        uint64_t* __restrict__ keys)
{
    int64_t n = qbr::sort_count(num_pairs, 0, cap);
    for (int64_t i = (int64_t)blockIdx.x * QB_BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * QB_BLOCK) {
        uint32_t id = ids[i];
        keys[i] = ((uint64_t)tiles[i] << 32) | __float_as_uint(splats[3 * (int64_t)id].z);
    }
}

// Packed pairs of a one-tile image: the ids in emission order, tile 0.
__global__ __launch_bounds__(QB_BLOCK) void k_one_tile(const uint32_t* __restrict__ packed,
                                                       const int64_t* __restrict__ num_pairs, int64_t cap,
                                                       uint16_t* __restrict__ tiles, uint32_t* __restrict__ ids)
{
    int64_t n = qbr::sort_count(num_pairs, 0, cap);
    for (int64_t i = (int64_t)blockIdx.x * QB_BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * QB_BLOCK) {
        tiles[i] = 0;
        ids[i] = packed[i];
    }
}

int tile_bits(int64_t num_tiles)
{
    int b = 0;
    while ((1ll << b) < num_tiles) ++b;
    return b;
}

struct SortWs {
    uint16_t* tiles_sorted;
    uint16_t* ktmp;
    uint32_t* vtmp;
    uint32_t* radix;
};

SortWs carve(QbArena& a, int64_t cap)
{
    SortWs w;
    w.tiles_sorted = a.take<uint16_t>(cap);
    w.ktmp = a.take<uint16_t>(cap);
    w.vtmp = a.take<uint32_t>(cap);
    w.radix = a.take<uint32_t>((int64_t)(qbr::radix_scratch_bytes<kSortMinTile, 1>(cap) / sizeof(uint32_t)));
    return w;
}

}  // namespace

extern "C" size_t qb_sort_workspace_size(int64_t pair_capacity)
{
    if (pair_capacity < 0) return 0;
    QbArena a{nullptr, 0, 0};
    carve(a, pair_capacity);
    return a.used + 256;
}

// The tile sort in radix workgroups of NT lanes x NI pairs, the first pass
// taking first_bits of the tile bits (0: an even split).
template <int NT, int NI>
static qb_status tile_sort(const uint16_t* pair_tiles, const uint32_t* pair_ids, uint16_t* tiles_sorted,
                           uint32_t* ids, uint16_t* ktmp, uint32_t* vtmp, const int64_t* num_pairs,
                           int64_t cap, int bits, uint32_t* radix, int first_bits, hipStream_t s)
{
    static_assert(NT * NI >= kSortMinTile, "the workspace is sized for tiles of at least kSortMinTile pairs");
    return qbr::radix_sort<uint16_t, NT, NI>(pair_tiles, pair_ids, tiles_sorted, ids, ktmp, vtmp, num_pairs, 0,
                                             cap, 0, bits, radix, s, nullptr, nullptr, first_bits);
}

// Digit width of the first pass for a variant: the even split of the two
// passes (ceil(bits / 2)) for the shape variants, 2 bits narrower or wider
// for the digit-width variants, kept within 1..8 with at most 8 bits left.
static int first_pass_bits(int variant, int bits)
{
    int even = (bits + 1) / 2;
    int want = variant == QB_SORT_512x8_NARROW_FIRST ? even - 2 : variant == QB_SORT_512x8_WIDE_FIRST ? even + 2 : even;
    if (bits <= 8) return 0;   // one pass: no split
    return max(max(1, bits - 8), min(8, want));
}

extern "C" qb_status qb_sort(int64_t pair_capacity, const int64_t* num_pairs, int32_t num_tiles,
                             const uint16_t* pair_tiles, const uint32_t* pair_ids, const qb_splat* splats,
                             uint64_t* keys, uint32_t* ids, uint32_t* ranges, void* workspace,
                             size_t workspace_bytes, qb_stream_t stream)
{
    return qb_sort_ex(pair_capacity, num_pairs, num_tiles, pair_tiles, pair_ids, splats, keys, ids, ranges,
                      workspace, workspace_bytes, QB_SORT_512x8, 0, stream);
}

// The tile sort of packed pairs (tile << id_bits | id) in radix workgroups of
// NT lanes x NI pairs: the passes move the 4-byte packed pairs alone, the
// last one writes the sorted tiles and ids apart.
template <int NT, int NI>
static qb_status packed_sort(const uint32_t* packed, uint16_t* tiles_sorted, uint32_t* ids, uint32_t* tmp,
                             const int64_t* num_pairs, int64_t cap, int id_bits, int bits, uint32_t* radix,
                             int first_bits, hipStream_t s)
{
    static_assert(NT * NI >= kSortMinTile, "the workspace is sized for tiles of at least kSortMinTile pairs");
    return qbr::radix_sort_packed<NT, NI>(packed, tmp, tiles_sorted, ids, num_pairs, cap, id_bits, id_bits + bits,
                                          radix, s, first_bits);
}

extern "C" qb_status qb_sort_ex(int64_t pair_capacity, const int64_t* num_pairs, int32_t num_tiles,
                                const uint16_t* pair_tiles, const uint32_t* pair_ids, const qb_splat* splats,
                                uint64_t* keys, uint32_t* ids, uint32_t* ranges, void* workspace,
                                size_t workspace_bytes, int32_t variant, int32_t packed_id_bits,
                                qb_stream_t stream)
{
    if (pair_capacity < 0 || pair_capacity > (int64_t)0xFFFFFFFF || !num_pairs || num_tiles < 1 ||
        num_tiles > 65536 || !ranges || !workspace || variant < 0 || variant >= QB_SORT_VARIANTS)
        return QB_ERR_INVALID_ARG;
    if (packed_id_bits != 0 &&
        (packed_id_bits < 1 || packed_id_bits > 31 || packed_id_bits + tile_bits(num_tiles) > 32))
        return QB_ERR_INVALID_ARG;
    if (pair_capacity > 0 && ((!packed_id_bits && !pair_tiles) || !pair_ids || !ids)) return QB_ERR_INVALID_ARG;
    if (keys && !splats) return QB_ERR_INVALID_ARG;
    if ((const void*)pair_ids == (const void*)ids) return QB_ERR_INVALID_ARG;
    if (workspace_bytes < qb_sort_workspace_size(pair_capacity)) return QB_ERR_INVALID_ARG;
    hipStream_t s = qb_hip_stream(stream);
    QbArena a{(char*)(((uintptr_t)workspace + 255) & ~(uintptr_t)255), workspace_bytes - 256, 0};
    SortWs w = carve(a, pair_capacity);
    if (!a.ok()) return QB_ERR_INVALID_ARG;
    if (pair_capacity > 0) {
        int bits = tile_bits(num_tiles);
#define QB_TILE_SORT(NT, NI)                                                                                   \
    tile_sort<NT, NI>(pair_tiles, pair_ids, w.tiles_sorted, ids, w.ktmp, w.vtmp, num_pairs, pair_capacity, bits, \
                      w.radix, first_pass_bits(variant, bits), s)
#define QB_PACKED_SORT(NT, NI)                                                                                 \
    packed_sort<NT, NI>(pair_ids, w.tiles_sorted, ids, w.vtmp, num_pairs, pair_capacity, packed_id_bits, bits,    \
                        w.radix, first_pass_bits(variant, bits), s)
        if (packed_id_bits && bits > 0) {
            switch (variant) {
            case QB_SORT_1024x8: QB_CHECK(QB_PACKED_SORT(1024, 8)); break;
            case QB_SORT_512x16: QB_CHECK(QB_PACKED_SORT(512, 16)); break;
            case QB_SORT_256x16: QB_CHECK(QB_PACKED_SORT(256, 16)); break;
            default: QB_CHECK(QB_PACKED_SORT(512, 8)); break;
            }
        } else if (packed_id_bits) {
            // one tile: the packed pairs are the ids, already in order
            int64_t g = qb_div_up(pair_capacity, QB_BLOCK);
            if (g > 8192) g = 8192;
            QB_LAUNCH(k_one_tile, g, QB_BLOCK, 0, s, pair_ids, num_pairs, pair_capacity, w.tiles_sorted, ids);
        } else {
            switch (variant) {
            case QB_SORT_1024x8: QB_CHECK(QB_TILE_SORT(1024, 8)); break;
            case QB_SORT_512x16: QB_CHECK(QB_TILE_SORT(512, 16)); break;
            case QB_SORT_256x16: QB_CHECK(QB_TILE_SORT(256, 16)); break;
            default: QB_CHECK(QB_TILE_SORT(512, 8)); break;   // 512x8 and its digit-width variants
            }
        }
#undef QB_PACKED_SORT
#undef QB_TILE_SORT
        if (keys) {
            int64_t g = qb_div_up(pair_capacity, QB_BLOCK);
            if (g > 8192) g = 8192;
            QB_LAUNCH(k_make_keys, g, QB_BLOCK, 0, s, (const uint16_t*)w.tiles_sorted, (const uint32_t*)ids,
                      reinterpret_cast<const float4*>(splats), num_pairs, pair_capacity, keys);
        }
    }
    QB_LAUNCH(k_ranges, qb_div_up(num_tiles, QB_BLOCK / 64), QB_BLOCK, 0, s, (const uint16_t*)w.tiles_sorted, num_pairs,
              pair_capacity, (int)num_tiles, ranges);
    return QB_OK;
}
