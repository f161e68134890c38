// qb_intersect: DuplicateWithKeys with the QPass traversal (Sec. 2, Sec. 3.2).
//
//  1. key every Gaussian by its depth bits (0xFFFFFFFF when it covers no
//     tile; qb_project_ex writes these keys, else they are derived here from
//     the splats and counts) and stable-radix-sort the ids: the (depth, id)
//     order that orders the Gaussians within every tile (those that cover no
//     tile emit nothing and may fall anywhere in it)
//  2. gather the tile counts in that order (in the sort's last pass) and
//     scan them: the pair offsets and the total
//  3. emit: a 256-lane workgroup takes 256 consecutive Gaussians of that
//     order and runs QPass for each (one lane per Gaussian); the non-empty
//     runs (blocks of scanlines with one tile interval) go to a run list in
//     LDS with the block-relative index of their first pair.  The workgroup
//     then walks its pairs pair-parallel, 64 consecutive pairs per wave per
//     step.  The run of each pair comes from a per-step owner table (every run
//     that starts inside the step marks its first pair; a ballot and a prefix
//     bit count give each pair the number of runs started up to it), its tile
//     from a reciprocal multiply and two 24-bit multiply-adds on the pair's
//     offset in the run; the stores of a wave are contiguous.
// A pair is stored compactly as (uint16 tile, uint32 Gaussian id); its key
// tile << 32 | bits(depth) is implied by the id.
// The naive traversal (QB_BOX_QUADBOX_NAIVE, the ablation without QPass)
// replaces step 3 by one lane per Gaussian that walks its sub-box rects with
// nested loops and writes its pairs one by one, as DuplicateWithKeys does.
#include <mutex>

#include "qb_bin.h"

namespace {

// Depth-sort workgroup shapes (lanes x keys per lane) and emission workgroup
// sizes, indexed by qb_depth_variant / qb_emit_variant; the first of each is
// qb_intersect's (512 x 4: 2048 keys per workgroup, about 500 workgroups at
// 10^6 Gaussians; 256-lane emission).  The workspace covers the depth-sort
// shape with the most workgroups.
constexpr int kDepthMinTile = 2048;

__global__ __launch_bounds__(QB_BLOCK) void k_depth_keys(int64_t n, const float4* __restrict__ splats,
                                                         const int32_t* __restrict__ counts,
                                                         uint32_t* __restrict__ keys)
{
    int64_t i = (int64_t)blockIdx.x * QB_BLOCK + threadIdx.x;
    if (i >= n) return;
    float d = splats[3 * i].z;
    keys[i] = counts[i] > 0 ? __float_as_uint(d) : 0xFFFFFFFFu;
}

__global__ void k_store_total(const uint64_t* __restrict__ tot, int64_t* __restrict__ num_pairs)
{
    *num_pairs = tot ? (int64_t)*tot : 0;
}

// Stores pair dst: split (uint16 tile, uint32 id), or, with id_bits > 0,
// packed as tile << id_bits | id into out_id alone.
__device__ __forceinline__ void store_pair(int64_t dst, uint32_t tile, uint32_t id, int id_bits,
                                           uint16_t* __restrict__ out_tile, uint32_t* __restrict__ out_id)
{
    if (id_bits) {
        out_id[dst] = (tile << id_bits) | id;
    } else {
        out_tile[dst] = (uint16_t)tile;
        out_id[dst] = id;
    }
}

// kChains: independent cursors per wave.  The block's pairs are cut into
// (waves x kChains) contiguous ranges; a wave advances its kChains ranges in
// lockstep, 64 pairs each per step, so the LDS round trips of one range's
// step (owner table, run lookups) overlap with the other's.
//
// A run of n scanlines x len tiles holds its pairs scanline-major, so pair
// `local` of the run is on scanline q = local / len at offset local - q * len.
// Its tile is affine in (local, q): tbase + local * A + q * B, with
//   rows    (axis 1): tbase = s0 * tiles_x + lo, A = 1,       B = tiles_x - len
//   columns (axis 0): tbase = lo * tiles_x + s0, A = tiles_x, B = 1 - len * tiles_x
// (|A|, |B| < 2^17 and local, q < 2^16 with at most 65536 tiles, so 24-bit
// multiplies suffice).  q comes from the run's reciprocal r ~ 1/len (1 ulp):
// (local + 1/2) r is (local + 1/2) / len within a relative 2^-22, i.e. within
// 0.02 / len for local < 2^16, and the exact quotient sits at least 1/(2 len)
// from an integer, so truncation gives the exact q.
template <int kEmitThreads, int kChains>
__global__ __launch_bounds__(kEmitThreads) void k_emit(
    int64_t n, const uint32_t* __restrict__ order, const uint64_t* __restrict__ goff,
    const int4* __restrict__ rects, const uint32_t* __restrict__ sorted_counts, int tiles_x, int64_t cap,
    const int64_t* __restrict__ num_pairs, uint16_t* __restrict__ out_tile, uint32_t* __restrict__ out_id,
    int id_bits)
{
    // the run list holds kRunsPerLane runs per Gaussian on average (QuadBox
    // Gaussians have at most 5 runs, 2.3-3.4 on average, and no 128-Gaussian
    // block of the clustered, anisotropic or random test scenes averages
    // above 3.7); a block with more runs walks its two halves one after the
    // other (at most QB_MAX_SEG <= 2 * kRunsPerLane runs per Gaussian each).
    // The smaller list doubles the blocks that LDS lets a CU hold.
    constexpr int kRunsPerLane = 4;
    static_assert(QB_MAX_SEG <= 2 * kRunsPerLane, "a half block's runs fit the list");
    constexpr int kRuns = kEmitThreads * kRunsPerLane;
    constexpr int NW = kEmitThreads / 64;
    __shared__ uint32_t s_off[kRuns + 1];  // first pair of each run, relative to the walk's first pair
    __shared__ uint4 s_run[kRuns];         // Gaussian id, bits(r), tbase | A << 16, B
    __shared__ uint32_t s_scan[NW];
    __shared__ uint32_t s_tab[NW][kChains][64];

    if (*num_pairs > cap) return;  // overflow: the caller re-runs with more capacity
    int t = threadIdx.x;
    uint32_t lane = (uint32_t)t & 63u;
    int wave = __builtin_amdgcn_readfirstlane(t >> 6);
    int64_t k0 = (int64_t)blockIdx.x * kEmitThreads;
    int64_t k = k0 + t;
    uint32_t gi = 0;
    QRuns q;
#pragma unroll
    for (int i = 0; i < QB_MAX_SEG; ++i) q.n[i] = 0;
    q.total = 0;
    q.axis = 0;
    if (k < n) {
        gi = order[k];
        if (sorted_counts[k] > 0) qbb::gaussian_runs(rects, gi, q);
    }
    uint32_t cnt = (uint32_t)q.total;
    uint32_t nr = 0;
#pragma unroll
    for (int i = 0; i < QB_MAX_SEG; ++i) nr += (q.n[i] > 0 && q.len[i] > 0) ? 1u : 0u;
    uint32_t total, nruns;
    uint32_t off = qbr::block_exclusive_scan<uint32_t, kEmitThreads>(cnt, &total, s_scan);
    uint32_t slot = qbr::block_exclusive_scan<uint32_t, kEmitThreads>(nr, &nruns, s_scan);
    total = __builtin_amdgcn_readfirstlane(total);
    nruns = __builtin_amdgcn_readfirstlane(nruns);
    int64_t block_start = (int64_t)goff[k0];
    // One walk: the runs of the lanes that take part (mine) go to the run
    // list at their slots, and the walk's `total` pairs are written from
    // pair `start` on.  Ends with a barrier, so that a second walk may reuse
    // the list.
    auto walk = [&](bool mine, uint32_t off, uint32_t slot, uint32_t total, uint32_t nruns, int64_t start) {
#pragma unroll
        for (int i = 0; i < QB_MAX_SEG; ++i) {
            uint32_t len = (uint32_t)q.len[i];
            uint32_t sz = (uint32_t)q.n[i] * len;
            if (mine && sz > 0) {
                uint32_t tb, a;
                int32_t b;
                if (q.axis) {
                    tb = (uint32_t)(q.s0[i] * tiles_x + q.lo[i]);
                    a = 1;
                    b = tiles_x - (int)len;
                } else {
                    tb = (uint32_t)(q.lo[i] * tiles_x + q.s0[i]);
                    a = (uint32_t)tiles_x;
                    b = 1 - (int)len * tiles_x;
                }
                s_off[slot] = off;
                s_run[slot] = make_uint4(gi, __float_as_uint(__builtin_amdgcn_rcpf((float)len)), tb | a << 16,
                                         (uint32_t)b);
                ++slot;
                off += sz;
            }
        }
        if (t == 0) s_off[nruns] = total;  // sentinel
#pragma unroll
        for (int c = 0; c < kChains; ++c) s_tab[wave][c][lane] = 0xFFFFFFFFu;
        // the pairs of the walk fill [start, start + total) <= num_pairs <= cap;
        // the bound below only keeps a stale offset table inside the buffer
        if (start + (int64_t)total > cap) total = cap > start ? (uint32_t)(cap - start) : 0u;
        __syncthreads();
        // each of the block's waves x kChains ranges is a contiguous share of its
        // pairs, walked 64 per step; the run holding a step's first pair is the
        // run of the previous step's last pair, so only a range's first step
        // searches for it
        uint32_t per = (total + NW * kChains - 1) / (NW * kChains);
        uint32_t base[kChains], hi[kChains];
        int cur[kChains];
#pragma unroll
        for (int c = 0; c < kChains; ++c) {
            uint32_t lo = min(total, (uint32_t)(wave * kChains + c) * per);
            base[c] = lo;
            hi[c] = min(total, lo + per);
            int a = 0, b = (int)nruns;
            while (b - a > 1) {
                int mid = (a + b) >> 1;
                if (__builtin_amdgcn_readfirstlane(s_off[mid]) <= lo) a = mid; else b = mid;
            }
            cur[c] = a;
        }
        for (;;) {
            bool left = false;
#pragma unroll
            for (int c = 0; c < kChains; ++c) left = left || base[c] < hi[c];
            if (!left) break;
            // every later run that starts inside a range's step writes its start
            // into the owner table slot of its first pair.  Starts only grow, so a
            // slot holds the current step's pair exactly when that pair starts a
            // run; the run of a pair is cur + the run starts at or before it.
#pragma unroll
            for (int c = 0; c < kChains; ++c) {
                uint32_t jj = (uint32_t)cur[c] + 1u + lane;
                if (base[c] < hi[c] && jj < nruns) {
                    uint32_t d = s_off[jj] - base[c];
                    if (d < 64u) s_tab[wave][c][d] = base[c] + d;
                }
            }
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int c = 0; c < kChains; ++c) {
                if (base[c] < hi[c]) {
                    uint32_t p = base[c] + lane;
                    uint64_t m = __builtin_amdgcn_ballot_w64(s_tab[wave][c][lane] == p);
                    uint32_t c0 = (uint32_t)cur[c] + (uint32_t)(m & 1u);
                    m >>= 1;
                    uint32_t o = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, c0));
                    if (p < hi[c]) {
                        uint32_t local = p - s_off[o];
                        uint4 rr = s_run[o];
                        float r = __uint_as_float(rr.y);
                        uint32_t qq = (uint32_t)__builtin_fmaf((float)local, r, 0.5f * r);
                        uint32_t tile = (rr.z & 0xFFFFu) + __umul24(local, rr.z >> 16) + (uint32_t)__mul24((int)qq, (int)rr.w);
                        int64_t wbase = start + base[c];
                        if (id_bits) {
                            out_id[wbase + lane] = (tile << id_bits) | rr.x;
                        } else {
                            out_tile[wbase + lane] = (uint16_t)tile;
                            out_id[wbase + lane] = rr.x;
                        }
                    }
                    cur[c] = __builtin_amdgcn_readlane((int)o, 63);
                    base[c] += 64;
                }
            }
            __builtin_amdgcn_wave_barrier();
        }
        __syncthreads();
    };
    if (nruns <= (uint32_t)kRuns) {
        walk(true, off, slot, total, nruns, block_start);
    } else {
        // two walks: the first half of the lanes' Gaussians, then the second
        int64_t start = block_start;
        for (int part = 0; part < 2; ++part) {
            bool mine = (t >= part * (kEmitThreads / 2)) && (t < (part + 1) * (kEmitThreads / 2));
            uint32_t pt, pr;
            uint32_t po = qbr::block_exclusive_scan<uint32_t, kEmitThreads>(mine ? cnt : 0u, &pt, s_scan);
            uint32_t ps = qbr::block_exclusive_scan<uint32_t, kEmitThreads>(mine ? nr : 0u, &pr, s_scan);
            pt = __builtin_amdgcn_readfirstlane(pt);
            pr = __builtin_amdgcn_readfirstlane(pr);
            walk(mine, po, ps, pt, pr, start);
            start += pt;
        }
    }
}

__global__ __launch_bounds__(QB_BLOCK) void k_emit_naive(
    int64_t n, const uint32_t* __restrict__ order, const uint64_t* __restrict__ goff,
    const int4* __restrict__ rects, const uint32_t* __restrict__ sorted_counts, int tiles_x, int64_t cap,
    const int64_t* __restrict__ num_pairs, uint16_t* __restrict__ out_tile, uint32_t* __restrict__ out_id,
    int id_bits)
{
    if (*num_pairs > cap) return;  // overflow: the caller re-runs with more capacity
    int64_t k = (int64_t)blockIdx.x * QB_BLOCK + threadIdx.x;
    if (k >= n) return;
    uint32_t gi = order[k];
    if (sorted_counts[k] == 0) return;
    int4 p0 = rects[2 * (int64_t)gi], p1 = rects[2 * (int64_t)gi + 1];
    QRect r[4] = {qbb::unpack_rect(p0.x, p0.y), qbb::unpack_rect(p0.z, p0.w), qbb::unpack_rect(p1.x, p1.y),
                  qbb::unpack_rect(p1.z, p1.w)};
    int64_t base = (int64_t)goff[k];
    naive_walk(r, [&](int tx, int ty, int c) {
        int64_t dst = base + c;
        if (dst < cap) store_pair(dst, (uint32_t)(ty * tiles_x + tx), gi, id_bits, out_tile, out_id);
    });
}

struct IsectWs {
    uint32_t *dk0, *dv0, *dk1, *dv1;  // depth sort ping-pong; dv0 ends as the order
    uint32_t* csorted;                // counts in that order
    uint64_t* offs;                   // pair offsets
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
    w.scan64 = a.take<uint64_t>(qbr::scan_scratch(n));
    w.radix = a.take<uint32_t>((int64_t)(qbr::radix_scratch_bytes<kDepthMinTile, 1>(n) / sizeof(uint32_t)));
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

// The depth sort of (keys, ids) in radix workgroups of NT lanes x NI keys;
// the last pass also gathers the tile counts into the sorted order, which
// ends in w.dv0.  keys: the depth keys (qb_project_ex's, or w.dk0 after
// k_depth_keys wrote them there); the ids are the positions.  With at most
// kFusedBlocks workgroups the passes cover only the span of the keys of the
// Gaussians that cover a tile (the others, 0xFFFFFFFF, emit nothing, so
// their place in the order is free): the positive binary32 depths of one
// view seldom span more than 2^24 key values, and the fourth pass then
// returns at once.  The pair offsets' array, written after the sort, holds
// values between passes.
template <int NT, int NI>
static qb_status depth_sort(IsectWs& w, const uint32_t* keys, int64_t n, const int32_t* counts, hipStream_t s)
{
    static_assert(NT * NI >= kDepthMinTile, "the workspace is sized for tiles of at least kDepthMinTile keys");
    if (qb_div_up(n, NT * NI) <= qbr::kFusedBlocks)
        return qbr::radix_sort_span<NT, NI>(keys, w.dk1, w.dv1, w.dk0, reinterpret_cast<uint32_t*>(w.offs), w.dv0,
                                            n, w.radix, s, counts, w.csorted);
    // four 8-bit passes over the whole key: keys -> (dk1, dv1) -> (dk0, dv0) -> ...
    return qbr::radix_sort<uint32_t, NT, NI>(keys, nullptr, w.dk0, w.dv0, w.dk1, w.dv1, (const int64_t*)nullptr, n,
                                             n, 0, 32, w.radix, s, counts, w.csorted);
}

template <int NT, int C>
static qb_status launch_emit(int64_t n, const uint32_t* order, const uint64_t* offs, const int4* r4,
                             const uint32_t* csorted, int tiles_x, int64_t cap, const int64_t* num_pairs,
                             uint16_t* pair_tiles, uint32_t* pair_ids, int id_bits, hipStream_t s)
{
    QB_LAUNCH((k_emit<NT, C>), qb_div_up(n, NT), NT, 0, s, n, order, offs, r4, csorted, tiles_x, cap, num_pairs,
              pair_tiles, pair_ids, id_bits);
    return QB_OK;
}

// The stages of qb_intersect over a workspace of `workspace_bytes` bytes at
// `workspace` (already checked to be large enough for n).
static qb_status intersect_impl(int64_t n, const qb_splat* splats, const qb_rects* rects, const int32_t* counts,
                                int tiles_x, int32_t mode, int64_t pair_capacity, uint16_t* pair_tiles,
                                uint32_t* pair_ids, int64_t* num_pairs, void* workspace, size_t workspace_bytes,
                                const uint32_t* depth_keys, int32_t depth_variant, int32_t emit_variant,
                                int id_bits, hipStream_t s)
{
    QbArena a{(char*)(((uintptr_t)workspace + 255) & ~(uintptr_t)255), workspace_bytes - 256, 0};
    IsectWs w = carve(a, n);
    if (!a.ok()) return QB_ERR_INVALID_ARG;
    if (n == 0) {
        QB_LAUNCH(k_store_total, 1, 1, 0, s, (const uint64_t*)nullptr, num_pairs);  // no pairs
        return QB_OK;
    }
    int64_t grid = qb_div_up(n, QB_BLOCK);
    const uint32_t* keys = depth_keys;
    if (!keys) {
        QB_LAUNCH(k_depth_keys, grid, QB_BLOCK, 0, s, n, reinterpret_cast<const float4*>(splats), counts, w.dk0);
        keys = w.dk0;
    }
    switch (depth_variant) {
    case QB_DEPTH_512x4: QB_CHECK((depth_sort<512, 4>(w, keys, n, counts, s))); break;
    case QB_DEPTH_256x8: QB_CHECK((depth_sort<256, 8>(w, keys, n, counts, s))); break;
    case QB_DEPTH_512x8: QB_CHECK((depth_sort<512, 8>(w, keys, n, counts, s))); break;
    default: QB_CHECK((depth_sort<1024, 4>(w, keys, n, counts, s))); break;
    }
    // pair offsets; the total (a count, below 2^63) lands in *num_pairs
    QB_CHECK((qbr::exclusive_scan<uint32_t, uint64_t>(w.csorted, w.offs, n, w.scan64,
                                                      reinterpret_cast<uint64_t*>(num_pairs), s)));
    const uint32_t* order = w.dv0;
    const int4* r4 = reinterpret_cast<const int4*>(rects);
    if (pair_capacity > 0 && (mode & ~QB_CLIP_3SIGMA) == QB_BOX_QUADBOX_NAIVE)
        QB_LAUNCH(k_emit_naive, grid, QB_BLOCK, 0, s, n, order, (const uint64_t*)w.offs, r4,
                  (const uint32_t*)w.csorted, tiles_x, pair_capacity, (const int64_t*)num_pairs, pair_tiles, pair_ids,
                  id_bits);
    else if (pair_capacity > 0) {
        const uint64_t* offs = w.offs;
        const uint32_t* cs = w.csorted;
#define QB_EMIT(NT, C) \
    QB_CHECK((launch_emit<NT, C>(n, order, offs, r4, cs, tiles_x, pair_capacity, num_pairs, pair_tiles, pair_ids, \
                                 id_bits, s)))
        switch (emit_variant) {
        case QB_EMIT_128: QB_EMIT(128, 1); break;
        case QB_EMIT_512: QB_EMIT(512, 1); break;
        case QB_EMIT_256_2CHAINS: QB_EMIT(256, 2); break;
        case QB_EMIT_128_2CHAINS: QB_EMIT(128, 2); break;
        default: QB_EMIT(256, 1); break;
        }
#undef QB_EMIT
    }
    return QB_OK;
}

// Host-side argument checks shared by qb_intersect and qb_intersect_noalloc;
// sets the tile-row width on success.
static qb_status intersect_args(int64_t n, const qb_splat* splats, const qb_rects* rects, const int32_t* counts,
                                int32_t width, int32_t height, int32_t mode, int64_t pair_capacity,
                                const uint16_t* pair_tiles, const uint32_t* pair_ids, const int64_t* num_pairs,
                                int* tiles_x_out)
{
    if (n < 0 || n >= (int64_t)1 << 31 || width <= 0 || height <= 0 || !qb_valid_mode(mode) || pair_capacity < 0 ||
        pair_capacity > (int64_t)0xFFFFFFFF || !num_pairs)
        return QB_ERR_INVALID_ARG;
    int tiles_x = (int)qb_div_up(width, QB_TILE);
    int64_t tiles = (int64_t)tiles_x * qb_div_up(height, QB_TILE);
    if (tiles > 65536) return QB_ERR_UNSUPPORTED;
    if (n > 0 && (!splats || !rects || !counts)) return QB_ERR_INVALID_ARG;
    if (pair_capacity > 0 && (!pair_tiles || !pair_ids)) return QB_ERR_INVALID_ARG;
    *tiles_x_out = tiles_x;
    return QB_OK;
}

// Bits of the tile id for num_tiles tiles.
static int tile_id_bits(int64_t num_tiles)
{
    int b = 0;
    while ((1ll << b) < num_tiles) ++b;
    return b;
}

extern "C" int32_t qb_pair_id_bits(int64_t n, int32_t width, int32_t height)
{
    if (n < 0 || width <= 0 || height <= 0) return 0;
    int64_t tiles = qb_div_up(width, QB_TILE) * qb_div_up(height, QB_TILE);
    if (tiles > 65536) return 0;
    int b = tile_id_bits(n > 1 ? n : 2);
    return b + tile_id_bits(tiles) <= 32 ? b : 0;
}

extern "C" qb_status qb_intersect(int64_t n, const qb_splat* splats, const qb_rects* rects,
                                  const int32_t* counts, int32_t width, int32_t height, int32_t mode,
                                  int64_t pair_capacity,
                                  uint16_t* pair_tiles, uint32_t* pair_ids, int64_t* num_pairs, void* workspace,
                                  size_t workspace_bytes, qb_stream_t stream)
{
    return qb_intersect_ex(n, splats, rects, counts, width, height, mode, pair_capacity, pair_tiles, pair_ids,
                           num_pairs, workspace, workspace_bytes, nullptr, QB_DEPTH_512x4, QB_EMIT_256, 0, stream);
}

extern "C" qb_status qb_intersect_ex(int64_t n, const qb_splat* splats, const qb_rects* rects,
                                     const int32_t* counts, int32_t width, int32_t height, int32_t mode,
                                     int64_t pair_capacity, uint16_t* pair_tiles, uint32_t* pair_ids,
                                     int64_t* num_pairs, void* workspace, size_t workspace_bytes,
                                     const uint32_t* depth_keys, int32_t depth_variant, int32_t emit_variant,
                                     int32_t packed_id_bits, qb_stream_t stream)
{
    int tiles_x = 0;
    // packed pairs live in pair_ids alone: pair_tiles may be NULL
    uint16_t* tiles_arg = packed_id_bits ? reinterpret_cast<uint16_t*>(pair_ids) : pair_tiles;
    QB_CHECK(intersect_args(n, splats, rects, counts, width, height, mode, pair_capacity, tiles_arg, pair_ids,
                            num_pairs, &tiles_x));
    if (depth_variant < 0 || depth_variant >= QB_DEPTH_VARIANTS || emit_variant < 0 ||
        emit_variant >= QB_EMIT_VARIANTS)
        return QB_ERR_INVALID_ARG;
    if (packed_id_bits != 0) {
        int64_t tiles = (int64_t)tiles_x * qb_div_up(height, QB_TILE);
        if (packed_id_bits < 1 || packed_id_bits > 31 || n > ((int64_t)1 << packed_id_bits) ||
            packed_id_bits + tile_id_bits(tiles) > 32)
            return QB_ERR_INVALID_ARG;
    }
    if (!workspace || workspace_bytes < qb_intersect_workspace_size(n)) return QB_ERR_INVALID_ARG;
    return intersect_impl(n, splats, rects, counts, tiles_x, mode, pair_capacity, pair_tiles, pair_ids, num_pairs,
                          workspace, workspace_bytes, depth_keys, depth_variant, emit_variant, packed_id_bits,
                          qb_hip_stream(stream));
}

// ---- qb_intersect without a caller workspace --------------------------------
// The workspace of qb_intersect_noalloc: a static device array, one copy per
// GPU the library runs on, held until the process ends.  Host code never
// passes `scratch` itself to a kernel (on the host the name stands for a
// host-side shadow, not a device address): the first call on a device looks
// up that device's address with hipGetSymbolAddress, with the device
// current, and every later call on the device uses that address.
namespace {
constexpr size_t kNoallocScratchBytes = (size_t)60 << 20;
__device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices];   // device address of `scratch` on each device, once looked up

// Address of `scratch` on the current device, or nullptr on failure.
void* scratch_on_current_device()
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return nullptr;
        g_scratch_dev[dev] = ptr;
    }
    return g_scratch_dev[dev];
}
}  // namespace

extern "C" qb_status qb_intersect_noalloc(int64_t n, const qb_splat* splats, const qb_rects* rects,
                                          const int32_t* counts, int32_t width, int32_t height, int32_t mode,
                                          int64_t pair_capacity, uint16_t* pair_tiles, uint32_t* pair_ids,
                                          int64_t* num_pairs, qb_stream_t stream)
{
    int tiles_x = 0;
    QB_CHECK(intersect_args(n, splats, rects, counts, width, height, mode, pair_capacity, pair_tiles, pair_ids,
                            num_pairs, &tiles_x));
    if (n > QB_NOALLOC_MAX_GAUSSIANS) return QB_ERR_INVALID_ARG;
    // the static array holds the workspace of the largest n accepted
    if (qb_intersect_workspace_size(QB_NOALLOC_MAX_GAUSSIANS) > kNoallocScratchBytes) return QB_ERR_UNSUPPORTED;
    void* ws = scratch_on_current_device();
    if (!ws) return QB_ERR_HIP;
    return intersect_impl(n, splats, rects, counts, tiles_x, mode, pair_capacity, pair_tiles, pair_ids, num_pairs,
                          ws, kNoallocScratchBytes, nullptr, QB_DEPTH_512x4, QB_EMIT_256, 0, qb_hip_stream(stream));
}
