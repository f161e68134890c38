// Device-wide exclusive scan and a stable LSD radix sort for wave64 (gfx950).
//
// Both are reduce-then-scan: no workgroup ever waits on another, so there is
// no inter-workgroup spin and no forward-progress assumption.
//   scan:  up to 32768 items in one 1024-lane workgroup; beyond that a
//          per-block reduction, then the per-block scan, whose workgroups
//          add up the raw totals of the blocks before them (up to 1024
//          blocks; beyond that the totals are scanned recursively first)
//   radix pass (<= 8 bits):
//     upsweep   per-block digit histogram in LDS, stored digit-major
//     scan      exclusive scan of the digit-major histogram (global offsets);
//               with at most kFusedBlocks blocks there is no scan launch: the
//               histograms are stored block-major and every downsweep
//               workgroup sums the rows itself (16-byte loads, all in flight)
//     downsweep per-block stable ranks: each wave owns a contiguous run of the
//               block's items and ranks 64 at a time by matching digits with
//               one ballot per digit bit; per-wave digit counts are combined
//               across waves in LDS; items are reordered by digit in LDS and
//               then written out as contiguous runs (coalesced stores).
#pragma once

#include <climits>
#include <type_traits>

#include "qb_common.h"

namespace qbr {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;  // 2048 items per block
constexpr int kBigScanThreads = 1024;
constexpr int kBigScanItems = 32;
constexpr int kBigScanTile = kBigScanThreads * kBigScanItems;  // 32768 items, one workgroup

constexpr int kRadixBits = 8;
constexpr int kRadix = 1 << kRadixBits;
constexpr int kFusedBlocks = 512;

// DPP lane shift within the wave (update_dpp with `identity` where the
// source lane falls outside the row or the row is masked off).  Controls:
// 0x111/0x112/0x114/0x118 = row_shr 1/2/4/8 (rows of 16 lanes), 0x142 =
// row_bcast 15 (lane 15 of each row to the next row; rows 1 and 3 written),
// 0x143 = row_bcast 31 (lane 31 to rows 2 and 3).  Every lane of the wave
// must be active.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ int dpp_shift(int v, int identity)
{
    return __builtin_amdgcn_update_dpp(identity, v, CTRL, ROW_MASK, 0xF, false);
}

// Inclusive scan across one wave64.  32-bit integers: Hillis-Steele within
// rows of 16 by DPP row shifts, then the row broadcasts (six full-rate VALU
// adds).  64-bit: over lane shuffles.
template <typename T>
__device__ __forceinline__ T wave_inclusive_scan(T v)
{
    static_assert(std::is_integral<T>::value, "integer scans only");
    if constexpr (sizeof(T) == 4) {
        int x = (int)v;
        x += dpp_shift<0x111, 0xF>(x, 0);
        x += dpp_shift<0x112, 0xF>(x, 0);
        x += dpp_shift<0x114, 0xF>(x, 0);
        x += dpp_shift<0x118, 0xF>(x, 0);
        x += dpp_shift<0x142, 0xA>(x, 0);
        x += dpp_shift<0x143, 0xC>(x, 0);
        return (T)x;
    } else {
        int lane = threadIdx.x & 63;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            T o = __shfl_up(v, off, 64);
            if (lane >= off) v += o;
        }
        return v;
    }
}

// Exclusive scan over a block of NT threads; returns the block total too.
// lds must hold NT/64 elements.
template <typename T, int NT>
__device__ __forceinline__ T block_exclusive_scan(T v, T* total, T* lds)
{
    int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    T inc = wave_inclusive_scan(v);
    if (lane == 63) lds[wave] = inc;
    __syncthreads();
    T wbase = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) {
        T x = lds[w];
        if (w < wave) wbase += x;
        tot += x;
    }
    __syncthreads();
    *total = tot;
    return wbase + inc - v;
}

// ---- device-wide exclusive scan --------------------------------------------

template <typename TIn, typename T>
__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(const TIn* __restrict__ in, int64_t n,
                                                              T* __restrict__ block_sums)
{
    __shared__ T lds[kScanThreads / 64];
    int64_t base = (int64_t)blockIdx.x * kScanTile;
    T s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        int64_t idx = base + (int64_t)k * kScanThreads + threadIdx.x;
        if (idx < n) s += (T)in[idx];
    }
    T tot;
    block_exclusive_scan<T, kScanThreads>(s, &tot, lds);
    if (threadIdx.x == 0) block_sums[blockIdx.x] = tot;
}

// LDS index with one pad word per 32, so that lane t touching item t*NI + k
// (the per-thread serial scan) hits distinct banks.
__device__ __forceinline__ int pad32(int i) { return i + (i >> 5); }

// Block scan of NT*NI items: coalesced load to LDS, per-thread serial scan of
// NI consecutive items, block scan of the thread totals, coalesced store.
// The block's base is block_base[b] (scanned block totals) or, when
// block_sums is given instead, the sum of the raw totals of blocks 0..b-1.
template <typename TIn, typename T, int NT, int NI>
__global__ __launch_bounds__(NT) void k_scan_apply(const TIn* __restrict__ in, int64_t n,
                                                   const T* __restrict__ block_base,
                                                   const T* __restrict__ block_sums, T* __restrict__ out,
                                                   T* __restrict__ total_out)
{
    __shared__ T tile[NT * NI + NT * NI / 32];
    __shared__ T lds[NT / 64];
    T b0 = 0;
    if (block_base) {
        b0 = block_base[blockIdx.x];
    } else if (block_sums) {
        T part = 0;
        for (int i = threadIdx.x; i < (int)blockIdx.x; i += NT) part += block_sums[i];
        block_exclusive_scan<T, NT>(part, &b0, lds);
    }
    int64_t base = (int64_t)blockIdx.x * (NT * NI);
    const TIn* src = in + base;
    int lim = (int)min((int64_t)(NT * NI), n - base);
#pragma unroll 8
    for (int k = 0; k < NI; ++k) {
        int idx = k * NT + threadIdx.x;
        tile[pad32(idx)] = idx < lim ? (T)src[idx] : (T)0;
    }
    __syncthreads();
    T s = 0;
#pragma unroll
    for (int k = 0; k < NI; ++k) s += tile[pad32(threadIdx.x * NI + k)];
    T tot;
    T tb = block_exclusive_scan<T, NT>(s, &tot, lds);
    T run = b0 + tb;
    T bb = run - tb;
#pragma unroll
    for (int k = 0; k < NI; ++k) {
        T v = tile[pad32(threadIdx.x * NI + k)];
        tile[pad32(threadIdx.x * NI + k)] = run;
        run += v;
    }
    __syncthreads();
    T* dst = out + base;
#pragma unroll 8
    for (int k = 0; k < NI; ++k) {
        int idx = k * NT + threadIdx.x;
        if (idx < lim) dst[idx] = tile[pad32(idx)];
    }
    if (total_out && blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) *total_out = bb + tot;
}

// Up to this many blocks, each apply block sums the raw block totals before
// it itself (at most kDirectSums reads), which saves the scan of the totals.
constexpr int64_t kDirectSums = 1024;

// Scratch elements of type T the recursive scan of n items needs.
inline int64_t scan_scratch(int64_t n)
{
    int64_t need = 0;
    while (n > kScanTile) {
        n = qb_div_up(n, kScanTile);
        need += 2 * qb_div_up(n, 64) * 64;
    }
    return need + 64;
}

// out[i] = sum of in[0..i); *total_out (device, optional) = sum of all.
template <typename TIn, typename T>
qb_status exclusive_scan(const TIn* in, T* out, int64_t n, T* scratch, T* total_out, hipStream_t s)
{
    if (n <= 0) return QB_OK;
    if (n <= kScanTile) {
        QB_LAUNCH((k_scan_apply<TIn, T, kScanThreads, kScanItems>), 1, kScanThreads, 0, s, in, n,
                  (const T*)nullptr, (const T*)nullptr, out, total_out);
        return QB_OK;
    }
    if constexpr (sizeof(T) == 4) {
        if (n <= kBigScanTile) {
            QB_LAUNCH((k_scan_apply<TIn, T, kBigScanThreads, kBigScanItems>), 1, kBigScanThreads, 0, s, in, n,
                      (const T*)nullptr, (const T*)nullptr, out, total_out);
            return QB_OK;
        }
    }
    int64_t nb = qb_div_up(n, kScanTile);
    int64_t pad = qb_div_up(nb, 64) * 64;
    T* sums = scratch;
    T* sums_scan = scratch + pad;
    QB_LAUNCH((k_scan_reduce<TIn, T>), nb, kScanThreads, 0, s, in, n, sums);
    if (nb <= kDirectSums) {
        QB_LAUNCH((k_scan_apply<TIn, T, kScanThreads, kScanItems>), nb, kScanThreads, 0, s, in, n,
                  (const T*)nullptr, (const T*)sums, out, total_out);
        return QB_OK;
    }
    QB_CHECK((exclusive_scan<T, T>(sums, sums_scan, nb, scratch + 2 * pad, (T*)nullptr, s)));
    QB_LAUNCH((k_scan_apply<TIn, T, kScanThreads, kScanItems>), nb, kScanThreads, 0, s, in, n,
              (const T*)sums_scan, (const T*)nullptr, out, total_out);
    return QB_OK;
}

// ---- radix sort --------------------------------------------------------------

// Number of items the sort sees: *n_dev clamped to [0, cap]; a count above
// the capacity means the producer overflowed, and nothing is sorted.
__device__ __forceinline__ int64_t sort_count(const int64_t* n_dev, int64_t n_host, int64_t cap)
{
    int64_t n = n_dev ? *n_dev : n_host;
    if (n < 0 || n > cap) n = 0;
    return n;
}

template <typename K>
__device__ __forceinline__ uint32_t digit_of(K key, int shift, uint32_t mask)
{
    return (uint32_t)(key >> shift) & mask;
}

// Pass control of a 32-bit key sort whose pass count is settled on the device
// (radix_sort_span).  Keys equal to kNoKey are placed anywhere: they order
// nothing.  Pass 0's upsweep stores each block's (min, max) over the other
// keys in range[]; every pass-0 downsweep workgroup reduces them to the
// span's base b (the minimum rounded down to a multiple of 256), stores the
// other keys as key - b (kNoKey as 0: bits 0..7 of every other key are kept,
// so pass 0's own digits are those of the raw keys), and takes
// np = max(1, ceil(bits(max - b) / 8)) passes, which block 0 stores in *np.
// A later pass returns at once when pass >= *np.  The last pass writes to
// fin_keys (skipped when null) / fin_vals and gathers; the others write to
// their own outputs and do not gather.  pass < 0: an ordinary sort.
constexpr uint32_t kNoKey = 0xFFFFFFFFu;

struct PassCtl {
    uint2* range;
    int32_t* np;
    int pass;
    uint32_t* fin_keys;
    uint32_t* fin_vals;
};

inline PassCtl no_pass_ctl() { return PassCtl{nullptr, nullptr, -1, nullptr, nullptr}; }

__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = min(v, (uint32_t)__shfl_xor((int)v, o));
    return v;
}

__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, (uint32_t)__shfl_xor((int)v, o));
    return v;
}

// Data tile of radix workgroup w.  Workgroups go to the 8 XCDs round-robin
// (w % 8), so within each group of 256 workgroups, workgroup 8j + x takes
// tile 32x + j: 32 consecutive tiles run on one XCD.  Their 32 histogram words of a digit (one
// 128-byte line), their 32 digit offsets, and the output lines where one
// tile's run of a digit meets the next tile's, then pass through one XCD's L2
// as whole lines instead of partial lines from up to eight.  A tail of fewer
// than 256 workgroups keeps its order.  A bijection on [0, nblocks).
__device__ __forceinline__ int64_t xcd_tile(int64_t w, int64_t nblocks)
{
    constexpr int64_t kGroup = 256;
    if (w >= (nblocks / kGroup) * kGroup) return w;
    int64_t r = w & (kGroup - 1);
    return (w - r) + (r & 7) * 32 + (r >> 3);
}

// Per-block digit histogram.  Digit-major layout (hist[d * nblocks + b]) feeds
// the flat scan; block-major (hist[b * 256 + d], every digit written) feeds a
// downsweep that derives its own offsets.
template <typename K, int NT, int NI, bool BLOCK_MAJOR, bool RANGE = false>
__global__ __launch_bounds__(NT) void k_radix_upsweep(const K* __restrict__ keys, const int64_t* n_dev,
                                                      int64_t n_host, int64_t cap, int shift, int bits,
                                                      uint32_t* __restrict__ hist, int64_t nblocks, PassCtl ctl)
{
    static_assert(!RANGE || sizeof(K) == 4, "key spans are taken over 32-bit keys");
    if (ctl.pass > 0 && ctl.pass >= *ctl.np) return;  // a pass past the key span
    constexpr int NW = NT / 64;
    // kSub histograms per wave, a lane adding into copy lane % kSub; rows
    // padded by one word so that one digit lies in a different bank in each
    // copy: lanes holding the same digit (common in the high bits of sorted
    // neighbours) meet kSub-fold less often on one address
    constexpr int kSub = 4;
    constexpr int kRow = kRadix + 1;
    __shared__ uint32_t h[NW * kSub][kRow];
    int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    uint32_t mask = (1u << bits) - 1u;
    const int64_t tile = xcd_tile(blockIdx.x, nblocks);
    int64_t base = tile * (NT * NI) + (int64_t)wave * 64 * NI;
    // the wave's keys as 16-byte vectors, loaded first and bounded by the
    // capacity (which the buffer holds), so that their latency overlaps the
    // count's read; used when all 64*NI keys turn out to be below the count
    constexpr int kPerVec = 16 / sizeof(K);
    constexpr int kVecs = (int)(NI * sizeof(K) / 16);
    const K* wk = keys + base;
    bool vec_ok = (NI * sizeof(K)) % 16 == 0 && base + 64 * NI <= cap && ((uintptr_t)wk & 15u) == 0;
    uint4 xv[kVecs > 0 ? kVecs : 1];
    if (vec_ok) {
        const uint4* src = reinterpret_cast<const uint4*>(wk + (int64_t)lane * NI);
#pragma unroll
        for (int q = 0; q < kVecs; ++q) xv[q] = src[q];
    }
    // only the digits this pass can produce (0..mask) are cleared and summed
    for (int r = wave; r < NW * kSub; r += NW)
        for (int c = lane; c <= (int)mask; c += 64) h[r][c] = 0;
    __syncthreads();
    int64_t n = sort_count(n_dev, n_host, cap);
    uint32_t* hw = h[wave * kSub + (lane & (kSub - 1))];
    // the histogram ignores order: when the wave's 64*NI keys are all valid
    // and 16-byte aligned, each lane takes NI consecutive keys (the vectors
    // above) and adds each run of equal digits among them with one atomic
    // (runs are common where neighbouring keys share their high bits, and
    // same-address LDS atomics from many lanes serialise); otherwise one key
    // per lane per step
    bool vec = vec_ok && base + 64 * NI <= n;
    uint32_t klo = kNoKey, khi = 0u;  // RANGE: span of the keys other than kNoKey
    if (vec) {
        uint32_t cur = 0u, run = 0u;
#pragma unroll
        for (int q = 0; q < kVecs; ++q) {
            uint4 x = xv[q];
            const K* e = reinterpret_cast<const K*>(&x);
#pragma unroll
            for (int u = 0; u < kPerVec; ++u) {
                if (RANGE && (uint32_t)e[u] != kNoKey) {
                    klo = min(klo, (uint32_t)e[u]);
                    khi = max(khi, (uint32_t)e[u]);
                }
                uint32_t d = digit_of(e[u], shift, mask);
                if (run != 0u && d != cur) {
                    atomicAdd(&hw[cur], run);
                    run = 0u;
                }
                cur = d;
                ++run;
            }
        }
        atomicAdd(&hw[cur], run);   // run >= 1: the lane read NI >= 1 keys
    } else {
#pragma unroll 4
        for (int r = 0; r < NI; ++r) {
            int64_t idx = base + r * 64 + lane;
            if (idx < n) {
                K key = keys[idx];
                if (RANGE && (uint32_t)key != kNoKey) {
                    klo = min(klo, (uint32_t)key);
                    khi = max(khi, (uint32_t)key);
                }
                atomicAdd(&hw[digit_of(key, shift, mask)], 1u);
            }
        }
    }
    if (RANGE) {
        __shared__ uint32_t s_lo[NW], s_hi[NW];
        klo = wave_min_u32(klo);
        khi = wave_max_u32(khi);
        if (lane == 0) {
            s_lo[wave] = klo;
            s_hi[wave] = khi;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
#pragma unroll
            for (int w = 1; w < NW; ++w) {
                klo = min(klo, s_lo[w]);
                khi = max(khi, s_hi[w]);
            }
            ctl.range[tile] = make_uint2(klo, khi);
        }
    }
    __syncthreads();
    for (int d = threadIdx.x; d < kRadix; d += NT) {
        uint32_t t = 0;
        if (d <= (int)mask) {
#pragma unroll
            for (int w = 0; w < NW * kSub; ++w) t += h[w][d];
        }
        if (BLOCK_MAJOR)
            hist[tile * kRadix + d] = t;
        else if (d <= (int)mask)
            hist[(int64_t)d * nblocks + tile] = t;
    }
}

__device__ __forceinline__ bool b_any(const uint4& v) { return (v.x | v.y | v.z | v.w) != 0u; }

// FUSED: `offs` holds the raw block-major histograms of every block, and the
// workgroup derives its global digit offsets from them (digit totals scanned
// over digits, plus the counts of the earlier blocks); otherwise `offs` is the
// scanned digit-major histogram.  MODE: kMoveValues moves (key, value)
// pairs; kGather also writes gdst[pos] = gsrc[value] beside each moved value;
// kKeysOnly moves the keys alone (vals_in / vals_out unused); kKeysUnpack
// reads keys alone and writes each key split at bit `unpack_bits`: its high
// part to ((uint16_t*)keys_out)[pos], its low part to vals_out[pos].
enum { kMoveValues = 0, kGather = 1, kKeysOnly = 2, kKeysUnpack = 3 };

template <typename K, int NT, int NI, bool FUSED, int MODE>
__global__ __launch_bounds__(NT) void k_radix_downsweep(
    const K* __restrict__ keys_in, const uint32_t* __restrict__ vals_in, K* __restrict__ keys_out,
    uint32_t* __restrict__ vals_out, const int64_t* n_dev, int64_t n_host, int64_t cap, int shift, int bits,
    const uint32_t* __restrict__ offs, int64_t nblocks, const int32_t* __restrict__ gsrc,
    uint32_t* __restrict__ gdst, int unpack_bits, PassCtl ctl)
{
    constexpr bool VALUES = MODE == kMoveValues || MODE == kGather;
    static_assert(VALUES || sizeof(K) == 4, "keys-only passes move 32-bit keys");
    // pass control (PassCtl): last = write the final outputs and gather
    bool last = ctl.pass < 0;
    if (ctl.pass > 0) {
        int np = *ctl.np;
        if (ctl.pass >= np) return;
        last = ctl.pass == np - 1;
    }
    constexpr int NW = NT / 64;
    constexpr int TILE = NT * NI;
    __shared__ uint32_t wcnt[NW][kRadix];   // per-wave counts, then per-wave starts
    __shared__ uint32_t gbase[kRadix];      // global start of each digit for this block
    __shared__ uint32_t lstart[kRadix];     // block-local start of each digit
    __shared__ uint32_t scan_lds[NW];
    __shared__ uint32_t acc[FUSED ? 2 : 1][kRadix];   // FUSED: digit totals, counts in earlier blocks
    __shared__ K s_key[TILE];
    __shared__ uint32_t s_val[VALUES ? TILE : 1];
    int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t tile = xcd_tile(blockIdx.x, nblocks);   // the data tile
    int64_t blk0 = tile * TILE;
    int64_t base = blk0 + (int64_t)wave * 64 * NI;
    // the block's items are loaded first, bounded by the capacity (which the
    // buffers hold) rather than the count, so that their latency overlaps
    // the reads of the count and of the digit offsets
    K kv[NI];
    uint32_t vv[NI];
#pragma unroll
    for (int r = 0; r < NI; ++r) {
        int64_t idx = base + r * 64 + lane;
        bool inb = idx < cap;
        kv[r] = inb ? keys_in[idx] : (K)0;
        if (VALUES) vv[r] = inb ? (vals_in ? vals_in[idx] : (uint32_t)idx) : 0u;
    }
    uint32_t mask = (1u << bits) - 1u;
    // without the fused prologue, this block's digit offsets are read early too
    uint32_t gb_own = 0u;
    if (!FUSED && threadIdx.x <= mask) gb_own = offs[(int64_t)threadIdx.x * nblocks + tile];
    int64_t n = sort_count(n_dev, n_host, cap);
    if (blk0 >= n) return;
    int cnt_blk = (int)min((int64_t)TILE, n - blk0);
    for (int d = threadIdx.x; d < NW * kRadix; d += NT) (&wcnt[0][0])[d] = 0;
    if (FUSED) {
        static_assert(!FUSED || NT >= kRadix, "one lane per digit");
        // Every digit's total over all blocks and its count in the blocks
        // before this one.  Lane c of each wave reads digits 4c..4c+3 of one
        // block's 1 KB row as one 16-byte load; wave w takes blocks w, w + NW,
        // ..., so all the loads are independent and in flight together; the
        // waves' partial sums meet in LDS by atomic adds.
        for (int d = threadIdx.x; d < 2 * kRadix; d += NT) (&acc[0][0])[d] = 0u;
        __syncthreads();
        uint4 tot4 = make_uint4(0u, 0u, 0u, 0u), pre4 = make_uint4(0u, 0u, 0u, 0u);
        const uint4* rows = reinterpret_cast<const uint4*>(offs);
#pragma unroll 4
        for (int b = wave; b < (int)nblocks; b += NW) {
            uint4 v = rows[(int64_t)b * (kRadix / 4) + lane];
            bool before = b < (int)tile;
            tot4.x += v.x; tot4.y += v.y; tot4.z += v.z; tot4.w += v.w;
            pre4.x += before ? v.x : 0u; pre4.y += before ? v.y : 0u;
            pre4.z += before ? v.z : 0u; pre4.w += before ? v.w : 0u;
        }
        if (b_any(tot4)) {
            atomicAdd(&acc[0][4 * lane + 0], tot4.x);
            atomicAdd(&acc[0][4 * lane + 1], tot4.y);
            atomicAdd(&acc[0][4 * lane + 2], tot4.z);
            atomicAdd(&acc[0][4 * lane + 3], tot4.w);
        }
        if (b_any(pre4)) {
            atomicAdd(&acc[1][4 * lane + 0], pre4.x);
            atomicAdd(&acc[1][4 * lane + 1], pre4.y);
            atomicAdd(&acc[1][4 * lane + 2], pre4.z);
            atomicAdd(&acc[1][4 * lane + 3], pre4.w);
        }
        __syncthreads();
        int d = threadIdx.x;
        uint32_t tot = d < kRadix ? acc[0][d] : 0u, pre = d < kRadix ? acc[1][d] : 0u;
        uint32_t all;
        uint32_t start = block_exclusive_scan<uint32_t, NT>(d < kRadix ? tot : 0u, &all, gbase);
        if (d < kRadix) gbase[d] = start + pre;  // scan scratch reused after its last read
    } else {
        if (threadIdx.x <= mask) gbase[threadIdx.x] = gb_own;  // NT >= 256 > mask
    }
    uint32_t span_base = 0u;
    if (ctl.pass == 0) {
        // the span of the keys other than kNoKey over every block
        __shared__ uint32_t s_lo[NW], s_hi[NW];
        uint32_t lo = kNoKey, hi = 0u;
        for (int b = threadIdx.x; b < (int)nblocks; b += NT) {
            uint2 r = ctl.range[b];
            lo = min(lo, r.x);
            hi = max(hi, r.y);
        }
        lo = wave_min_u32(lo);
        hi = wave_max_u32(hi);
        if (lane == 0) {
            s_lo[wave] = lo;
            s_hi[wave] = hi;
        }
        __syncthreads();
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            lo = min(lo, s_lo[w]);
            hi = max(hi, s_hi[w]);
        }
        int np = 1;
        if (lo <= hi) {
            span_base = lo & ~0xFFu;
            uint32_t span = hi - span_base;
            int sb = span ? 32 - __clz((int)span) : 0;
            np = max(1, (sb + 7) >> 3);
        }
        if (blockIdx.x == 0 && threadIdx.x == 0) *ctl.np = np;
        last = np == 1;
    }
    __syncthreads();

    const uint64_t lt = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
    uint32_t rank[NI];
    uint32_t dig[NI];
#pragma unroll
    for (int r = 0; r < NI; ++r) {
        int64_t idx = base + r * 64 + lane;
        bool valid = idx < n;
        uint32_t d = digit_of(kv[r], shift, mask);
        uint64_t peers = __ballot(valid);
        for (int b = 0; b < bits; ++b) {
            bool bit = (d >> b) & 1u;
            uint64_t m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        uint32_t below = (uint32_t)__popcll(peers & lt);
        uint32_t cnt = (uint32_t)__popcll(peers);
        uint32_t old = valid ? wcnt[wave][d] : 0u;
        __builtin_amdgcn_wave_barrier();
        if (valid && below + 1 == cnt) wcnt[wave][d] = old + cnt;
        __builtin_amdgcn_wave_barrier();
        dig[r] = valid ? d : 0xFFFFFFFFu;
        rank[r] = old + below;
    }
    __syncthreads();
    // per digit: starts of each wave's items, block total, then block-local
    // digit starts (exclusive scan over digits)
    uint32_t tot_d = 0;
    int d_own = threadIdx.x;
    if (d_own < kRadix && d_own <= (int)mask) {
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            uint32_t t = wcnt[w][d_own];
            wcnt[w][d_own] = tot_d;
            tot_d += t;
        }
    }
    static_assert(NT >= kRadix, "one lane per digit");
    uint32_t dummy;
    uint32_t ls = block_exclusive_scan<uint32_t, NT>(d_own < kRadix ? tot_d : 0u, &dummy, scan_lds);
    if (d_own < kRadix) lstart[d_own] = ls;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < NI; ++r) {
        if (dig[r] == 0xFFFFFFFFu) continue;
        uint32_t lp = lstart[dig[r]] + wcnt[wave][dig[r]] + rank[r];
        s_key[lp] = kv[r];
        if (VALUES) s_val[lp] = vv[r];
    }
    __syncthreads();
    K* ko = keys_out;
    uint32_t* vo = vals_out;
    if (ctl.pass >= 0 && last) {
        ko = reinterpret_cast<K*>(ctl.fin_keys);
        vo = ctl.fin_vals;
    }
    bool gather = MODE == kGather && last;
    for (int i = threadIdx.x; i < cnt_blk; i += NT) {
        K k = s_key[i];
        uint32_t d = digit_of(k, shift, mask);
        uint32_t pos = gbase[d] + (uint32_t)i - lstart[d];
        if constexpr (MODE == kKeysUnpack) {
            reinterpret_cast<uint16_t*>(keys_out)[pos] = (uint16_t)((uint32_t)k >> unpack_bits);
            vals_out[pos] = (uint32_t)k & ((1u << unpack_bits) - 1u);
        } else if constexpr (MODE == kKeysOnly) {
            keys_out[pos] = k;
        } else {
            uint32_t v = s_val[i];
            if (ctl.pass == 0) k = (uint32_t)k == kNoKey ? (K)0 : (K)((uint32_t)k - span_base);
            if (ko) ko[pos] = k;
            vo[pos] = v;
            if (gather) gdst[pos] = (uint32_t)gsrc[v];
        }
    }
}

// Scratch bytes of one sort over `cap` items with NT*NI items per block.
template <int NT, int NI>
inline size_t radix_scratch_bytes(int64_t cap)
{
    int64_t nb = qb_div_up(cap > 0 ? cap : 1, NT * NI);
    int64_t hist = nb * kRadix;
    return (size_t)(2 * hist + scan_scratch(hist) + 256) * sizeof(uint32_t);
}

template <typename K, int NT, int NI>
__global__ __launch_bounds__(QB_BLOCK) void k_copy_items(const K* __restrict__ kin, const uint32_t* __restrict__ vin,
                                                         K* __restrict__ kout, uint32_t* __restrict__ vout,
                                                         const int64_t* n_dev, int64_t n_host, int64_t cap)
{
    int64_t n = sort_count(n_dev, n_host, cap);
    for (int64_t i = (int64_t)blockIdx.x * QB_BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * QB_BLOCK) {
        kout[i] = kin[i];
        vout[i] = vin[i];
    }
}

// Stable sort of (keys, vals) by key bits [lo_bit, hi_bit) in passes of at
// most 8 bits (bits spread evenly over the passes).  vin may be null: the
// values are then the input positions 0, 1, 2, ...  Reads (kin, vin), ends in
// (kout, vout), and uses (ktmp, vtmp) for the intermediate passes; kin may
// alias kout only when the pass count is even.  The item count is *n_dev when
// n_dev is given (clamped as in sort_count), else n_host; cap sizes the grid.
// gsrc/gdst (both or neither): the last pass also writes gdst[i] = gsrc[vout[i]].
// first_bits > 0
// sets the first pass's digit width (at most 8, leaving at least one bit; the
// pass count is unchanged, so the later passes must hold the rest: callers
// keep total - first_bits <= 8 per remaining pass); 0 splits evenly.
template <typename K, int NT, int NI>
qb_status radix_sort(const K* kin, const uint32_t* vin, K* kout, uint32_t* vout, K* ktmp, uint32_t* vtmp,
                     const int64_t* n_dev, int64_t n_host, int64_t cap, int lo_bit, int hi_bit,
                     uint32_t* scratch, hipStream_t s, const int32_t* gsrc = nullptr, uint32_t* gdst = nullptr,
                     int first_bits = 0)
{
    if (cap <= 0) return QB_OK;
    if ((gsrc != nullptr) != (gdst != nullptr) || (gsrc && hi_bit <= lo_bit)) return QB_ERR_INVALID_ARG;
    int total_bits = hi_bit - lo_bit;
    int np = total_bits > 0 ? (total_bits + kRadixBits - 1) / kRadixBits : 0;
    if (np == 0) {
        if (gsrc) return QB_ERR_INVALID_ARG;
        if ((const void*)kin != (const void*)kout) {
            int64_t g = qb_div_up(cap, QB_BLOCK);
            if (g > 4096) g = 4096;
            QB_LAUNCH((k_copy_items<K, NT, NI>), g, QB_BLOCK, 0, s, kin, vin, kout, vout, n_dev, n_host, cap);
        }
        return QB_OK;
    }
    int64_t nb = qb_div_up(cap, NT * NI);
    int64_t hn = nb * kRadix;
    uint32_t* hist = scratch;
    uint32_t* offs = scratch + hn;
    uint32_t* sscr = scratch + 2 * hn;
    // few blocks: every downsweep workgroup reads all histograms itself
    // (at most kFusedBlocks KB, from L2), which saves the two scan launches
    bool fused = nb <= kFusedBlocks && NT >= kRadix;
    int shift = lo_bit;
    const K* src_k = kin;
    const uint32_t* src_v = vin;
    for (int p = 0; p < np; ++p) {
        int bits = (total_bits - (shift - lo_bit) + (np - p) - 1) / (np - p);
        if (p == 0 && np > 1 && first_bits > 0)
            bits = min(first_bits, min(kRadixBits, total_bits - 1));   // the later passes share the rest
        bool to_out = ((np - 1 - p) & 1) == 0;
        K* dk = to_out ? kout : ktmp;
        uint32_t* dv = to_out ? vout : vtmp;
        int64_t hn_used = (int64_t)(1 << bits) * nb;
        bool gather = gsrc && p == np - 1;
        const uint32_t* o = (const uint32_t*)hist;
        if (fused) {
            QB_LAUNCH((k_radix_upsweep<K, NT, NI, true>), nb, NT, 0, s, src_k, n_dev, n_host, cap, shift, bits,
                      hist, nb, no_pass_ctl());
        } else {
            QB_LAUNCH((k_radix_upsweep<K, NT, NI, false>), nb, NT, 0, s, src_k, n_dev, n_host, cap, shift, bits,
                      hist, nb, no_pass_ctl());
            QB_CHECK((exclusive_scan<uint32_t, uint32_t>(hist, offs, hn_used, sscr, (uint32_t*)nullptr, s)));
            o = (const uint32_t*)offs;
        }
#define QB_DOWNSWEEP(F, M)                                                                                    \
    QB_LAUNCH((k_radix_downsweep<K, NT, NI, F, M>), nb, NT, 0, s, src_k, src_v, dk, dv, n_dev, n_host, cap,  \
              shift, bits, o, nb, M == kGather ? gsrc : (const int32_t*)nullptr,                              \
              M == kGather ? gdst : (uint32_t*)nullptr, 0, no_pass_ctl())
        if (fused && gather) QB_DOWNSWEEP(true, kGather);
        else if (fused) QB_DOWNSWEEP(true, kMoveValues);
        else if (gather) QB_DOWNSWEEP(false, kGather);
        else QB_DOWNSWEEP(false, kMoveValues);
#undef QB_DOWNSWEEP
        src_k = dk;
        src_v = dv;
        shift += bits;
    }
    return QB_OK;
}

// Stable sort of 32-bit packed keys by their bits [lo_bit, hi_bit) (at most
// two passes of at most 8 bits), moving the keys alone; the last pass writes
// each sorted key split at lo_bit: key >> lo_bit to hi_out (uint16), the low
// lo_bit bits to lo_out.  tmp holds the keys between the passes.  Counts and
// grid as radix_sort; first_bits as there.
template <int NT, int NI>
qb_status radix_sort_packed(const uint32_t* kin, uint32_t* tmp, uint16_t* hi_out, uint32_t* lo_out,
                            const int64_t* n_dev, int64_t cap, int lo_bit, int hi_bit, uint32_t* scratch,
                            hipStream_t s, int first_bits = 0)
{
    if (cap <= 0) return QB_OK;
    int total_bits = hi_bit - lo_bit;
    int np = (total_bits + kRadixBits - 1) / kRadixBits;
    if (total_bits <= 0 || np > 2 || lo_bit <= 0 || hi_bit > 32 || hi_bit - lo_bit > 16) return QB_ERR_INVALID_ARG;
    int64_t nb = qb_div_up(cap, NT * NI);
    int64_t hn = nb * kRadix;
    uint32_t* hist = scratch;
    uint32_t* offs = scratch + hn;
    uint32_t* sscr = scratch + 2 * hn;
    bool fused = nb <= kFusedBlocks && NT >= kRadix;
    int shift = lo_bit;
    const uint32_t* src = kin;
    for (int p = 0; p < np; ++p) {
        int bits = (total_bits - (shift - lo_bit) + (np - p) - 1) / (np - p);
        if (p == 0 && np > 1 && first_bits > 0) bits = min(first_bits, min(kRadixBits, total_bits - 1));
        bool last = p == np - 1;
        int64_t hn_used = (int64_t)(1 << bits) * nb;
        const uint32_t* o = (const uint32_t*)hist;
        if (fused) {
            QB_LAUNCH((k_radix_upsweep<uint32_t, NT, NI, true>), nb, NT, 0, s, src, n_dev, (int64_t)0, cap, shift,
                      bits, hist, nb, no_pass_ctl());
        } else {
            QB_LAUNCH((k_radix_upsweep<uint32_t, NT, NI, false>), nb, NT, 0, s, src, n_dev, (int64_t)0, cap, shift,
                      bits, hist, nb, no_pass_ctl());
            QB_CHECK((exclusive_scan<uint32_t, uint32_t>(hist, offs, hn_used, sscr, (uint32_t*)nullptr, s)));
            o = (const uint32_t*)offs;
        }
#define QB_DOWNSWEEP_PACKED(F, M, OUTK, OUTV)                                                                  \
    QB_LAUNCH((k_radix_downsweep<uint32_t, NT, NI, F, M>), nb, NT, 0, s, src, (const uint32_t*)nullptr, OUTK,   \
              OUTV, n_dev, (int64_t)0, cap, shift, bits, o, nb, (const int32_t*)nullptr, (uint32_t*)nullptr,     \
              lo_bit, no_pass_ctl())
        uint32_t* hk = reinterpret_cast<uint32_t*>(hi_out);
        if (last && fused) QB_DOWNSWEEP_PACKED(true, kKeysUnpack, hk, lo_out);
        else if (last) QB_DOWNSWEEP_PACKED(false, kKeysUnpack, hk, lo_out);
        else if (fused) QB_DOWNSWEEP_PACKED(true, kKeysOnly, tmp, (uint32_t*)nullptr);
        else QB_DOWNSWEEP_PACKED(false, kKeysOnly, tmp, (uint32_t*)nullptr);
#undef QB_DOWNSWEEP_PACKED
        src = tmp;
        shift += bits;
    }
    return QB_OK;
}

// Stable sort of n 32-bit keys (kNoKey: placed anywhere) with their
// positions as values, in 8-bit passes over the span of the other keys only
// (PassCtl): the pass count is settled on the device by the first pass, and
// the passes beyond it return at once.  Reads kin; (ka, va) and (kb, vb) hold
// the items between passes (pass p writes to a when p is even, b when odd;
// kb may be kin's buffer, which only pass 0 reads); the last pass writes the
// sorted positions to fin_vals and gdst[i] = gsrc[fin_vals[i]], but no keys.
// n items (host count) in at most kFusedBlocks blocks of NT*NI; scratch as
// radix_scratch_bytes.
template <int NT, int NI>
qb_status radix_sort_span(const uint32_t* kin, uint32_t* ka, uint32_t* va, uint32_t* kb, uint32_t* vb,
                          uint32_t* fin_vals, int64_t n, uint32_t* scratch, hipStream_t s, const int32_t* gsrc,
                          uint32_t* gdst)
{
    static_assert(NT >= kRadix, "one lane per digit");
    if (n <= 0) return QB_OK;
    int64_t nb = qb_div_up(n, NT * NI);
    if (nb > kFusedBlocks || !gsrc || !gdst) return QB_ERR_INVALID_ARG;
    int64_t hn = nb * kRadix;
    uint32_t* hist = scratch;
    // block key ranges and the pass count in the scan-offset area, which a
    // fused sort does not use (2 * nb + 1 <= 256 * nb words)
    uint2* range = reinterpret_cast<uint2*>(scratch + hn);
    int32_t* np = reinterpret_cast<int32_t*>(scratch + hn + 2 * nb);
    const uint32_t* src_k = kin;
    const uint32_t* src_v = nullptr;
    for (int p = 0; p < 32 / kRadixBits; ++p) {
        uint32_t* dk = (p & 1) ? kb : ka;
        uint32_t* dv = (p & 1) ? vb : va;
        PassCtl ctl{range, np, p, nullptr, fin_vals};
        int shift = p * kRadixBits;
        if (p == 0)
            QB_LAUNCH((k_radix_upsweep<uint32_t, NT, NI, true, true>), nb, NT, 0, s, src_k, (const int64_t*)nullptr,
                      n, n, shift, kRadixBits, hist, nb, ctl);
        else
            QB_LAUNCH((k_radix_upsweep<uint32_t, NT, NI, true, false>), nb, NT, 0, s, src_k, (const int64_t*)nullptr,
                      n, n, shift, kRadixBits, hist, nb, ctl);
        QB_LAUNCH((k_radix_downsweep<uint32_t, NT, NI, true, kGather>), nb, NT, 0, s, src_k, src_v, dk, dv,
                  (const int64_t*)nullptr, n, n, shift, kRadixBits, (const uint32_t*)hist, nb, gsrc, gdst, 0, ctl);
        src_k = dk;
        src_v = dv;
    }
    return QB_OK;
}

}  // namespace qbr
