// Stable LSD radix passes (8-bit digits) and an exclusive scan, in the
// reduce-then-scan form: no block ever waits on another block.
//
// One pass over `count` keys, partitions of kSortTile consecutive items:
//   upsweep   : per-partition digit counts -> counts[digit][partition]
//   scan_rows : exclusive scan of each digit row, row totals
//   downsweep : each partition ranks its items stably in LDS (wave ballots
//               per digit bit, per-wave running counters), stages them in
//               digit order and writes each digit run to
//               sum_{d' < d} total(d') + counts[d][p] + local rank,
//               so a partition's stores of one digit are contiguous.
// The first depth pass drops culled items (depth key 0xFFFFFFFF), so the
// later passes and everything after them see only the visible items.  The
// downsweep of the last depth pass also writes, in sorted order, each
// item's tile rectangle and its number of (strip, item) entries (tile rows
// times strip columns of the rectangle); the scan below turns those into
// entry offsets and also sums the (tile, item) pairs.
#include "common.hpp"
#include "pairs.hpp"

namespace sgs {

__device__ __forceinline__ int64_t pass_count(const uint32_t* count_ptr, int64_t count_host) {
    int64_t c = count_host;
    if (count_ptr && (int64_t)*count_ptr < c) c = *count_ptr;
    return c;
}

__device__ __forceinline__ uint32_t rect_pairs(uint64_t r) {
    const int tx0 = (int)(r & 0xFFFF), tx1 = (int)((r >> 16) & 0xFFFF);
    const int ty0 = (int)((r >> 32) & 0xFFFF), ty1 = (int)((r >> 48) & 0xFFFF);
    const int w = tx1 - tx0 + 1, h = ty1 - ty0 + 1;
    return (w > 0 && h > 0) ? (uint32_t)(w * h) : 0u;
}

// (strip, item) entries of a tile rectangle: rows times strip columns
__device__ __forceinline__ uint32_t rect_entries(uint64_t r) {
    const int tx0 = (int)(r & 0xFFFF), tx1 = (int)((r >> 16) & 0xFFFF);
    const int ty0 = (int)((r >> 32) & 0xFFFF), ty1 = (int)((r >> 48) & 0xFFFF);
    const int w = (tx1 >> kStripShift) - (tx0 >> kStripShift) + 1, h = ty1 - ty0 + 1;
    return (tx1 >= tx0 && h > 0) ? (uint32_t)(w * h) : 0u;
}

// ---------------------------------------------------------------------------

// Digit histogram of one partition (per-wave LDS rows, atomics).  A digit of
// fewer than 8 bits takes few values, each repeated across a wave's lanes;
// its bins are spread over 2^c copies per wave (c = min(3, 8 - bits)),
// picked by lane, so equal digits rarely hit the same LDS word.  Only the
// 2^bits live digit rows are written.
template <typename KeyT>
__global__ void __launch_bounds__(kSortThreads)
k_upsweep(const KeyT* __restrict__ keys, const uint32_t* count_ptr, int64_t count_host,
          int shift, uint32_t* __restrict__ counts, int64_t parts, bool drop, int digit_bits) {
    constexpr int WAVES = kSortThreads / 64;
    __shared__ uint32_t hist[WAVES][kRadix];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int cl = kRadixBits - digit_bits < 3 ? kRadixBits - digit_bits : 3;
    const uint32_t dmask = (1u << digit_bits) - 1u, cmask = (1u << cl) - 1u;
    for (int i = tid; i < WAVES * kRadix; i += kSortThreads) (&hist[0][0])[i] = 0;
    __syncthreads();
    const int64_t count = pass_count(count_ptr, count_host);
    const int64_t p = xcd_part(blockIdx.x, (count + kSortTile - 1) / kSortTile);
    const int64_t base = p * kSortTile;
    const uint32_t lane_bin = (uint32_t)lane & cmask;
    auto add = [&](uint32_t key) {
        if (!drop || key != 0xFFFFFFFFu) atomicAdd(&hist[wave][(((key >> shift) & dmask) << cl) | lane_bin], 1u);
    };
    if (base + kSortTile <= count && ((uintptr_t)keys & 15u) == 0) {
        // a full partition: 16-byte loads, each wave instruction reading 1 KB
        // contiguous (a histogram does not depend on the order of the items)
        constexpr int PER = 16 / (int)sizeof(KeyT);
        const uint4* __restrict__ src = reinterpret_cast<const uint4*>(keys + base);
#pragma unroll
        for (int j = 0; j < kSortItems / PER; ++j) {
            const uint4 q = src[j * kSortThreads + tid];
            const uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                if constexpr (sizeof(KeyT) == 2) {
                    add(w[e] & 0xFFFFu);
                    add(w[e] >> 16);
                } else {
                    add(w[e]);
                }
            }
        }
    } else {
#pragma unroll 4
        for (int k = 0; k < kSortItems; ++k) {
            const int64_t i = base + (int64_t)k * kSortThreads + tid;
            if (i < count) add(keys[i]);
        }
    }
    __syncthreads();
    const int d = tid;
    if (d > (int)dmask) return;
    uint32_t c = 0;
#pragma unroll
    for (int w = 0; w < WAVES; ++w)
        for (int j = 0; j <= (int)cmask; ++j) c += hist[w][(d << cl) + j];
    counts[(int64_t)d * parts + p] = c;
}

constexpr int kScanRowThreads = 1024;
constexpr int kScanRowItems = 16;

// block d: exclusive scan of counts[d][0 .. live) in place, where the row
// holds `parts` entries of `per` items each and live covers the pass's
// items (count_ptr / count_host); totals[d] = row sum (also added to
// *kept_out when given).  Entries past live are neither read nor written.
// Each thread owns 16 consecutive entries per round, read and written as
// four 16-byte words when the row is 16-byte aligned, so a row of up to 16K
// partitions takes one round; wave scans with lane shuffles, then a scan of
// the 16 wave totals.
__global__ void __launch_bounds__(kScanRowThreads)
k_scan_rows(uint32_t* __restrict__ counts, int64_t parts, uint32_t* __restrict__ totals,
            uint32_t* kept_out, const uint32_t* count_ptr, int64_t count_host, int per) {
    constexpr int WAVES = kScanRowThreads / 64;
    constexpr int IT = kScanRowItems;
    __shared__ uint32_t s_w[WAVES];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    uint32_t* row = counts + (int64_t)blockIdx.x * parts;
    const bool vec = (reinterpret_cast<uintptr_t>(row) & 15) == 0;
    const int64_t items = pass_count(count_ptr, count_host);
    const int64_t live_parts = (items + per - 1) / per;
    const int64_t live = live_parts < parts ? live_parts : parts;
    uint32_t carry = 0;
    for (int64_t b0 = 0; b0 < live; b0 += kScanRowThreads * IT) {
        const int64_t i0 = b0 + (int64_t)tid * IT;
        const bool whole = vec && i0 + IT <= live;
        uint32_t v[IT], run = 0;
        if (whole) {
#pragma unroll
            for (int q = 0; q < IT / 4; ++q) {
                const uint4 t = *reinterpret_cast<const uint4*>(row + i0 + 4 * q);
                v[4 * q] = t.x; v[4 * q + 1] = t.y; v[4 * q + 2] = t.z; v[4 * q + 3] = t.w;
            }
        } else {
#pragma unroll
            for (int k = 0; k < IT; ++k) v[k] = i0 + k < live ? row[i0 + k] : 0u;
        }
#pragma unroll
        for (int k = 0; k < IT; ++k) run += v[k];
        uint32_t x = run;   // inclusive scan over the wave
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t y = __shfl_up(x, off);
            if (lane >= off) x += y;
        }
        if (lane == 63) s_w[w] = x;
        __syncthreads();
        if (w == 0) {
            uint32_t t = lane < WAVES ? s_w[lane] : 0u;
#pragma unroll
            for (int off = 1; off < WAVES; off <<= 1) {
                const uint32_t y = __shfl_up(t, off);
                if (lane >= off) t += y;
            }
            if (lane < WAVES) s_w[lane] = t;   // inclusive over waves
        }
        __syncthreads();
        uint32_t off = carry + (w > 0 ? s_w[w - 1] : 0u) + x - run;
#pragma unroll
        for (int k = 0; k < IT; ++k) {
            const uint32_t e = off;
            off += v[k];
            v[k] = e;
        }
        if (whole) {
#pragma unroll
            for (int q = 0; q < IT / 4; ++q)
                *reinterpret_cast<uint4*>(row + i0 + 4 * q) =
                    make_uint4(v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]);
        } else {
#pragma unroll
            for (int k = 0; k < IT; ++k)
                if (i0 + k < live) row[i0 + k] = v[k];
        }
        carry += s_w[WAVES - 1];
        __syncthreads();
    }
    if (tid == 0) {
        totals[blockIdx.x] = carry;
        if (kept_out) atomicAdd(kept_out, carry);
    }
}

// Exclusive scan of one value per thread of a block of WAVES waves: lane
// shuffles within each wave, then the wave totals through s_w (WAVES words no
// other thread touches until the next barrier).  One barrier; *total
// receives the block's sum.
template <int WAVES>
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t* s_w, uint32_t* total) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    if (lane == 63) s_w[wave] = x;
    __syncthreads();
    uint32_t before = 0, all = 0;
#pragma unroll
    for (int w = 0; w < WAVES; ++w) {
        const uint32_t t = s_w[w];
        before += w < wave ? t : 0u;
        all += t;
    }
    *total = all;
    return before + x - v;
}

// The downsweep runs 512 threads of 8 items over a kSortTile partition: a
// wave's serial ranking chain is 8 items long, and three blocks (24 waves)
// share a CU.
constexpr int kDownThreads = 512;
constexpr int kDownItems = kSortTile / kDownThreads;

// The downsweep after its items are in registers (key[k], val[k] of item
// k * 64 + lane of this wave; lim: the wave's valid items): stable ranking
// by digit, block digit offsets, staging in LDS in digit order and the
// scatter to s_global[d] + staged index.  Expects s_global to hold the
// partition's digit starts, s_wave cleared and s_kv free (a barrier after
// their last use).
template <typename KeyT, int NB>
__device__ __forceinline__ void rank_scatter(uint32_t (&key)[kDownItems], const uint32_t (&val)[kDownItems],
                                             int lim, bool drop, int shift, uint64_t* s_kv,
                                             uint32_t (*s_wave)[kRadix], uint32_t* s_local,
                                             uint32_t* s_global, uint32_t* s_scan1,
                                             KeyT* __restrict__ keys_out, uint32_t* __restrict__ vals_out,
                                             const uint64_t* __restrict__ rects,
                                             uint32_t* __restrict__ pairs_out,
                                             uint64_t* __restrict__ rects_out, int64_t n_rects,
                                             uint32_t* __restrict__ ranges, int64_t n_tiles,
                                             int64_t out_limit) {
    constexpr int WAVES = kDownThreads / 64;
    // digits of 5 bits or more: lanes with equal digits are found through a
    // per-wave table of lane masks (one LDS OR and one read per item) instead
    // of NB ballots; the table lives in s_kv, which the ranking does not use
    // yet.  Shorter digits keep the ballots (few, and many lanes would share
    // a table entry).
    constexpr bool kLdsMatch = NB >= 5;
    static_assert(WAVES * kRadix * 8 <= kSortTile * 8, "match tables fit in s_kv");
    unsigned long long* s_match = reinterpret_cast<unsigned long long*>(s_kv);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    uint32_t rank2[kDownItems / 2];   // two 16-bit ranks per register
    if (kLdsMatch) {
        for (int i = tid; i < WAVES * kRadix; i += kDownThreads) s_match[i] = 0ull;
        __syncthreads();
    }

    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
    for (int k = 0; k < kDownItems; ++k) {
        const int li = k * 64 + lane;
        const bool valid = li < lim && !(drop && key[k] == 0xFFFFFFFFu);
        const uint32_t d = (key[k] >> shift) & (kRadix - 1);
        uint64_t m;
        if constexpr (kLdsMatch) {
            // a wave's LDS instructions execute in order: every lane's OR
            // lands before any lane reads, every read before the clear
            unsigned long long* slot = s_match + wave * kRadix + d;
            if (valid) atomicOr(slot, 1ull << lane);
            m = valid ? *slot : 0ull;
            if (valid) *slot = 0ull;
        } else {
            m = __ballot(valid);
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                const bool bit = (d >> b) & 1u;
                const uint64_t bb = __ballot(bit);
                m &= bit ? bb : ~bb;
            }
        }
        const uint64_t lower = m & lt_mask;
        const uint32_t prior = valid ? s_wave[wave][d] : 0u;
        const uint32_t r = prior + (uint32_t)__popcll(lower);
        rank2[k >> 1] = (k & 1) ? (rank2[k >> 1] | (r << 16)) : r;
        if (valid && lower == 0) s_wave[wave][d] = prior + (uint32_t)__popcll(m);
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    int n_valid;
    {
        // per digit: exclusive offsets of the waves, then the block's digit starts
        uint32_t total = 0;
        if (tid < kRadix) {
#pragma unroll
            for (int w = 0; w < WAVES; ++w) {
                const uint32_t c = s_wave[w][tid];
                s_wave[w][tid] = total;
                total += c;
            }
        }
        uint32_t kept;
        const uint32_t st = block_excl_scan<WAVES>(total, s_scan1, &kept);
        if (tid < kRadix) {
            s_local[tid] = st;
            s_global[tid] -= st;   // now: output index of staged slot i is s_global[d] + i
        }
        n_valid = (int)kept;
        __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < kDownItems; ++k) {
        const int li = k * 64 + lane;
        if (li < lim && !(drop && key[k] == 0xFFFFFFFFu)) {
            const uint32_t dd = (key[k] >> shift) & (kRadix - 1);
            const uint32_t pos = s_local[dd] + s_wave[wave][dd] + ((rank2[k >> 1] >> (16 * (k & 1))) & 0xFFFFu);
            s_kv[pos] = (uint64_t)key[k] | ((uint64_t)val[k] << 32);
        }
    }
    __syncthreads();
    // unrolled over the thread's fixed slots so that the LDS reads and the
    // stores of different items overlap
#pragma unroll
    for (int j = 0; j < kDownItems; ++j) {
        const int i = tid + j * kDownThreads;
        if (i >= n_valid) break;
        const uint64_t kv = s_kv[i];
        const uint32_t k = (uint32_t)kv, v = (uint32_t)(kv >> 32);
        const uint32_t dd = (k >> shift) & (kRadix - 1);
        const uint32_t out = s_global[dd] + (uint32_t)i;
        // counts that disagree with the items would point past the pass's
        // output: such an item is not written (the result is then wrong,
        // never out of bounds)
        if ((int64_t)out >= out_limit) continue;
        __builtin_assume(out < (1u << 30));
        if (keys_out) keys_out[out] = (KeyT)k;
        vals_out[out] = v;
        if (pairs_out) {   // last depth pass: entry count and rectangle in depth order
            const uint64_t r = v < (uint64_t)n_rects ? rects[v] : 1ull;   // 1: no pairs
            pairs_out[out] = rect_entries(r);
            if (rects_out) rects_out[out] = r;
        }
        // last tile pass: a key change between neighbours of this block's run
        // of one digit is a tile boundary (run starts, where the previous
        // staged key has another digit, are checked by k_range_edges)
        if (ranges && i > 0) {
            const uint32_t pk = (uint32_t)s_kv[i - 1];
            if (pk != k && ((pk >> shift) & (kRadix - 1)) == dd) {
                if (k < (uint64_t)n_tiles) ranges[2 * (int64_t)k] = out;
                if (pk < (uint64_t)n_tiles) ranges[2 * (int64_t)pk + 1] = out;
            }
        }
    }
}

// NB: significant bits of the digit (the key has no bits above shift + NB),
// so ranking needs NB ballots instead of kRadixBits.
template <typename KeyT, int NB>
__global__ void __launch_bounds__(kDownThreads)
k_downsweep(const KeyT* __restrict__ keys_in, const uint32_t* __restrict__ vals_in,
            KeyT* __restrict__ keys_out, uint32_t* __restrict__ vals_out,
            const uint32_t* count_ptr, int64_t count_host, int shift,
            const uint32_t* __restrict__ counts, const uint32_t* __restrict__ totals, int64_t parts,
            const uint64_t* __restrict__ rects, uint32_t* __restrict__ pairs_out,
            uint64_t* __restrict__ rects_out, int64_t n_rects,
            bool drop, int cstride, uint32_t* __restrict__ ranges, int64_t n_tiles) {
    constexpr int WAVES = kDownThreads / 64;
    constexpr int WAVE_ITEMS = 64 * kDownItems;
    // staged (key, value) words: key in the low half, value in the high half
    __shared__ __align__(16) uint64_t s_kv[kSortTile];
    __shared__ uint32_t s_wave[WAVES][kRadix];
    __shared__ uint32_t s_local[kRadix];
    __shared__ uint32_t s_global[kRadix];
    __shared__ uint32_t s_scan[2][WAVES];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t count = pass_count(count_ptr, count_host);
    const int64_t p = xcd_part(blockIdx.x, (count + kSortTile - 1) / kSortTile);
    const int64_t base = p * kSortTile;
    if (base >= count) return;
    // thread d < 2^NB owns digit d; digits from 2^NB on do not occur (their
    // rows are neither written by the upsweep nor scanned)
    constexpr int kLive = 1 << NB;
    const uint32_t tot = tid < kLive ? totals[tid] : 0u;
    const uint32_t cnt_dp = tid < kLive ? counts[((int64_t)tid * parts + p) * cstride] : 0u;

    // this partition's items, issued before the digit-start scan so that
    // their latency overlaps it.  A full partition comes in by direct
    // 16-byte global->LDS loads (keys into the first half of s_kv, values
    // into the second, no
    // registers held in flight); the ragged last one by per-lane loads.
    uint32_t key[kDownItems], val[kDownItems];
    // this wave's items in 32-bit offsets from a wave-uniform base pointer
    // (counts stay below 2^30)
    const int64_t wbase = base + (int64_t)wave * WAVE_ITEMS;
    const int64_t left = count - wbase;
    const int lim = left <= 0 ? 0 : (left >= WAVE_ITEMS ? WAVE_ITEMS : (int)left);
    const bool full = base + kSortTile <= count && ((uintptr_t)keys_in & 15u) == 0 &&
                      ((uintptr_t)vals_in & 15u) == 0;
    if (full) {
        constexpr int KCH = kSortTile * (int)sizeof(KeyT) / 1024;   // 1 KB chunks of keys
        const char* gk = reinterpret_cast<const char*>(keys_in + base);
        for (int c = wave; c < KCH; c += WAVES)
            __builtin_amdgcn_global_load_lds(
                (const __attribute__((address_space(1))) void*)(gk + c * 1024 + lane * 16),
                (__attribute__((address_space(3))) void*)(reinterpret_cast<char*>(s_kv) + c * 1024),
                16, 0, 0);
        if (vals_in) {
            const char* gv = reinterpret_cast<const char*>(vals_in + base);
            for (int c = wave; c < kSortTile * 4 / 1024; c += WAVES)
                __builtin_amdgcn_global_load_lds(
                    (const __attribute__((address_space(1))) void*)(gv + c * 1024 + lane * 16),
                    (__attribute__((address_space(3))) void*)(reinterpret_cast<char*>(s_kv) + kSortTile * 4 + c * 1024),
                    16, 0, 0);
        }
    } else {
        const KeyT* __restrict__ kin = keys_in + wbase;
        const uint32_t* __restrict__ vin = vals_in ? vals_in + wbase : nullptr;
#pragma unroll
        for (int k = 0; k < kDownItems; ++k) {
            const int li = k * 64 + lane;
            if (li < lim) {
                key[k] = kin[li];
                val[k] = vin ? vin[li] : (uint32_t)wbase + (uint32_t)li;
            } else {
                key[k] = 0xFFFFFFFFu;
                val[k] = 0;
            }
        }
    }
    for (int i = tid; i < WAVES * kRadix; i += kDownThreads) (&s_wave[0][0])[i] = 0;
    // this wave's direct loads have landed; the scan's barrier publishes them
    if (full) __builtin_amdgcn_s_waitcnt(0);
    // global start of this partition's run of digit d
    {
        uint32_t all;
        const uint32_t st = block_excl_scan<WAVES>(tot, s_scan[0], &all);
        if (tid < kRadix) s_global[tid] = st + cnt_dp;
    }
    if (full) {
        const KeyT* sk = reinterpret_cast<const KeyT*>(s_kv) + wave * WAVE_ITEMS;
        const uint32_t* sv = reinterpret_cast<const uint32_t*>(s_kv) + kSortTile + wave * WAVE_ITEMS;
#pragma unroll
        for (int k = 0; k < kDownItems; ++k) {
            const int li = k * 64 + lane;
            key[k] = sk[li];
            val[k] = vals_in ? sv[li] : (uint32_t)wbase + (uint32_t)li;
        }
        __syncthreads();   // the staged input is read before the tables reuse s_kv
    }
    rank_scatter<KeyT, NB>(key, val, lim, drop, shift, s_kv, s_wave, s_local, s_global, s_scan[1],
                           keys_out, vals_out, rects, pairs_out, rects_out, n_rects, ranges, n_tiles,
                           count);
}

// Fused first tile pass: the pairs of each kSortTile partition are
// generated from the item rectangles (as the duplicate does) into LDS
// instead of being written out and read back, then ranked by their first
// tile digit and scattered.  The duplicate has counted that digit per
// chunk (counts[d][2 parts], two chunks per partition) and the rows are
// scanned.  Positions that got no pair hold the key 0xFFFFFFFF and are
// dropped, as the duplicate's counts dropped them.
template <typename KeyT, int NB>
__global__ void __launch_bounds__(kDownThreads)
k_dup_scatter(Workspace ws, int64_t n, KeyT* __restrict__ keys_out, uint32_t* __restrict__ vals_out,
              const uint32_t* __restrict__ counts, const uint32_t* __restrict__ totals,
              int64_t parts, uint32_t* __restrict__ ranges, int64_t n_tiles) {
    constexpr int WAVES = kDownThreads / 64;
    constexpr int WAVE_ITEMS = 64 * kDownItems;
    constexpr int RUN = kDupChunk / kDownThreads;   // pairs per thread per chunk
    static_assert(2 * kDupChunk == kSortTile, "two chunks per partition");
    // the staged (key, value) words; before them, one chunk's items
    constexpr int kItemBytes = 4 * kChunkItems * 4;
    constexpr int kKvBytes = kSortTile * 8;
    __shared__ __align__(16) unsigned char s_raw[kItemBytes > kKvBytes ? kItemBytes : kKvBytes];
    uint64_t* s_kv = reinterpret_cast<uint64_t*>(s_raw);
    uint32_t* s_it = reinterpret_cast<uint32_t*>(s_raw);
    const ChunkItems ci = {s_it, s_it + kChunkItems, s_it + 2 * kChunkItems, s_it + 3 * kChunkItems};
    __shared__ uint32_t s_wave[WAVES][kRadix];
    __shared__ uint32_t s_local[kRadix];
    __shared__ uint32_t s_global[kRadix];
    __shared__ uint32_t s_scan[2][WAVES];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint32_t P = ws.header[kHdrEntries];
    const int64_t Pc = (int64_t)P < ws.capacity ? (int64_t)P : ws.capacity;
    const uint32_t nn = (uint32_t)n;
    const int64_t n_vis = ws.header[kHdrVisible] < ws.n_items ? ws.header[kHdrVisible] : ws.n_items;
    const int64_t p = xcd_part(blockIdx.x, (Pc + kSortTile - 1) / kSortTile);
    const int64_t base = p * kSortTile;
    if (base >= Pc) return;
    constexpr int kLive = 1 << NB;
    const uint32_t tot = tid < kLive ? totals[tid] : 0u;
    const uint32_t cnt_dp = tid < kLive ? counts[((int64_t)tid * parts + p) * 2] : 0u;
    for (int i = tid; i < WAVES * kRadix; i += kDownThreads) (&s_wave[0][0])[i] = 0;

    // the partition's two chunks, RUN consecutive pairs per thread each
    uint32_t tl[2][RUN], vl[2][RUN];
    int got[2] = {0, 0};
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int64_t chunk = 2 * p + h;
        const int64_t p0 = chunk * kDupChunk;
        if (p0 >= Pc) continue;   // uniform
        const int64_t p1 = p0 + kDupChunk < Pc ? p0 + kDupChunk : Pc;
        __syncthreads();   // the item arrays are free
        const int nloc = load_chunk_items(ws, chunk, p1, Pc, n_vis, nn, ci, tid, kDownThreads);
        __syncthreads();
        const int64_t q0 = p0 + (int64_t)tid * RUN;
        if (nloc > 0 && q0 < p1) {
            got[h] = p1 - q0 < RUN ? (int)(p1 - q0) : RUN;
            gen_pairs<RUN>(ci, nloc, q0, got[h], tl[h], vl[h]);
        }
    }
    __syncthreads();   // the item arrays are done: s_kv takes the pairs
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int e = 0; e < RUN; ++e)
            s_kv[h * kDupChunk + tid * RUN + e] =
                e < got[h] ? ((uint64_t)tl[h][e] | ((uint64_t)vl[h][e] << 32)) : 0xFFFFFFFFull;
    // global start of this partition's run of digit d (the barrier also
    // publishes the staged pairs)
    {
        uint32_t all;
        const uint32_t st = block_excl_scan<WAVES>(tot, s_scan[0], &all);
        if (tid < kRadix) s_global[tid] = st + cnt_dp;
    }
    const int64_t left = Pc - (base + (int64_t)wave * WAVE_ITEMS);
    const int lim = left <= 0 ? 0 : (left >= WAVE_ITEMS ? WAVE_ITEMS : (int)left);
    uint32_t key[kDownItems], val[kDownItems];
#pragma unroll
    for (int k = 0; k < kDownItems; ++k) {
        const int li = k * 64 + lane;
        const uint64_t kv = li < lim ? s_kv[wave * WAVE_ITEMS + li] : 0xFFFFFFFFull;
        key[k] = (uint32_t)kv;
        val[k] = (uint32_t)(kv >> 32);
    }
    __syncthreads();   // the pairs are read before the tables reuse s_kv
    rank_scatter<KeyT, NB>(key, val, lim, true, 0, s_kv, s_wave, s_local, s_global, s_scan[1],
                           keys_out, vals_out, nullptr, nullptr, nullptr, 0, ranges, n_tiles, Pc);
}

// Tile boundaries at the start of each (digit, partition) run of the last
// tile pass, where the previous element was written by another block, and
// the end of the last tile.  Block (x, d) checks partitions x * 256 + t.
template <typename KeyT>
__global__ void __launch_bounds__(256)
k_range_edges(const KeyT* __restrict__ keys, const uint32_t* __restrict__ counts,
              const uint32_t* __restrict__ totals, int64_t parts, int cstride,
              const uint32_t* count_ptr, int64_t count_host, uint32_t* __restrict__ ranges,
              int64_t n_tiles) {
    __shared__ uint32_t s_part[256 / 64];
    const int d = blockIdx.y;
    // start of digit d: the totals of the digits below it, summed by the
    // block (one total per thread, a wave reduction, then the wave sums)
    {
        uint32_t t = (int)threadIdx.x < d ? totals[threadIdx.x] : 0u;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) t += __shfl_down(t, off, 64);
        if ((threadIdx.x & 63) == 0) s_part[threadIdx.x >> 6] = t;
    }
    __syncthreads();
    const uint32_t s_base = s_part[0] + s_part[1] + s_part[2] + s_part[3];
    const int64_t count = pass_count(count_ptr, count_host);
    // the partitions holding the pass's items (the row scans leave the
    // others untouched)
    const int64_t lp = (count + kSortTile - 1) / kSortTile;
    const int64_t live = lp < parts ? lp : parts;
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p < live) {
        const uint32_t off = counts[((int64_t)d * parts + p) * cstride];
        const uint32_t next =
            p + 1 < live ? counts[((int64_t)d * parts + p + 1) * cstride] : totals[d];
        const int64_t at = (int64_t)s_base + off;
        if (next > off && at > 0 && at < count) {
            const uint32_t a = keys[at - 1], b = keys[at];
            if (a != b) {
                if (b < (uint64_t)n_tiles) ranges[2 * (int64_t)b] = (uint32_t)at;
                if (a < (uint64_t)n_tiles) ranges[2 * (int64_t)a + 1] = (uint32_t)at;
            }
        }
    }
    if (blockIdx.x == 0 && d == 0 && threadIdx.x == 0 && count > 0) {
        const uint32_t last = keys[count - 1];
        if (last < (uint64_t)n_tiles) ranges[2 * (int64_t)last + 1] = (uint32_t)count;
    }
}

template <typename KeyT, int NB>
static void downsweep_t(dim3 grid, hipStream_t s, const KeyT* keys_in, const uint32_t* vals_in,
                        KeyT* keys_out, uint32_t* vals_out, const uint32_t* count_ptr,
                        int64_t count_host, int shift, const uint32_t* counts,
                        const uint32_t* totals, int64_t parts, const uint64_t* rects,
                        uint32_t* pairs_out, uint64_t* rects_out, int64_t n_rects, bool drop,
                        int cstride, uint32_t* ranges, int64_t n_tiles) {
    hipLaunchKernelGGL((k_downsweep<KeyT, NB>), grid, dim3(kDownThreads), 0, s, keys_in, vals_in,
                       keys_out, vals_out, count_ptr, count_host, shift, counts, totals, parts,
                       rects, pairs_out, rects_out, n_rects, drop, cstride, ranges, n_tiles);
}

template <typename KeyT>
static void radix_pass_t(const KeyT* keys_in, const uint32_t* vals_in, KeyT* keys_out,
                         uint32_t* vals_out, const uint32_t* count_ptr, int64_t count_host, int shift,
                         uint32_t* counts, uint32_t* totals, int64_t parts, const uint64_t* rects,
                         uint32_t* pairs_out, uint64_t* rects_out, int64_t n_rects,
                         bool drop_culled, uint32_t* kept_out, int digit_bits, bool counted,
                         uint32_t* ranges, int64_t n_tiles, hipStream_t s) {
    if (parts <= 0) return;
    // counted: the digit counts of every half partition are already in
    // counts[d][2 parts] (written by the pass's producer)
    const int cstride = counted ? 2 : 1;
    const int bits = digit_bits < 1 ? 1 : (digit_bits > kRadixBits ? kRadixBits : digit_bits);
    if (!counted) {
        const dim3 ug((unsigned)parts), ub(kSortThreads);
        hipLaunchKernelGGL(k_upsweep<KeyT>, ug, ub, 0, s, keys_in, count_ptr, count_host, shift,
                           counts, parts, drop_culled, bits);
    }
    hipLaunchKernelGGL(k_scan_rows, dim3(1u << bits), dim3(kScanRowThreads), 0, s, counts,
                       parts * cstride, totals, drop_culled ? kept_out : nullptr, count_ptr,
                       count_host, kSortTile / cstride);
    const dim3 g((unsigned)parts);
#define SGS_DOWNSWEEP(NB)                                                                      \
    downsweep_t<KeyT, NB>(g, s, keys_in, vals_in, keys_out, vals_out, count_ptr, count_host,   \
                          shift, counts, totals, parts, rects, pairs_out, rects_out, n_rects,    \
                          drop_culled, cstride, ranges, n_tiles)
    switch (bits) {
        case 1: SGS_DOWNSWEEP(1); break;
        case 2: SGS_DOWNSWEEP(2); break;
        case 3: SGS_DOWNSWEEP(3); break;
        case 4: SGS_DOWNSWEEP(4); break;
        case 5: SGS_DOWNSWEEP(5); break;
        case 6: SGS_DOWNSWEEP(6); break;
        case 7: SGS_DOWNSWEEP(7); break;
        default: SGS_DOWNSWEEP(8); break;
    }
#undef SGS_DOWNSWEEP
    if (ranges) {
        // the pass's output keys are sorted; its counts hold each partition's
        // exclusive offset within its digit (the key has digit_bits bits here)
        const int digits = 1 << bits;
        const dim3 eg((unsigned)((parts + 255) / 256), (unsigned)digits);
        hipLaunchKernelGGL(k_range_edges<KeyT>, eg, dim3(256), 0, s, keys_out, counts, totals, parts,
                           cstride, count_ptr, count_host, ranges, n_tiles);
    }
}

void launch_radix_pass(const uint32_t* keys_in, const uint32_t* vals_in, uint32_t* keys_out,
                       uint32_t* vals_out, const uint32_t* count_ptr, int64_t count_host, int shift,
                       uint32_t* counts, uint32_t* totals, int64_t parts, const uint64_t* rects,
                       uint32_t* pairs_out, uint64_t* rects_out, int64_t n_rects, bool drop_culled,
                       uint32_t* kept_out, hipStream_t s, int digit_bits, bool counted,
                       uint32_t* ranges, int64_t n_tiles) {
    radix_pass_t<uint32_t>(keys_in, vals_in, keys_out, vals_out, count_ptr, count_host, shift, counts,
                           totals, parts, rects, pairs_out, rects_out, n_rects, drop_culled,
                           kept_out, digit_bits, counted, ranges, n_tiles, s);
}

void launch_radix_pass16(const uint16_t* keys_in, const uint32_t* vals_in, uint16_t* keys_out,
                         uint32_t* vals_out, const uint32_t* count_ptr, int64_t count_host, int shift,
                         uint32_t* counts, uint32_t* totals, int64_t parts, hipStream_t s,
                         int digit_bits, bool counted, uint32_t* ranges, int64_t n_tiles) {
    radix_pass_t<uint16_t>(keys_in, vals_in, keys_out, vals_out, count_ptr, count_host, shift, counts,
                           totals, parts, nullptr, nullptr, nullptr, 0, false, nullptr, digit_bits, counted,
                           ranges, n_tiles, s);
}

template <typename KeyT>
static void dup_scatter_t(const Workspace& ws, int64_t n, KeyT* keys_out, uint32_t* vals_out,
                          int64_t parts, int digit_bits, uint32_t* ranges, int64_t pair_capacity,
                          hipStream_t s) {
    if (parts <= 0) return;
    const int bits = digit_bits < 1 ? 1 : (digit_bits > kRadixBits ? kRadixBits : digit_bits);
    hipLaunchKernelGGL(k_scan_rows, dim3(1u << bits), dim3(kScanRowThreads), 0, s, ws.counts,
                       parts * 2, ws.totals, nullptr, ws.header + kHdrEntries, pair_capacity, kDupChunk);
    const dim3 g((unsigned)parts), b(kDownThreads);
#define SGS_DUPSCAT(NB)                                                                        \
    hipLaunchKernelGGL((k_dup_scatter<KeyT, NB>), g, b, 0, s, ws, n, keys_out, vals_out,      \
                       ws.counts, ws.totals, parts, ranges, ws.n_strips)
    switch (bits) {
        case 1: SGS_DUPSCAT(1); break;
        case 2: SGS_DUPSCAT(2); break;
        case 3: SGS_DUPSCAT(3); break;
        case 4: SGS_DUPSCAT(4); break;
        case 5: SGS_DUPSCAT(5); break;
        case 6: SGS_DUPSCAT(6); break;
        case 7: SGS_DUPSCAT(7); break;
        default: SGS_DUPSCAT(8); break;
    }
#undef SGS_DUPSCAT
    if (ranges) {
        const dim3 eg((unsigned)((parts + 255) / 256), 1u << bits);
        hipLaunchKernelGGL(k_range_edges<KeyT>, eg, dim3(256), 0, s, keys_out, ws.counts, ws.totals,
                           parts, 2, ws.header + kHdrEntries, pair_capacity, ranges, ws.n_strips);
    }
}

void launch_dup_scatter(const Workspace& ws, int64_t n, uint32_t* keys_out, uint32_t* vals_out,
                        int64_t parts, int digit_bits, uint32_t* ranges, int64_t pair_capacity,
                        hipStream_t s) {
    if (ws.key16)
        dup_scatter_t<uint16_t>(ws, n, reinterpret_cast<uint16_t*>(keys_out), vals_out, parts,
                                digit_bits, ranges, pair_capacity, s);
    else
        dup_scatter_t<uint32_t>(ws, n, keys_out, vals_out, parts, digit_bits, ranges, pair_capacity, s);
}

// ---------------------------------------------------------------------------
// exclusive scan of the per-item entry counts (in depth order) -> entry
// offsets; the (tile, item) pairs of the same items are summed beside it
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint64_t block_sum_u64(uint64_t v, uint64_t* s) {
    const int tid = threadIdx.x;
    s[tid] = v;
    __syncthreads();
    for (int off = blockDim.x / 2; off > 0; off >>= 1) {
        if (tid < off) s[tid] += s[tid + off];
        __syncthreads();
    }
    const uint64_t r = s[0];
    __syncthreads();
    return r;
}

// block sums of the entry counts in block_sums[b] and of the pairs of the
// same items (from their tile rectangles) in block_sums[nb + b]
__global__ void __launch_bounds__(kScanThreads)
k_scan_reduce(const uint32_t* __restrict__ in, const uint64_t* __restrict__ rects,
              const uint32_t* n_ptr, int64_t n_max, uint64_t* __restrict__ block_sums) {
    __shared__ uint64_t s[kScanThreads];
    const int64_t n = pass_count(n_ptr, n_max);
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    uint64_t run = 0, pairs = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        const int64_t i = base + (int64_t)k * kScanThreads + threadIdx.x;
        if (i < n) {
            run += in[i];
            pairs += rect_pairs(rects[i]);
        }
    }
    const uint64_t tot = block_sum_u64(run, s);
    const uint64_t ptot = block_sum_u64(pairs, s);
    if (threadIdx.x == 0) {
        block_sums[blockIdx.x] = tot;
        block_sums[gridDim.x + blockIdx.x] = ptot;
    }
}

// one block: exclusive scan of the entry block sums; E = their total, P =
// the pairs' total, capacity flag when P exceeds the capacity
__global__ void __launch_bounds__(1024)
k_scan_sums(uint64_t* __restrict__ block_sums, int64_t nb, uint32_t* header, int64_t capacity,
            uint32_t* pair_offsets) {
    __shared__ uint64_t s[1024];
    const int tid = threadIdx.x;
    uint64_t carry = 0, pairs = 0;
    for (int64_t b0 = 0; b0 < nb; b0 += 1024) {
        const int64_t i = b0 + tid;
        const uint64_t v = i < nb ? block_sums[i] : 0ull;
        pairs += i < nb ? block_sums[nb + i] : 0ull;
        s[tid] = v;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            const uint64_t t = tid >= off ? s[tid - off] : 0ull;
            __syncthreads();
            s[tid] += t;
            __syncthreads();
        }
        if (i < nb) block_sums[i] = carry + s[tid] - v;
        carry += s[1023];
        __syncthreads();
    }
    const uint64_t P = block_sum_u64(pairs, s);
    if (tid == 0) {
        header[kHdrEntries] = (uint32_t)(carry < 0xFFFFFFFFull ? carry : 0xFFFFFFFFull);
        header[kHdrPairs] = (uint32_t)(P < 0xFFFFFFFFull ? P : 0xFFFFFFFFull);
        pair_offsets[header[kHdrVisible]] = header[kHdrEntries];
        if (P > (uint64_t)capacity) atomicOr(&header[kHdrStatus], SGS_STATUS_CAPACITY);
    }
}

// block-local scan + block offset; marks the first item of every duplicate chunk
__global__ void __launch_bounds__(kScanThreads)
k_scan_final(const uint32_t* __restrict__ in, const uint32_t* n_ptr, int64_t n_max,
             const uint64_t* __restrict__ block_sums, uint32_t* __restrict__ out,
             uint32_t* __restrict__ chunk_start, int64_t dup_chunks, int64_t capacity) {
    __shared__ uint32_t s_w[kScanThreads / 64];
    const int64_t n = pass_count(n_ptr, n_max);
    if ((int64_t)blockIdx.x * kScanTile >= n) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    // thread owns kScanItems consecutive items
    uint32_t v[kScanItems], run = 0;
    const int64_t t0 = base + (int64_t)tid * kScanItems;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        v[k] = (t0 + k < n) ? in[t0 + k] : 0u;
        run += v[k];
    }
    uint32_t incl = run;
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t t = __shfl_up(incl, off, 64);
        if (lane >= off) incl += t;
    }
    if (lane == 63) s_w[wave] = incl;
    __syncthreads();
    uint64_t wex = 0;
    for (int w = 0; w < wave; ++w) wex += s_w[w];
    uint64_t off = block_sums[blockIdx.x] + wex + (incl - run);
    const uint64_t cap = (uint64_t)capacity;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        const int64_t i = t0 + k;
        if (i < n) {
            out[i] = (uint32_t)(off < 0xFFFFFFFFull ? off : 0xFFFFFFFFull);
            if (v[k] > 0 && off < cap) {
                uint64_t c = (off + kDupChunk - 1) / kDupChunk;
                for (; c * kDupChunk < off + v[k] && (int64_t)c < dup_chunks; ++c)
                    chunk_start[c] = (uint32_t)i;
            }
            off += v[k];
        }
    }
}

void launch_scan_pairs(const Workspace& ws, hipStream_t s) {
    const int64_t n = ws.n_items;
    const int64_t nb = (n + kScanTile - 1) / kScanTile;
    if (nb <= 0) return;
    const uint32_t* nv = ws.header + kHdrVisible;
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(kScanThreads), 0, s, ws.pair_counts,
                       ws.sorted_rects, nv, n, ws.scan_sums);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(1024), 0, s, ws.scan_sums, nb, ws.header,
                       ws.capacity, ws.pair_offsets);
    hipLaunchKernelGGL(k_scan_final, dim3((unsigned)nb), dim3(kScanThreads), 0, s, ws.pair_counts,
                       nv, n, ws.scan_sums, ws.pair_offsets, ws.chunk_start, ws.dup_chunks,
                       ws.capacity);
}

}  // namespace sgs
