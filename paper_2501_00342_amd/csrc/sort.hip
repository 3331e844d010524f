// Binning and sorting of (tile, depth) pairs.
//
// The pairs must come out in ascending key order, key = (tile << 32) |
// bits(float32 depth), ties by Gaussian index (the order a stable sort of
// index-ordered emission gives).  Instead of a radix sort over the whole
// 64-bit key, the work is split in two stable radix sorts that give the
// same order:
//   1. the (camera, Gaussian) items are sorted by their 32-bit depth key
//      (four 8-bit passes over n_items, values = item index);
//   2. pairs are emitted item by item in that order (each item's tiles
//      row-major) and stably partitioned by tile id (ceil(bits/8) passes).
// A stable partition of a depth-ordered sequence is ordered by (tile,
// depth, item).  Every pass is one LDS-staged "onesweep" kernel: a block
// takes a partition ticket, ranks its keys in LDS with wave ballots,
// publishes per-digit counts, resolves its global digit offsets by
// decoupled look-back over earlier partitions, and writes its keys out in
// digit order from LDS so that the stores of each digit run are contiguous.
#include "common.hpp"

namespace sgs {

constexpr uint32_t kFlagAgg = 1u << 30;
constexpr uint32_t kFlagInc = 2u << 30;
constexpr uint32_t kValMask = (1u << 30) - 1;

__device__ __forceinline__ uint32_t ld_acquire_dev(const uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_release_dev(uint32_t* p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// --------------------------------------------------------------------------
// fill / clear / setup
// --------------------------------------------------------------------------

__global__ void k_fill_u32(uint32_t* p, uint32_t v, int64_t count) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

void launch_fill_u32(uint32_t* p, uint32_t v, int64_t count, hipStream_t s) {
    if (count <= 0) return;
    int64_t blocks = (count + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, s, p, v, count);
}

void launch_clear(const Workspace& ws, hipStream_t s) {
    launch_fill_u32(ws.header, 0u, kHdrWords, s);
    launch_fill_u32(ws.lookback, 0u, ws.lookback_pass_words * (kDepthPasses + ws.tile_passes), s);
    launch_fill_u32(reinterpret_cast<uint32_t*>(ws.scan_lookback), 0u, 2 * ws.scan_parts, s);
    launch_fill_u32(ws.ranges, 0u, 2 * ws.n_tiles, s);
}

__global__ void k_setup(Workspace ws, const sgs_camera* __restrict__ cams, int n_cams, int tw,
                        int th) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int64_t tiles = 0, pix = 0;
    bool ok = true;
    for (int c = 0; c < n_cams; ++c) {
        CamTable t;
        t.W = cams[c].width;
        t.H = cams[c].height;
        ok = ok && t.W > 0 && t.H > 0 && t.W <= SGS_MAX_IMAGE_SIDE && t.H <= SGS_MAX_IMAGE_SIDE;
        t.GX = ok ? (t.W + tw - 1) / tw : 0;
        t.GY = ok ? (t.H + th - 1) / th : 0;
        t.tile_base = (int32_t)tiles;
        t.pad = 0;
        t.pix_base = pix;
        ws.cams[c] = t;
        tiles += (int64_t)t.GX * t.GY;
        pix += (int64_t)t.W * t.H;
    }
    // the device cameras must describe the sizes the host planned for
    if (!ok || pix != ws.n_pixels || tiles != ws.n_tiles)
        atomicOr(&ws.header[kHdrStatus], SGS_STATUS_CAMERAS);
}

void launch_setup(const Workspace& ws, const sgs_camera* dev_cams, int n_cams, int tile_w, int tile_h,
                  hipStream_t s) {
    hipLaunchKernelGGL(k_setup, dim3(1), dim3(64), 0, s, ws, dev_cams, n_cams, tile_w, tile_h);
}

// --------------------------------------------------------------------------
// digit histograms: sum the per-block partial rows, exclusive scan per pass
// --------------------------------------------------------------------------

// level 1: block (pass, f) sums rows f, f + kHistFold, ... of one pass
__global__ void __launch_bounds__(kRadix)
k_hist_fold(const uint32_t* __restrict__ partial, int passes, int rows, uint32_t* fold) {
    const int pass = blockIdx.x / kHistFold;
    const int f = blockIdx.x % kHistFold;
    const int d = threadIdx.x;
    uint32_t sum = 0;
    for (int r = f; r < rows; r += kHistFold) sum += partial[((int64_t)r * passes + pass) * kRadix + d];
    fold[((int64_t)f * passes + pass) * kRadix + d] = sum;
}

// level 2: one block per pass sums the folded rows and scans the 256 digits
__global__ void __launch_bounds__(kRadix)
k_hist_scan(const uint32_t* __restrict__ fold, int passes, uint32_t* digit_offsets) {
    const int pass = blockIdx.x;
    const int d = threadIdx.x;
    uint32_t sum = 0;
    for (int f = 0; f < kHistFold; ++f) sum += fold[((int64_t)f * passes + pass) * kRadix + d];
    __shared__ uint32_t s[kRadix];
    s[d] = sum;
    __syncthreads();
    for (int off = 1; off < kRadix; off <<= 1) {
        const uint32_t v = d >= off ? s[d - off] : 0u;
        __syncthreads();
        s[d] += v;
        __syncthreads();
    }
    digit_offsets[pass * kRadix + d] = s[d] - sum;
}

void launch_hist_scan(const Workspace& ws, int passes, int digit_row0, int hist_rows, hipStream_t s) {
    hipLaunchKernelGGL(k_hist_fold, dim3(passes * kHistFold), dim3(kRadix), 0, s, ws.hist_partial,
                       passes, hist_rows, ws.hist_fold);
    hipLaunchKernelGGL(k_hist_scan, dim3(passes), dim3(kRadix), 0, s, ws.hist_fold, passes,
                       ws.digit_offsets + digit_row0 * kRadix);
}

// --------------------------------------------------------------------------
// onesweep pass
// --------------------------------------------------------------------------

__global__ void __launch_bounds__(kSortThreads)
k_onesweep(const uint32_t* __restrict__ keys_in, const uint32_t* __restrict__ vals_in,
           uint32_t* __restrict__ keys_out, uint32_t* __restrict__ vals_out,
           const uint32_t* count_ptr, int64_t count_host, int shift,
           const uint32_t* __restrict__ digit_offsets, uint32_t* lookback, uint32_t* ticket) {
    constexpr int WAVES = kSortThreads / 64;
    constexpr int WAVE_ITEMS = 64 * kSortItems;
    __shared__ uint32_t s_keys[kSortTile];
    __shared__ uint32_t s_vals[kSortTile];
    __shared__ uint32_t s_wave[WAVES][kRadix];    // per-wave digit counts -> offsets
    __shared__ uint32_t s_local[kRadix];          // block-local exclusive digit start
    __shared__ uint32_t s_global[kRadix];         // global start of this block's digit run
    __shared__ uint32_t s_part;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    if (tid == 0) s_part = atomicAdd(ticket, 1u);
    for (int i = tid; i < WAVES * kRadix; i += kSortThreads) (&s_wave[0][0])[i] = 0;
    __syncthreads();
    const int64_t part = s_part;
    int64_t count = count_host;
    if (count_ptr && (int64_t)*count_ptr < count) count = *count_ptr;
    const int64_t base = part * kSortTile;
    if (base >= count) return;   // every later ticket is beyond the count too

    // load: wave w owns items [base + w*WAVE_ITEMS, +WAVE_ITEMS); round k = 64 items
    uint32_t key[kSortItems], val[kSortItems];
    uint16_t rank[kSortItems];
    const int64_t wbase = base + (int64_t)wave * WAVE_ITEMS;
#pragma unroll
    for (int k = 0; k < kSortItems; ++k) {
        const int64_t i = wbase + k * 64 + lane;
        if (i < count) {
            key[k] = keys_in[i];
            val[k] = vals_in ? vals_in[i] : (uint32_t)i;
        } else {
            key[k] = 0xFFFFFFFFu;
            val[k] = 0;
        }
    }
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    // stable ranking inside each wave, round by round
#pragma unroll
    for (int k = 0; k < kSortItems; ++k) {
        const int64_t i = wbase + k * 64 + lane;
        const bool valid = i < count;
        const uint32_t d = (key[k] >> shift) & (kRadix - 1);
        uint64_t m = __ballot(valid);
#pragma unroll
        for (int b = 0; b < kRadixBits; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t bb = __ballot(bit);
            m &= bit ? bb : ~bb;
        }
        const uint64_t lower = m & lt_mask;
        const uint32_t prior = valid ? s_wave[wave][d] : 0u;
        rank[k] = (uint16_t)(prior + __popcll(lower));
        if (valid && lower == 0) s_wave[wave][d] = prior + (uint32_t)__popcll(m);
        // the leader's store must land before the next round's loads
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();

    // per digit: block count, per-wave exclusive offsets
    const int d = tid;  // kSortThreads == kRadix
    uint32_t total = 0;
#pragma unroll
    for (int w = 0; w < WAVES; ++w) {
        const uint32_t c = s_wave[w][d];
        s_wave[w][d] = total;
        total += c;
    }
    // publish, then look back over earlier partitions
    uint32_t* my = lookback + part * kRadix;
    if (part == 0) {
        st_release_dev(my + d, kFlagInc | total);
    } else {
        st_release_dev(my + d, kFlagAgg | total);
    }
    uint32_t prefix = 0;
    if (part > 0) {
        int64_t p = part - 1;
        while (true) {
            const uint32_t v = ld_acquire_dev(lookback + p * kRadix + d);
            const uint32_t flag = v & ~kValMask;
            if (flag == 0u) {
                __builtin_amdgcn_s_sleep(1);
                continue;
            }
            prefix += v & kValMask;
            if (flag == kFlagInc) break;
            --p;
        }
        st_release_dev(my + d, kFlagInc | (prefix + total));
    }
    s_global[d] = digit_offsets[d] + prefix;
    // block-local exclusive scan of the digit totals
    s_local[d] = total;
    __syncthreads();
    for (int off = 1; off < kRadix; off <<= 1) {
        const uint32_t v = d >= off ? s_local[d - off] : 0u;
        __syncthreads();
        s_local[d] += v;
        __syncthreads();
    }
    s_local[d] -= total;
    __syncthreads();

    // stage in LDS in digit order
    int n_valid = 0;
#pragma unroll
    for (int k = 0; k < kSortItems; ++k) {
        const int64_t i = wbase + k * 64 + lane;
        if (i < count) {
            const uint32_t dd = (key[k] >> shift) & (kRadix - 1);
            const uint32_t pos = s_local[dd] + s_wave[wave][dd] + rank[k];
            s_keys[pos] = key[k];
            s_vals[pos] = val[k];
        }
    }
    __syncthreads();
    const int64_t rem = count - base;
    n_valid = (int)(rem < kSortTile ? rem : kSortTile);
    for (int i = tid; i < n_valid; i += kSortThreads) {
        const uint32_t k = s_keys[i];
        const uint32_t dd = (k >> shift) & (kRadix - 1);
        const uint32_t out = s_global[dd] + (uint32_t)(i - (int)s_local[dd]);
        if (keys_out) keys_out[out] = k;
        vals_out[out] = s_vals[i];
    }
}

void launch_onesweep(const uint32_t* keys_in, const uint32_t* vals_in, uint32_t* keys_out,
                     uint32_t* vals_out, const uint32_t* count_ptr, int64_t count_host,
                     int shift, const uint32_t* digit_offsets, uint32_t* lookback,
                     uint32_t* ticket, int64_t parts, hipStream_t s) {
    if (parts <= 0) return;
    hipLaunchKernelGGL(k_onesweep, dim3((unsigned)parts), dim3(kSortThreads), 0, s, keys_in,
                       vals_in, keys_out, vals_out, count_ptr, count_host, shift, digit_offsets,
                       lookback, ticket);
}

// --------------------------------------------------------------------------
// exclusive scan of pair counts in depth order (decoupled look-back)
// --------------------------------------------------------------------------

__device__ __forceinline__ uint32_t rect_pairs(uint64_t r) {
    const int tx0 = (int)(r & 0xFFFF), tx1 = (int)((r >> 16) & 0xFFFF);
    const int ty0 = (int)((r >> 32) & 0xFFFF), ty1 = (int)((r >> 48) & 0xFFFF);
    const int w = tx1 - tx0 + 1, h = ty1 - ty0 + 1;
    return (w > 0 && h > 0) ? (uint32_t)(w * h) : 0u;
}

constexpr uint64_t kFlagAgg64 = 1ull << 62;
constexpr uint64_t kFlagInc64 = 2ull << 62;
constexpr uint64_t kValMask64 = (1ull << 62) - 1;

__global__ void __launch_bounds__(kScanThreads)
k_scan_pairs(Workspace ws) {
    __shared__ uint32_t s_wsum[kScanThreads / 64];
    __shared__ uint64_t s_prefix;
    __shared__ uint32_t s_part;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (tid == 0) s_part = atomicAdd(&ws.header[kHdrTicketBase + kTicketScan], 1u);
    __syncthreads();
    const int64_t part = s_part;
    const int64_t n = ws.n_items;
    const int64_t base = part * kScanTile;
    if (base >= n) return;
    // thread owns kScanItems consecutive items (<= 16 * 2^26 pairs: no u32 overflow)
    uint32_t cnt[kScanItems];
    uint32_t run = 0;
    const int64_t t0 = base + (int64_t)tid * kScanItems;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        const int64_t i = t0 + k;
        uint32_t c = 0;
        if (i < n) {
            const uint32_t item = ws.sorted_items[i];
            c = item < (uint64_t)n ? rect_pairs(ws.tile_rects[item]) : 0u;
        }
        cnt[k] = c;
        run += c;
    }
    uint32_t incl = run;
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t v = __shfl_up(incl, off, 64);
        if (lane >= off) incl += v;
    }
    if (lane == 63) s_wsum[wave] = incl;
    __syncthreads();
    uint64_t wexcl = 0, btotal = 0;
    for (int w = 0; w < kScanThreads / 64; ++w) {
        if (w < wave) wexcl += s_wsum[w];
        btotal += s_wsum[w];
    }
    if (tid == 0) {
        uint64_t* lb = ws.scan_lookback;
        if (part == 0) {
            __hip_atomic_store(lb, kFlagInc64 | btotal, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            s_prefix = 0;
        } else {
            __hip_atomic_store(lb + part, kFlagAgg64 | btotal, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            uint64_t prefix = 0;
            int64_t p = part - 1;
            while (true) {
                const uint64_t v = __hip_atomic_load(lb + p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                const uint64_t flag = v & ~kValMask64;
                if (flag == 0u) {
                    __builtin_amdgcn_s_sleep(1);
                    continue;
                }
                prefix += v & kValMask64;
                if (flag == kFlagInc64) break;
                --p;
            }
            __hip_atomic_store(lb + part, kFlagInc64 | (prefix + btotal), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
            s_prefix = prefix;
        }
    }
    __syncthreads();
    uint64_t off = s_prefix + wexcl + incl - run;
    const uint64_t cap = (uint64_t)ws.capacity;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        const int64_t i = t0 + k;
        if (i < n) {
            ws.pair_offsets[i] = (uint32_t)(off < 0xFFFFFFFFull ? off : 0xFFFFFFFFull);
            // mark every duplicate chunk that starts inside this item's pairs
            if (cnt[k] > 0 && off < cap) {
                uint64_t c = (off + kDupChunk - 1) / kDupChunk;
                for (; c * kDupChunk < off + cnt[k] && (int64_t)c < ws.dup_chunks; ++c)
                    ws.chunk_start[c] = (uint32_t)i;
            }
            off += cnt[k];
            if (i == n - 1) {
                ws.pair_offsets[n] = (uint32_t)(off < 0xFFFFFFFFull ? off : 0xFFFFFFFFull);
                ws.header[kHdrPairs] = (uint32_t)(off < 0xFFFFFFFFull ? off : 0xFFFFFFFFull);
                if (off > cap) atomicOr(&ws.header[kHdrStatus], SGS_STATUS_CAPACITY);
            }
        }
    }
}

void launch_scan_pairs(const Workspace& ws, hipStream_t s) {
    hipLaunchKernelGGL(k_scan_pairs, dim3((unsigned)ws.scan_parts), dim3(kScanThreads), 0, s, ws);
}

// --------------------------------------------------------------------------
// duplicate: one block per 4096-pair chunk, one thread per pair (balanced)
// --------------------------------------------------------------------------

__global__ void __launch_bounds__(256)
k_duplicate(Workspace ws, int64_t n, int tile_passes) {
    __shared__ uint32_t s_off[kDupChunk + 1];
    __shared__ uint32_t s_origin[kDupChunk + 1];   // global tile id of the rectangle origin
    __shared__ uint32_t s_wgx[kDupChunk + 1];      // width | GX << 16
    __shared__ uint32_t s_item[kDupChunk + 1];
    __shared__ uint32_t hist[kMaxTilePasses][kRadix];
    const int tid = threadIdx.x;
    for (int i = tid; i < kMaxTilePasses * kRadix; i += 256) (&hist[0][0])[i] = 0;
    const uint32_t P = ws.header[kHdrPairs];
    const int64_t Pc = (int64_t)P < ws.capacity ? (int64_t)P : ws.capacity;
    const uint32_t nn = (uint32_t)n;
    for (int64_t chunk = blockIdx.x; chunk * kDupChunk < Pc; chunk += gridDim.x) {
        const int64_t p0 = chunk * kDupChunk;
        const int64_t p1 = (p0 + kDupChunk < Pc) ? p0 + kDupChunk : Pc;
        const int64_t i0 = ws.chunk_start[chunk];
        if (i0 >= ws.n_items) continue;   // uniform: no chunk start was recorded
        // items i0 .. cover [p0, p1); each has >= 1 pair until the culled tail
        int64_t i_end = ws.n_items;
        if (chunk + 1 < ws.dup_chunks && p1 < Pc) i_end = (int64_t)ws.chunk_start[chunk + 1] + 1;
        int64_t nloc = i_end - i0;
        if (nloc > kDupChunk + 1) nloc = kDupChunk + 1;
        if (nloc < 1) continue;
        __syncthreads();   // previous chunk done with LDS
        for (int j = tid; j < nloc; j += 256) {
            const int64_t i = i0 + j;
            uint32_t item = ws.sorted_items[i];
            if (item >= (uint64_t)ws.n_items) item = 0;
            s_off[j] = ws.pair_offsets[i];
            s_item[j] = item;
            const uint64_t r = ws.tile_rects[item];
            const int tx0 = (int)(r & 0xFFFF), tx1 = (int)((r >> 16) & 0xFFFF);
            const int ty0 = (int)((r >> 32) & 0xFFFF);
            const CamTable ct = ws.cams[item / nn];
            s_origin[j] = (uint32_t)(ct.tile_base + ty0 * ct.GX + tx0);
            s_wgx[j] = (uint32_t)(tx1 - tx0 + 1) | ((uint32_t)ct.GX << 16);
        }
        __syncthreads();
        for (int64_t p = p0 + tid; p < p1; p += 256) {
            int lo = 0, hi = (int)nloc - 1;     // last local item with offset <= p
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if ((int64_t)s_off[mid] <= p) lo = mid; else hi = mid - 1;
            }
            const uint32_t wgx = s_wgx[lo];
            const int w = (int)(wgx & 0xFFFF), gx = (int)(wgx >> 16);
            const int j = (int)(p - s_off[lo]);
            // j / w in float: the quotient is at least 0.5/w from an integer
            int ty = (int)(((float)j + 0.5f) * (1.0f / (float)w));
            int tx = j - ty * w;
            if (tx < 0) { --ty; tx += w; } else if (tx >= w) { ++ty; tx -= w; }
            const uint32_t tile = s_origin[lo] + (uint32_t)(ty * gx + tx);
            ws.pair_tiles[p] = tile;
            ws.pair_values[p] = s_item[lo];
            for (int ps = 0; ps < tile_passes; ++ps)
                atomicAdd(&hist[ps][(tile >> (ps * kRadixBits)) & (kRadix - 1)], 1u);
        }
    }
    __syncthreads();
    uint32_t* row = ws.hist_partial + (int64_t)blockIdx.x * tile_passes * kRadix;
    for (int i = tid; i < tile_passes * kRadix; i += 256) row[i] = (&hist[0][0])[i];
}

void launch_duplicate(const Workspace& ws, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_duplicate, dim3((unsigned)ws.dup_blocks), dim3(256), 0, s, ws, n,
                       ws.tile_passes);
}

// --------------------------------------------------------------------------
// tile ranges from the sorted tile ids
// --------------------------------------------------------------------------

__global__ void k_ranges(Workspace ws) {
    const uint32_t P = ws.header[kHdrPairs];
    const int64_t Pc = (int64_t)P < ws.capacity ? (int64_t)P : ws.capacity;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < Pc;
         i += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t t = ws.pair_tiles[i];
        if ((int64_t)t >= ws.n_tiles) continue;
        if (i == 0 || ws.pair_tiles[i - 1] != t) ws.ranges[2 * (int64_t)t] = (uint32_t)i;
        if (i == Pc - 1 || ws.pair_tiles[i + 1] != t) ws.ranges[2 * (int64_t)t + 1] = (uint32_t)(i + 1);
    }
}

void launch_ranges(const Workspace& ws, hipStream_t s) {
    int64_t blocks = (ws.capacity + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_ranges, dim3((unsigned)blocks), dim3(256), 0, s, ws);
}

// --------------------------------------------------------------------------
// sorted 64-bit keys for inspection
// --------------------------------------------------------------------------

__global__ void k_read_keys(Workspace ws, int64_t count, uint64_t* keys) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t item = ws.pair_values[i];
        const uint32_t dk = item < (uint64_t)ws.n_items ? ws.depth_keys[item] : 0xFFFFFFFFu;
        keys[i] = ((uint64_t)ws.pair_tiles[i] << 32) | dk;
    }
}

void launch_read_keys(const Workspace& ws, int64_t count, uint64_t* keys, hipStream_t s) {
    if (count <= 0) return;
    int64_t blocks = (count + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_read_keys, dim3((unsigned)blocks), dim3(256), 0, s, ws, count, keys);
}

}  // namespace sgs
