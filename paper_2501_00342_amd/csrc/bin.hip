// Second binning level: strip entries -> (tile, item) pairs in key order.
//
// After the first level the (strip, item) entries are grouped by strip, in
// ascending strip id, and within a strip in depth order; each entry's value
// is its item's position in the depth order (sorted_items, sorted_rects).
// A strip is the run of tiles x0 .. x0 + SW - 1 (SW <= kStripTiles) of one
// tile row; the entry of an item with tile columns tx0 .. tx1 covers the
// strip's tiles max(tx0, x0) .. min(tx1, x0 + SW - 1).  A tile's pairs are
// the entries covering it, in entry order, so writing them in that order
// gives the order of a stable sort on (tile << 32 | depth) keys.
//
// Each strip's entries are cut in chunks of kBinChunk, each of kBinSubs
// sub-chunks of kBinSub:
//   k_bin_chunks   one block: the chunk table (per strip its first chunk and
//                  chunk count, per chunk its entry range and the strip's
//                  first tile, width and first column)
//   k_bin_count    one wave per sub-chunk: how many of its entries cover
//                  each tile of the strip (difference array over the tiles)
//   k_bin_strips   per strip: for each tile, the counts of the strip's
//                  earlier sub-chunks (exclusive sums), and each tile's total
//   k_bin_tiles    one block: exclusive scan of the tile totals over all
//                  tiles -> first position of each tile, and the ranges
//   k_bin_scatter  one workgroup per chunk, wave w taking sub-chunk w, lane
//                  t holding tile t of the strip: for 64 entries at a time,
//                  lane t forms the mask of the entries covering its tile
//                  and appends them, in order, to its tile's run, staged in
//                  LDS per tile (the sub-chunk counts place each wave's part
//                  of the run); the staged pairs are then stored with
//                  consecutive threads on consecutive positions.  A chunk
//                  with more pairs than the LDS stage goes through it in
//                  several windows.
// Positions at or past the capacity are never written; the ranges are
// clamped to the capacity (the scan has then set SGS_STATUS_CAPACITY).
#include "common.hpp"

namespace sgs {

static_assert(kStripTiles == 64, "one wave lane per tile of a strip");
static_assert(kBinSub % 64 == 0 && kBinSub / 64 <= 8, "whole entry batches per lane");
constexpr int kBinBatches = kBinSub / 64;   // entries per lane of a sub-chunk

// Inclusive scans over the 64 lanes of a wave with DPP moves: shifts by 1,
// 2, 4 and 8 lanes within each row of 16, then lane 15 of rows 0 and 2 into
// rows 1 and 3, then lane 31 into rows 2 and 3.  A lane whose source lies
// outside its row (or in a row the mask leaves out) receives 0, the identity
// of both operations.
#define SGS_DPP(x, ctrl, rows) \
    ((uint32_t)__builtin_amdgcn_update_dpp(0, (int)(x), (ctrl), (rows), 0xF, false))

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
    v += SGS_DPP(v, 0x111, 0xF);
    v += SGS_DPP(v, 0x112, 0xF);
    v += SGS_DPP(v, 0x114, 0xF);
    v += SGS_DPP(v, 0x118, 0xF);
    v += SGS_DPP(v, 0x142, 0xA);
    v += SGS_DPP(v, 0x143, 0xC);
    return v;
}

__device__ __forceinline__ uint32_t wave_prefix_or32(uint32_t v) {
    v |= SGS_DPP(v, 0x111, 0xF);
    v |= SGS_DPP(v, 0x112, 0xF);
    v |= SGS_DPP(v, 0x114, 0xF);
    v |= SGS_DPP(v, 0x118, 0xF);
    v |= SGS_DPP(v, 0x142, 0xA);
    v |= SGS_DPP(v, 0x143, 0xC);
    return v;
}

// inclusive OR of v over lanes 0 .. lane
__device__ __forceinline__ uint64_t wave_prefix_or(uint64_t v) {
    return (uint64_t)wave_prefix_or32((uint32_t)v) | ((uint64_t)wave_prefix_or32((uint32_t)(v >> 32)) << 32);
}

__device__ __forceinline__ uint64_t wave_incl_scan64(uint64_t v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint64_t y = __shfl_up(v, off, 64);
        if (lane >= off) v += y;
    }
    return v;
}

// ---------------------------------------------------------------------------
// chunk table (one block of 1024 threads; thread t owns a run of strips)
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(1024) k_bin_chunks(Workspace ws) {
    const int n_cams = ws.n_cams;
    constexpr int WAVES = 1024 / 64;
    __shared__ uint32_t s_w[WAVES];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t S = ws.n_strips;
    const int64_t per = (S + 1023) / 1024;
    const int64_t s0 = (int64_t)tid * per < S ? (int64_t)tid * per : S;
    const int64_t s1 = s0 + per < S ? s0 + per : S;
    uint32_t local = 0;
    for (int64_t s = s0; s < s1; ++s) {
        const uint32_t a = ws.strip_ranges[2 * s], b = ws.strip_ranges[2 * s + 1];
        const uint32_t e = b > a ? b - a : 0u;
        local += (e + kBinChunk - 1) / kBinChunk;
    }
    // exclusive scan of the chunk counts over threads
    const uint32_t incl = wave_incl_scan(local);
    if (lane == 63) s_w[wave] = incl;
    __syncthreads();
    uint32_t before = 0, total = 0;
#pragma unroll
    for (int w = 0; w < WAVES; ++w) {
        before += w < wave ? s_w[w] : 0u;
        total += s_w[w];
    }
    int64_t cb = before + incl - local;
    if (s0 < s1 && n_cams > 0) {
        // the camera of s0: the last one whose first strip is <= s0
        int lo = 0, hi = n_cams - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if ((int64_t)ws.cams[mid].strip_base <= s0) lo = mid; else hi = mid - 1;
        }
        int cam = lo;
        for (int64_t s = s0; s < s1; ++s) {
            while (cam + 1 < n_cams && (int64_t)ws.cams[cam + 1].strip_base <= s) ++cam;
            const CamTable ct = ws.cams[cam];
            const int SX = (ct.GX + kStripTiles - 1) >> kStripShift;
            const int64_t ls = s - ct.strip_base;
            uint32_t tb = 0, shape = 0;
            if (SX > 0 && ls >= 0 && ls < (int64_t)SX * ct.GY) {
                const int ty = (int)(ls / SX), sx = (int)(ls - (int64_t)ty * SX);
                const int x0 = sx << kStripShift;
                const int sw = ct.GX - x0 < kStripTiles ? ct.GX - x0 : kStripTiles;
                tb = (uint32_t)(ct.tile_base + ty * ct.GX + x0);
                shape = (uint32_t)sw | ((uint32_t)x0 << 16);
            }
            const uint32_t a = ws.strip_ranges[2 * s], b = ws.strip_ranges[2 * s + 1];
            const uint32_t e = b > a ? b - a : 0u;
            int64_t nch = (e + kBinChunk - 1) / kBinChunk;
            if (cb + nch > ws.chunk_cap) nch = ws.chunk_cap > cb ? ws.chunk_cap - cb : 0;
            ws.strip_info[s] = make_uint4((uint32_t)cb, (uint32_t)nch, tb, shape);
            for (int64_t k = 0; k < nch; ++k) {
                const uint32_t c0 = a + (uint32_t)k * kBinChunk;
                uint32_t c1 = c0 + kBinChunk < b ? c0 + kBinChunk : b;
                if (shape == 0) c1 = c0;   // a strip the device cameras do not have: no work
                ws.chunk_info[cb + k] = make_uint4(c0, c1, tb, shape);
            }
            cb += nch;
        }
    }
    if (tid == 0)
        ws.header[kHdrChunks] = (uint32_t)((int64_t)total < ws.chunk_cap ? (int64_t)total : ws.chunk_cap);
}

// The chunk a wave takes in round r of a persistent grid of `blocks` blocks
// of `wpb` waves: consecutive chunks stay on one XCD (its L2 merges the
// partial lines that neighbouring chunks of a strip write to each tile).
__device__ __forceinline__ int64_t bin_chunk_of(int64_t round, int64_t n_chunks, int wpb, int wave) {
    const int64_t per_round = (int64_t)gridDim.x * wpb;
    const int64_t left = n_chunks - round * per_round;
    const int64_t live = left <= 0 ? 0 : (left + wpb - 1) / wpb;
    const int64_t blk = xcd_part(blockIdx.x, live < gridDim.x ? live : gridDim.x);
    return round * per_round + blk * wpb + wave;
}

// The local tile interval of an entry: first tile | tile count << 16 (count
// 0: it covers none of the strip's tiles)
__device__ __forceinline__ uint32_t entry_interval(uint64_t r, int x0, int sw) {
    const int tx0 = (int)(r & 0xFFFF) - x0, tx1 = (int)((r >> 16) & 0xFFFF) - x0;
    const int a = tx0 > 0 ? tx0 : 0, b = tx1 < sw - 1 ? tx1 : sw - 1;
    return b >= a ? (uint32_t)a | ((uint32_t)(b - a + 1) << 16) : 0xFFFFu;
}

// ---------------------------------------------------------------------------
// per chunk and tile: entries of the chunk covering the tile
// ---------------------------------------------------------------------------

constexpr int kBinWaves = 4;   // waves per block of the counting kernel

__global__ void __launch_bounds__(64 * kBinWaves)
k_bin_count(Workspace ws, const uint32_t* __restrict__ entries) {
    __shared__ int s_diff[kBinWaves][kStripTiles + 1];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t nsub = (int64_t)ws.header[kHdrChunks] * kBinSubs;
    const int64_t nvis = ws.header[kHdrVisible] < ws.n_items ? ws.header[kHdrVisible] : ws.n_items;
    for (int64_t round = 0;; ++round) {
        if (round * gridDim.x * kBinWaves >= nsub) break;   // uniform over the block
        const int64_t r = bin_chunk_of(round, nsub, kBinWaves, wave);
        if (r >= nsub) continue;   // uniform over the wave
        const uint4 ci = ws.chunk_info[r / kBinSubs];
        const int sw = (int)(ci.w & 0xFFFF), x0 = (int)(ci.w >> 16);
        const uint32_t e0 = ci.x + (uint32_t)(r % kBinSubs) * kBinSub;   // this sub-chunk's entries
        s_diff[wave][lane] = 0;
        if (lane == 0) s_diff[wave][kStripTiles] = 0;
        // loads without branches (clamped indices, validity applied after),
        // so that they are in flight together
        const uint32_t last = ci.y > ci.x ? ci.y - 1 : 0u;
        uint32_t slot[kBinBatches];
#pragma unroll
        for (int k = 0; k < kBinBatches; ++k) {
            const uint32_t e = e0 + (uint32_t)(k * 64 + lane);
            slot[k] = entries[e < ci.y ? e : last];
        }
        bool ok[kBinBatches];
        uint64_t rect[kBinBatches];
#pragma unroll
        for (int k = 0; k < kBinBatches; ++k) {
            ok[k] = e0 + (uint32_t)(k * 64 + lane) < ci.y && slot[k] < (uint64_t)nvis;
            rect[k] = ws.sorted_rects[ok[k] ? slot[k] : 0u];
        }
        __builtin_amdgcn_wave_barrier();
        // a wave's LDS operations complete in order: the clears land before
        // the additions, the additions before the reads
#pragma unroll
        for (int k = 0; k < kBinBatches; ++k) {
            const uint32_t iv = ok[k] ? entry_interval(rect[k], x0, sw) : 0xFFFFu;
            const int a = (int)(iv & 0xFFFF), w = (int)(iv >> 16);
            if (w > 0) {
                atomicAdd(&s_diff[wave][a], 1);
                atomicAdd(&s_diff[wave][a + w], -1);
            }
        }
        __builtin_amdgcn_wave_barrier();
        const uint32_t cnt = wave_incl_scan((uint32_t)s_diff[wave][lane]);
        ws.chunk_counts[r * kStripTiles + lane] = (uint16_t)cnt;   // 0 past the strip's width
        __builtin_amdgcn_wave_barrier();
    }
}

// ---------------------------------------------------------------------------
// per strip: exclusive sums of each tile's chunk counts over the strip's
// chunks (16 waves, each over a contiguous run of chunks), and tile totals
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(1024) k_bin_strips(Workspace ws) {
    constexpr int WAVES = 1024 / 64;
    __shared__ uint32_t s_seg[WAVES][kStripTiles];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int64_t s = blockIdx.x; s < ws.n_strips; s += gridDim.x) {
        const uint4 si = ws.strip_info[s];
        const int64_t cb = (int64_t)si.x * kBinSubs, nch = (int64_t)si.y * kBinSubs;   // sub-chunks
        const int sw = (int)(si.w & 0xFFFF);
        const int64_t seg = (nch + WAVES - 1) / WAVES;
        const int64_t k0 = (int64_t)wave * seg < nch ? (int64_t)wave * seg : nch;
        const int64_t k1 = k0 + seg < nch ? k0 + seg : nch;
        // eight sub-chunks' counts in flight at a time (indices clamped to
        // the wave's run, so the loads carry no branches)
        constexpr int U = 8;
        uint32_t sum = 0;
        for (int64_t k = k0; k < k1; k += U) {
            uint32_t v[U];
#pragma unroll
            for (int j = 0; j < U; ++j) {
                const int64_t kk = k + j < k1 ? k + j : k1 - 1;
                v[j] = ws.chunk_counts[(cb + kk) * kStripTiles + lane];
            }
#pragma unroll
            for (int j = 0; j < U; ++j) sum += k + j < k1 ? v[j] : 0u;
        }
        __syncthreads();   // the previous strip is done with s_seg
        s_seg[wave][lane] = sum;
        __syncthreads();
        uint32_t run = 0, total = 0;
#pragma unroll
        for (int w = 0; w < WAVES; ++w) {
            const uint32_t v = s_seg[w][lane];
            run += w < wave ? v : 0u;
            total += v;
        }
        for (int64_t k = k0; k < k1; k += U) {
            uint32_t v[U];
#pragma unroll
            for (int j = 0; j < U; ++j) {
                const int64_t kk = k + j < k1 ? k + j : k1 - 1;
                v[j] = ws.chunk_counts[(cb + kk) * kStripTiles + lane];
            }
#pragma unroll
            for (int j = 0; j < U; ++j) {
                if (k + j < k1) {
                    ws.chunk_offsets[(cb + k + j) * kStripTiles + lane] = run;
                    run += v[j];
                }
            }
        }
        if (wave == 0 && lane < sw && (int64_t)si.z + lane < ws.n_tiles) ws.tile_count[si.z + lane] = total;
    }
}

// ---------------------------------------------------------------------------
// one block: tile starts and ranges from the tile totals
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(1024) k_bin_tiles(Workspace ws) {
    constexpr int WAVES = 1024 / 64;
    constexpr int IT = 8;
    constexpr int N = 1024 * IT;   // tiles per round
    // the round's counts, then its starts (saturated to 32 bits); entry N
    // holds the start after the round
    __shared__ uint32_t s_v[N + 1];
    __shared__ uint64_t s_w[WAVES];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t T = ws.n_tiles;
    const uint64_t cap = (uint64_t)ws.capacity;
    auto sat = [](uint64_t x) { return (uint32_t)(x < 0xFFFFFFFFull ? x : 0xFFFFFFFFull); };
    uint64_t carry = 0;
    for (int64_t b0 = 0; b0 < T; b0 += N) {
        // coalesced loads, then each thread takes IT consecutive tiles
#pragma unroll
        for (int k = 0; k < IT; ++k) {
            const int64_t i = b0 + (int64_t)k * 1024 + tid;
            s_v[k * 1024 + tid] = i < T ? ws.tile_count[i] : 0u;
        }
        __syncthreads();
        uint32_t v[IT];
        uint64_t run = 0;
#pragma unroll
        for (int k = 0; k < IT; ++k) {
            v[k] = s_v[tid * IT + k];
            run += v[k];
        }
        const uint64_t incl = wave_incl_scan64(run);
        if (lane == 63) s_w[wave] = incl;
        __syncthreads();   // the counts are read and the wave totals written
        uint64_t before = 0, all = 0;
#pragma unroll
        for (int w = 0; w < WAVES; ++w) {
            before += w < wave ? s_w[w] : 0ull;
            all += s_w[w];
        }
        uint64_t st = carry + before + incl - run;
#pragma unroll
        for (int k = 0; k < IT; ++k) {
            s_v[tid * IT + k] = sat(st);
            st += v[k];
        }
        if (tid == 0) s_v[N] = sat(carry + all);
        __syncthreads();
        // coalesced stores: a tile's range ends where the next tile starts
        // (clamped to the capacity; a saturated start lies past it)
#pragma unroll
        for (int k = 0; k < IT; ++k) {
            const int j = k * 1024 + tid;
            const int64_t i = b0 + j;
            if (i < T) {
                const uint32_t a32 = s_v[j], e32 = s_v[j + 1];
                ws.tile_start[i] = a32;
                const uint64_t a = a32 < cap ? a32 : cap, e = e32 < cap ? e32 : cap;
                ws.ranges[2 * i] = a < e ? (uint32_t)a : 0u;
                ws.ranges[2 * i + 1] = a < e ? (uint32_t)e : 0u;
            }
        }
        carry += all;
        __syncthreads();   // s_v and s_w are read before the next round writes them
    }
}

// ---------------------------------------------------------------------------
// per chunk: the pairs, staged by tile, then stored
// ---------------------------------------------------------------------------

static_assert((kBinStage & (kBinStage - 1)) == 0, "the stage index is masked");

// The store of a staged window of n pairs whose first staged index is w0:
// thread tid takes staged indices tid + 256 j, four at a time so that their
// LDS reads are in flight together.  Staged value v = tile * kBinChunk +
// entry goes to s_gb[tile] + w0 + index (32-bit positions; one at or past
// the capacity, or below zero, is not written).
__device__ __forceinline__ void store_stage(uint32_t* __restrict__ out, const uint16_t* s_stage,
                                            const int32_t* s_gb, const uint32_t* s_item, uint32_t n,
                                            uint32_t w0, uint32_t cap) {
    constexpr uint32_t T = 64 * kBinSubs, U = 4;
    char* const ob = reinterpret_cast<char*>(out);
    for (uint32_t i0 = threadIdx.x; i0 < n; i0 += T * U) {
        uint32_t v[U];
#pragma unroll
        for (uint32_t u = 0; u < U; ++u) {
            const uint32_t i = i0 + u * T;
            v[u] = s_stage[i < n ? i : i0];
        }
        int32_t gb[U];
        uint32_t it[U];
#pragma unroll
        for (uint32_t u = 0; u < U; ++u) {
            gb[u] = s_gb[v[u] / kBinChunk];
            it[u] = s_item[v[u] % kBinChunk];
        }
#pragma unroll
        for (uint32_t u = 0; u < U; ++u) {
            const uint32_t i = i0 + u * T;
            const uint32_t g = (uint32_t)(gb[u] + (int32_t)(w0 + i));
            // (a byte offset below 2^32: g < cap < 2^30)
            if (i < n && g < cap) *reinterpret_cast<uint32_t*>(ob + 4u * g) = it[u];
        }
    }
}

// One workgroup per chunk, wave w taking sub-chunk w.  For each batch of 64
// entries (lane k holds entry k), an entry covering tiles a .. a + w - 1
// sets its bit k in the start mark of tile a and the end mark of tile a + w;
// lane t (tile t) then ORs the marks of tiles 0 .. t: the entries covering t
// are those started and not ended, in entry order = bit order.  Lane t walks
// its set bits and stages their indices at its tile's running position.
__global__ void __launch_bounds__(64 * kBinSubs)
k_bin_scatter(Workspace ws, const uint32_t* __restrict__ entries, const uint4* __restrict__ chunk_info) {
    static_assert(kStripTiles * kBinChunk <= 65536, "staged tile and entry index fit 16 bits");
    __shared__ uint32_t s_item[kBinChunk];                  // items of the chunk's entries
    __shared__ uint16_t s_stage[kBinStage];                 // tile * kBinChunk + entry, by tile
    __shared__ uint64_t s_start[kBinSubs][kStripTiles];     // entries starting at each tile
    __shared__ uint64_t s_end[kBinSubs][kStripTiles + 1];   // entries ending before each tile
    __shared__ int32_t s_gb[kStripTiles];                   // position of staged index 0 of each tile's run
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t nc = ws.header[kHdrChunks];
    const int64_t nvis = ws.header[kHdrVisible] < ws.n_items ? ws.header[kHdrVisible] : ws.n_items;
    const uint32_t cap = (uint32_t)ws.capacity;   // below 2^30
    s_start[wave][lane] = 0ull;
    s_end[wave][lane] = 0ull;
    for (int64_t round = 0;; ++round) {
        const int64_t c = bin_chunk_of(round, nc, 1, 0);
        if (c >= nc) break;   // uniform over the block
        const uint4 ci = chunk_info[c];
        const int sw = (int)(ci.w & 0xFFFF), x0 = (int)(ci.w >> 16);
        const uint32_t e0 = ci.x + (uint32_t)wave * kBinSub;   // this wave's sub-chunk
        // loads without branches (clamped indices, validity applied after),
        // so that they are in flight together: this wave's entries, every
        // sub-chunk's count of this lane's tile, the chunk's earlier count
        // and the tile's start
        const uint32_t last = ci.y > ci.x ? ci.y - 1 : 0u;
        uint32_t slot[kBinBatches];
#pragma unroll
        for (int k = 0; k < kBinBatches; ++k) {
            const uint32_t e = e0 + (uint32_t)(k * 64 + lane);
            slot[k] = entries[e < ci.y ? e : last];
        }
        uint32_t raw[kBinSubs];
#pragma unroll
        for (int q = 0; q < kBinSubs; ++q) raw[q] = ws.chunk_counts[(c * kBinSubs + q) * kStripTiles + lane];
        const uint32_t off = ws.chunk_offsets[c * kBinSubs * kStripTiles + lane];
        const bool live = lane < sw && (int64_t)ci.z + lane < ws.n_tiles;
        const uint32_t ts_l = ws.tile_start[live ? ci.z + lane : 0u];
        bool ok[kBinBatches];
        uint32_t item[kBinBatches];
        uint64_t rect[kBinBatches];
#pragma unroll
        for (int k = 0; k < kBinBatches; ++k) {
            ok[k] = e0 + (uint32_t)(k * 64 + lane) < ci.y && slot[k] < (uint64_t)nvis;
            const uint32_t sl = ok[k] ? slot[k] : 0u;
            item[k] = ws.sorted_items[sl];
            rect[k] = ws.sorted_rects[sl];
        }
        // this lane's tile: its pairs in the chunk, its first staged index,
        // this wave's part of its run, and where the run goes
        uint32_t cnt = 0, before = 0;
#pragma unroll
        for (int q = 0; q < kBinSubs; ++q) {
            cnt += raw[q];
            before += q < wave ? raw[q] : 0u;
        }
        if (!live) cnt = before = 0;
        const uint32_t incl = wave_incl_scan(cnt);
        const uint32_t lb = incl - cnt;
        const uint32_t total = __builtin_amdgcn_readlane(incl, 63);
        // position = gb + staged index, in 32 bits: a run that starts at or
        // past the capacity (< 2^30) gets gb = 2^30, so none of its
        // positions (staged indices < 2^15) is below the capacity
        const int64_t gb64 = (int64_t)(live ? ts_l : 0u) + off - lb;
        const int32_t gb = (int32_t)(gb64 < (int64_t(1) << 30) ? gb64 : (int64_t(1) << 30));
        if (wave == 0) s_gb[lane] = gb;
        // the masks of this wave's two batches, kept for the stage windows
        uint64_t msk[kBinBatches];
#pragma unroll
        for (int k = 0; k < kBinBatches; ++k) {
            s_item[wave * kBinSub + k * 64 + lane] = ok[k] ? item[k] : 0u;
            const uint32_t iv = ok[k] ? entry_interval(rect[k], x0, sw) : 0xFFFFu;
            const uint32_t a = iv & 0xFFFFu, w = iv >> 16;
            if (w > 0) {
                atomicOr(&s_start[wave][a], 1ull << lane);
                atomicOr(&s_end[wave][a + w], 1ull << lane);
            }
            __builtin_amdgcn_wave_barrier();
            // a wave's LDS operations complete in order: the marks are set
            // before they are read, and read before they are cleared
            const uint64_t st = s_start[wave][lane], en = s_end[wave][lane];
            s_start[wave][lane] = 0ull;
            s_end[wave][lane] = 0ull;
            const uint64_t m = wave_prefix_or(st) & ~wave_prefix_or(en);
            msk[k] = live ? m : 0ull;
            __builtin_amdgcn_wave_barrier();
        }
        // the chunk's pairs go through the stage in windows of kBinStage
        // staged indices (one window unless the chunk holds more pairs)
        if (total <= (uint32_t)kBinStage) {
            // one window: each lane walks its set bits, 32 at a time, with
            // the stage addressed in bytes (the mask keeps a count that
            // disagreed with the walk inside the stage)
            char* const stage = reinterpret_cast<char*>(s_stage);
            uint32_t pb = 2u * (lb + before);
#pragma unroll
            for (int k = 0; k < kBinBatches; ++k) {
                // a multiple of 64: the entry index is or-ed into the low bits
                const uint32_t tag = (uint32_t)lane * kBinChunk + (uint32_t)(wave * kBinSub + k * 64);
                uint32_t lo = (uint32_t)msk[k], hi = (uint32_t)(msk[k] >> 32);
                while (lo) {
                    *reinterpret_cast<uint16_t*>(stage + (pb & (2u * kBinStage - 2u))) =
                        (uint16_t)(tag | (uint32_t)__builtin_ctz(lo));
                    pb += 2u;
                    lo &= lo - 1u;
                }
                const uint32_t tag_hi = tag | 32u;
                while (hi) {
                    *reinterpret_cast<uint16_t*>(stage + (pb & (2u * kBinStage - 2u))) =
                        (uint16_t)(tag_hi | (uint32_t)__builtin_ctz(hi));
                    pb += 2u;
                    hi &= hi - 1u;
                }
            }
            __syncthreads();   // the stage, the items and s_gb are complete
            store_stage(ws.pair_values, s_stage, s_gb, s_item, total, 0u, cap);
            __syncthreads();   // stored before the next chunk stages
            continue;
        }
        for (uint32_t w0 = 0; w0 < total; w0 += kBinStage) {
            const uint32_t w1 = w0 + kBinStage;
            // each half mask whose run overlaps the window is walked up to
            // the window's end; the others are only counted
            uint32_t pos = lb + before;
#pragma unroll
            for (int h = 0; h < 2 * kBinBatches; ++h) {
                uint32_t m = (h & 1) ? (uint32_t)(msk[h >> 1] >> 32) : (uint32_t)msk[h >> 1];
                const uint32_t n = (uint32_t)__popc(m);
                if (pos < w1 && pos + n > w0) {
                    const uint32_t tag =
                        (uint32_t)lane * kBinChunk + (uint32_t)(wave * kBinSub + (h >> 1) * 64 + (h & 1) * 32);
                    uint32_t p = pos;
                    while (m && p < w1) {
                        // (below w0 the difference wraps past the stage)
                        if (p - w0 < (uint32_t)kBinStage) s_stage[p - w0] = (uint16_t)(tag | (uint32_t)__builtin_ctz(m));
                        m &= m - 1u;
                        ++p;
                    }
                }
                pos += n;
            }
            __syncthreads();   // the window, the items and s_gb are complete
            const uint32_t nw = total - w0 < (uint32_t)kBinStage ? total - w0 : (uint32_t)kBinStage;
            store_stage(ws.pair_values, s_stage, s_gb, s_item, nw, w0, cap);
            __syncthreads();   // the window is stored before the next one is staged
        }
    }
}

void launch_bin_tiles(const Workspace& ws, const uint32_t* entry_slots, hipStream_t s) {
    if (ws.n_strips <= 0 || ws.n_tiles <= 0) return;
    hipLaunchKernelGGL(k_bin_chunks, dim3(1), dim3(1024), 0, s, ws);
    // persistent grids no larger than what stays resident (a block that
    // waits for a free slot would run its whole loop after the others)
    const int64_t cus = ws.cus > 0 ? ws.cus : 256;
    const int64_t cblocks = (ws.chunk_cap * kBinSubs + kBinWaves - 1) / kBinWaves;
    const int64_t cmax = cus * 8;   // 32 waves per CU
    hipLaunchKernelGGL(k_bin_count, dim3((unsigned)(cblocks < cmax ? cblocks : cmax)),
                       dim3(64 * kBinWaves), 0, s, ws, entry_slots);
    const int64_t sblocks = ws.n_strips < 1024 ? ws.n_strips : 1024;
    hipLaunchKernelGGL(k_bin_strips, dim3((unsigned)sblocks), dim3(1024), 0, s, ws);
    hipLaunchKernelGGL(k_bin_tiles, dim3(1), dim3(1024), 0, s, ws);
    const int64_t wmax = cus * 7;   // LDS holds 7 of these blocks (22.5 KB each) per CU
    const int64_t wblocks = ws.chunk_cap < wmax ? ws.chunk_cap : wmax;
    hipLaunchKernelGGL(k_bin_scatter, dim3((unsigned)wblocks), dim3(64 * kBinSubs), 0, s, ws,
                       entry_slots, ws.chunk_info);
}

}  // namespace sgs
