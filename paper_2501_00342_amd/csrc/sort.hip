// Binning of (tile, depth) pairs: set-up, the first level's duplication,
// tile ranges.
//
// The pairs must come out in ascending key order, key = (tile << 32) |
// bits(float32 depth), ties by Gaussian index (the order a stable sort of
// index-ordered emission gives).  Instead of a radix sort over the whole
// 64-bit key, three stable steps give the same order:
//   1. the (camera, Gaussian) items are sorted by their 32-bit depth key
//      (four 8-bit passes over n_items, values = item index);
//   2. (strip, item) entries are emitted item by item in that order, one
//      per tile row and strip column (a strip: at most kStripTiles
//      consecutive tiles of a row) of the item's tile rectangle, and stably
//      partitioned by strip id (ceil(bits/8) radix passes);
//   3. each strip's entries, still in depth order, are expanded into the
//      pairs of the strip's tiles and written to their final positions
//      (bin.hip).
// Strips are numbered row-major within a camera, like the tiles, so tile
// order is strip order, then column within the strip.  A stable partition
// of a depth-ordered sequence is ordered by (tile, depth, item).  The radix
// passes live in radix.hip.
#include "common.hpp"
#include "pairs.hpp"

namespace sgs {


// --------------------------------------------------------------------------
// fill / clear / setup
// --------------------------------------------------------------------------

__global__ void k_fill_u32(uint32_t* p, uint32_t v, int64_t count) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// zeroes the 2D gradient record of every visible item (the backward blend
// adds only into those, and the backward preprocess reads only those), from
// the depth-order list: four consecutive threads clear the four 16-byte
// quarters of one record, so each record is one whole-line store
__global__ void __launch_bounds__(256) k_clear_grad2d(Workspace ws) {
    constexpr int Q = kG2 / 4;   // 16-byte quarters per record
    const int64_t nv = ws.header[kHdrVisible] < ws.n_items ? ws.header[kHdrVisible] : ws.n_items;
    const float4 z = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nv * Q;
         t += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t item = ws.sorted_items[t / Q];
        if (item >= (uint64_t)ws.n_items) continue;
        reinterpret_cast<float4*>(ws.grad2d)[(int64_t)item * Q + (t % Q)] = z;
    }
}

void launch_clear_grad2d(const Workspace& ws, hipStream_t s) {
    if (ws.n_items <= 0) return;
    int64_t blocks = (ws.n_items * (kG2 / 4) + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_clear_grad2d, dim3((unsigned)blocks), dim3(256), 0, s, ws);
}

void launch_fill_u32(uint32_t* p, uint32_t v, int64_t count, hipStream_t s) {
    if (count <= 0) return;
    int64_t blocks = (count + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, s, p, v, count);
}

// The start of a forward in one launch: every block clears tile and strip
// ranges; block 0 clears the header, then its thread 0 builds the camera
// table (after the clear, so a camera error bit survives it).
__global__ void __launch_bounds__(256)
k_setup(Workspace ws, const sgs_camera* __restrict__ cams, int n_cams, int tw, int th,
        float guard) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < 2 * ws.n_tiles;
         i += (int64_t)gridDim.x * blockDim.x)
        ws.ranges[i] = 0u;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < 2 * ws.n_strips;
         i += (int64_t)gridDim.x * blockDim.x)
        ws.strip_ranges[i] = 0u;
    if (blockIdx.x != 0) return;   // uniform
    if (threadIdx.x < kHdrWords) ws.header[threadIdx.x] = 0u;
    __syncthreads();
    if (threadIdx.x != 0) return;
    int64_t tiles = 0, pix = 0, strips = 0;
    bool ok = true;
    for (int c = 0; c < n_cams; ++c) {
        CamTable t;
        t.W = cams[c].width;
        t.H = cams[c].height;
        ok = ok && t.W > 0 && t.H > 0 && t.W <= SGS_MAX_IMAGE_SIDE && t.H <= SGS_MAX_IMAGE_SIDE;
        // the same camera rules the host checks: a positive near plane and
        // positive focal lengths (comparisons are false for NaN)
        ok = ok && cams[c].znear > 0.0f && cams[c].znear <= 3.0e38f && cams[c].fx > 0.0f &&
             cams[c].fx <= 3.0e38f && cams[c].fy > 0.0f && cams[c].fy <= 3.0e38f;
        t.GX = ok ? (t.W + tw - 1) / tw : 0;
        t.GY = ok ? (t.H + th - 1) / th : 0;
        t.tile_base = (int32_t)tiles;
        t.strip_base = (int32_t)strips;
        t.pix_base = pix;
        t.limx = (double)guard * ((0.5 * t.W) / (double)cams[c].fx);
        t.limy = (double)guard * ((0.5 * t.H) / (double)cams[c].fy);
        ws.cams[c] = t;
        tiles += (int64_t)t.GX * t.GY;
        strips += (int64_t)t.GY * ((t.GX + kStripTiles - 1) >> kStripShift);
        pix += (int64_t)t.W * t.H;
    }
    // the device cameras must be valid and describe the sizes the host planned for
    if (!ok || pix != ws.n_pixels || tiles != ws.n_tiles || strips != ws.n_strips)
        atomicOr(&ws.header[kHdrStatus], SGS_STATUS_CAMERAS);
}

void launch_setup(const Workspace& ws, const sgs_camera* dev_cams, int n_cams, int tile_w, int tile_h,
                  float guard, hipStream_t s) {
    const int64_t most = ws.n_tiles > ws.n_strips ? ws.n_tiles : ws.n_strips;
    int64_t blocks = (2 * most + 255) / 256;
    blocks = blocks < 1 ? 1 : (blocks > 1024 ? 1024 : blocks);
    hipLaunchKernelGGL(k_setup, dim3((unsigned)blocks), dim3(256), 0, s, ws, dev_cams, n_cams, tile_w,
                       tile_h, guard);
}

// --------------------------------------------------------------------------
// duplicate (counting): one block per 2048-entry chunk, eight consecutive
// entries per thread (balanced: entries, not Gaussians, are split between
// threads).  It generates every (strip, item) entry and counts the low 8
// bits of its strip id: chunk c's counts go to counts[d * 2 * pair_parts +
// c] (two chunks per radix partition), the first strip pass's digit
// histogram; chunks past the entry count are left alone.  The entries
// themselves are generated again by that pass, which scatters them
// directly (nothing else is written here).
// --------------------------------------------------------------------------

static_assert(2 * kDupChunk == kSortTile, "two duplicate chunks per radix partition");
constexpr int kDupRun = kDupChunk / 256;   // consecutive pairs per thread

__global__ void __launch_bounds__(256)
k_duplicate(Workspace ws, int64_t n) {
    __shared__ uint32_t s_off[kChunkItems];
    __shared__ uint32_t s_origin[kChunkItems];
    __shared__ uint32_t s_wgx[kChunkItems];
    __shared__ uint32_t s_item[kChunkItems];
    __shared__ uint32_t s_hist[kRadix];
    const ChunkItems ci = {s_off, s_origin, s_wgx, s_item};
    const int tid = threadIdx.x;
    const uint32_t P = ws.header[kHdrEntries];
    const int64_t Pc = (int64_t)P < ws.capacity ? (int64_t)P : ws.capacity;
    const uint32_t nn = (uint32_t)n;
    const int64_t n_vis = ws.header[kHdrVisible] < ws.n_items ? ws.header[kHdrVisible] : ws.n_items;
    const int64_t row = 2 * ws.pair_parts;   // histogram row length
    const int64_t n_chunks = (Pc + kDupChunk - 1) / kDupChunk;
    for (int64_t round = 0; round + blockIdx.x < n_chunks; round += gridDim.x) {
        const int64_t live = n_chunks - round < gridDim.x ? n_chunks - round : gridDim.x;
        const int64_t chunk = round + xcd_part(blockIdx.x, live);
        const int64_t p0 = chunk * kDupChunk;
        const int64_t p1 = (p0 + kDupChunk < Pc) ? p0 + kDupChunk : Pc;
        __syncthreads();   // previous chunk done with LDS
        s_hist[tid] = 0;
        const int nloc = load_chunk_items(ws, chunk, p1, Pc, n_vis, nn, ci, tid, 256);
        if (nloc < 1) {
            ws.counts[tid * row + chunk] = 0;
            continue;   // uniform
        }
        __syncthreads();
        // thread t walks the kDupRun consecutive entries from p0 + kDupRun t
        const int64_t q0 = p0 + (int64_t)tid * kDupRun;
        if (q0 < p1) {
            uint32_t tl[kDupRun], vl[kDupRun];
            const int cnt = p1 - q0 < kDupRun ? (int)(p1 - q0) : kDupRun;
            gen_pairs<kDupRun>(ci, nloc, q0, cnt, tl, vl);
#pragma unroll
            for (int e = 0; e < kDupRun; ++e)
                if (e < cnt) atomicAdd(&s_hist[tl[e] & (kRadix - 1)], 1u);
        }
        __syncthreads();
        ws.counts[tid * row + chunk] = s_hist[tid];
    }
    // (the row scans read only the chunks that hold entries)
}

void launch_duplicate_counts(const Workspace& ws, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_duplicate, dim3((unsigned)ws.dup_blocks), dim3(256), 0, s, ws, n);
}

// --------------------------------------------------------------------------
// heavy-first tile order for the queue schedule: key = 255 - bucket, bucket =
// 0 for an empty tile, else 1 + 8 e + m with e = floor(log2(length)) and m the
// three bits below the leading one (eight buckets per octave), so one stable
// 8-bit pass puts long tiles first and keeps tile order within a bucket
// --------------------------------------------------------------------------

__global__ void __launch_bounds__(256) k_tile_keys(Workspace ws) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= ws.n_tiles) return;
    const uint32_t a = ws.ranges[2 * t], b = ws.ranges[2 * t + 1];
    const uint32_t len = b > a ? b - a : 0u;
    uint32_t bucket = 0;
    if (len > 0) {
        const int e = 31 - __clz((int)len);
        const uint32_t m = (e >= 3 ? len >> (e - 3) : len << (3 - e)) & 7u;
        const uint32_t lb = 8u * (uint32_t)e + m;
        bucket = 1u + (lb > 254u ? 254u : lb);
    }
    ws.tile_keys[t] = 255u - bucket;
}

void launch_tile_order(const Workspace& ws, int64_t parts, hipStream_t s) {
    if (ws.n_tiles <= 0) return;
    const int64_t blocks = (ws.n_tiles + 255) / 256;
    hipLaunchKernelGGL(k_tile_keys, dim3((unsigned)blocks), dim3(256), 0, s, ws);
    launch_radix_pass(ws.tile_keys, nullptr, nullptr, ws.tile_order, nullptr, ws.n_tiles, 0,
                      ws.counts, ws.totals, parts, nullptr, nullptr, nullptr, 0, false, nullptr, s);
}

// --------------------------------------------------------------------------
// sorted 64-bit keys for inspection: positions outside every tile range keep
// all bits set; block t writes the keys of tile t's range
// --------------------------------------------------------------------------

__global__ void k_read_keys(Workspace ws, int64_t count, uint64_t* keys) {
    for (int64_t t = blockIdx.x; t < ws.n_tiles; t += gridDim.x) {
        const uint32_t a = ws.ranges[2 * t], b = ws.ranges[2 * t + 1];
        for (int64_t i = (int64_t)a + threadIdx.x; i < (int64_t)b && i < count; i += blockDim.x) {
            const uint32_t item = ws.pair_values[i];
            const uint32_t dk = item < (uint64_t)ws.n_items ? ws.depth_keys[item] : 0xFFFFFFFFu;
            keys[i] = ((uint64_t)t << 32) | dk;
        }
    }
}

void launch_read_keys(const Workspace& ws, int64_t count, uint64_t* keys, hipStream_t s) {
    if (count <= 0) return;
    int64_t blocks = (count + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, s,
                       reinterpret_cast<uint32_t*>(keys), 0xFFFFFFFFu, 2 * count);
    if (ws.n_tiles <= 0) return;
    const int64_t tb = ws.n_tiles < 65536 ? ws.n_tiles : 65536;
    hipLaunchKernelGGL(k_read_keys, dim3((unsigned)tb), dim3(256), 0, s, ws, count, keys);
}

}  // namespace sgs
