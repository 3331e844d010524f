// Generation of the (tile, item) pairs of a chunk of the depth-ordered pair
// sequence, shared by the duplicate (which counts or writes them) and the
// fused first tile pass (which ranks and scatters them directly).
//
// Pair q belongs to the item whose pair offset is the last one <= q; its
// tile is the item's rectangle walked row-major from the origin.
#pragma once

#include "common.hpp"

namespace sgs {

// a chunk of kDupChunk pairs overlaps at most kDupChunk + 1 items (every
// visible item has at least one pair)
constexpr int kChunkItems = kDupChunk + 1;

// LDS arrays of one chunk's items: pair offset, global tile id of the
// rectangle origin, rectangle width | GX << 16, item id
struct ChunkItems {
    uint32_t* off;
    uint32_t* origin;
    uint32_t* wgx;
    uint32_t* item;
};

// Loads the items whose pairs overlap chunk `chunk` (pairs [p0, p1) of Pc)
// into LDS, `nthreads` threads cooperating.  Returns how many; 0 when the
// chunk has no recorded start.  The caller synchronises before (the arrays
// are free) and after (the arrays are read).
__device__ __forceinline__ int load_chunk_items(const Workspace& ws, int64_t chunk, int64_t p1,
                                                int64_t Pc, int64_t n_vis, uint32_t nn,
                                                const ChunkItems& c, int tid, int nthreads) {
    const int64_t i0 = ws.chunk_start[chunk];
    int64_t i_end = n_vis;
    if (chunk + 1 < ws.dup_chunks && p1 < Pc) i_end = (int64_t)ws.chunk_start[chunk + 1] + 1;
    int64_t nloc = i0 < n_vis ? i_end - i0 : 0;   // 0: no chunk start was recorded
    if (nloc > kChunkItems) nloc = kChunkItems;
    if (nloc < 1) return 0;
    for (int j = tid; j < nloc; j += nthreads) {
        const int64_t i = i0 + j;
        uint32_t item = ws.sorted_items[i];
        if (item >= (uint64_t)ws.n_items) item = 0;
        c.off[j] = ws.pair_offsets[i];
        c.item[j] = item;
        const uint64_t r = ws.sorted_rects[i];   // written in depth order by the depth sort
        const int tx0 = (int)(r & 0xFFFF), tx1 = (int)((r >> 16) & 0xFFFF);
        const int ty0 = (int)((r >> 32) & 0xFFFF);
        const CamTable ct = ws.cams[item / nn];
        c.origin[j] = (uint32_t)(ct.tile_base + ty0 * ct.GX + tx0);
        c.wgx[j] = (uint32_t)(tx1 - tx0 + 1) | ((uint32_t)ct.GX << 16);
    }
    return (int)nloc;
}

// The cnt (<= RUN) consecutive pairs from q0 of a chunk whose nloc items are
// in LDS: one binary search for the first, then a walk along the
// rectangles.  tl: global tile ids, vl: item ids.
template <int RUN>
__device__ __forceinline__ void gen_pairs(const ChunkItems& c, int nloc, int64_t q0, int cnt,
                                          uint32_t (&tl)[RUN], uint32_t (&vl)[RUN]) {
    int lo = 0, hi = nloc - 1;   // last local item with offset <= q0
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if ((int64_t)c.off[mid] <= q0) lo = mid; else hi = mid - 1;
    }
    uint32_t wgx = c.wgx[lo];
    int w = (int)(wgx & 0xFFFF), gx = (int)(wgx >> 16);
    const int j = (int)(q0 - c.off[lo]);
    // j / w in float: the quotient is at least 0.5/w from an integer
    int ty = (int)(((float)j + 0.5f) * (1.0f / (float)w));
    int tx = j - ty * w;
    if (tx < 0) { --ty; tx += w; } else if (tx >= w) { ++ty; tx -= w; }
    uint32_t origin = c.origin[lo], item = c.item[lo];
    int64_t next = lo + 1 < nloc ? (int64_t)c.off[lo + 1] : INT64_MAX;
#pragma unroll
    for (int e = 0; e < RUN; ++e) {
        if (e < cnt) {
            if (q0 + e >= next) {   // the next item (every item has >= 1 pair)
                ++lo;
                wgx = c.wgx[lo];
                w = (int)(wgx & 0xFFFF);
                gx = (int)(wgx >> 16);
                origin = c.origin[lo];
                item = c.item[lo];
                next = lo + 1 < nloc ? (int64_t)c.off[lo + 1] : INT64_MAX;
                tx = ty = 0;
            }
            tl[e] = origin + (uint32_t)(ty * gx + tx);
            vl[e] = item;
            if (++tx == w) {
                tx = 0;
                ++ty;
            }
        }
    }
}

}  // namespace sgs
