// Generation of the first binning level's (strip, item) entries for a chunk
// of the depth-ordered entry sequence, shared by the duplicate (which
// counts them) and the fused first strip pass (which ranks and scatters
// them directly).
//
// A strip is a run of at most kStripTiles tiles of one tile row.  Entry q
// belongs to the item whose entry offset is the last one <= q; its strips
// are the item's strip rectangle (tile rows ty0..ty1, strip columns
// tx0 >> kStripShift .. tx1 >> kStripShift) walked row-major.  The entry's
// value is the item's position in the depth order.
#pragma once

#include "common.hpp"

namespace sgs {

// a chunk of kDupChunk entries overlaps at most kDupChunk + 1 items (every
// visible item has at least one entry)
constexpr int kChunkItems = kDupChunk + 1;

// LDS arrays of one chunk's items: entry offset, global strip id of the
// strip rectangle's origin, its width | strips per row << 16, and the
// item's position in the depth order
struct ChunkItems {
    uint32_t* off;
    uint32_t* origin;
    uint32_t* wgx;
    uint32_t* item;
};

// Loads the items whose entries overlap chunk `chunk` (entries [p0, p1) of Pc)
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
        c.item[j] = (uint32_t)i;
        const uint64_t r = ws.sorted_rects[i];   // written in depth order by the depth sort
        const int sx0 = (int)(r & 0xFFFF) >> kStripShift, sx1 = (int)((r >> 16) & 0xFFFF) >> kStripShift;
        const int ty0 = (int)((r >> 32) & 0xFFFF);
        const CamTable ct = ws.cams[item / nn];
        const int SX = (ct.GX + kStripTiles - 1) >> kStripShift;
        c.origin[j] = (uint32_t)(ct.strip_base + ty0 * SX + sx0);
        c.wgx[j] = (uint32_t)(sx1 - sx0 + 1) | ((uint32_t)SX << 16);
    }
    return (int)nloc;
}

// The cnt (<= RUN) consecutive entries from q0 of a chunk whose nloc items
// are in LDS: one binary search for the first, then a walk along the
// strip rectangles.  tl: global strip ids, vl: depth-order positions.
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
            if (q0 + e >= next) {   // the next item (every item has >= 1 entry)
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
