// Internal definitions shared by the HIP kernels and the host library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sgsplat.h"

namespace sgs {

constexpr int kRadixBits = 8;
constexpr int kRadix = 1 << kRadixBits;
constexpr int kSortThreads = 256;
constexpr int kSortItems = 16;                       // per thread
constexpr int kSortTile = kSortThreads * kSortItems; // items per onesweep partition
constexpr int kDupChunk = 2048;                      // pairs per duplicate chunk
constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanThreads * kScanItems;
constexpr int kPreThreads = 256;
constexpr int kPreTile = 128;                        // Gaussians per forward-preprocess block
constexpr int kPersistentBlocks = 1024;              // grid of the persistent kernels
constexpr int kDepthPasses = 4;                      // 32-bit depth keys
// binning of pairs in two levels: items go to row strips of at most
// kStripTiles tiles (one wave lane per tile), then each strip's entries to
// its tiles in chunks of kBinChunk entries: one workgroup per chunk, one
// wave per sub-chunk of kBinSub entries
constexpr int kStripShift = 6;
constexpr int kStripTiles = 1 << kStripShift;
static_assert(kStripTiles == SGS_STRIP_TILES, "strip width of the ABI");
constexpr int kBinSub = 128;                         // entries per counted sub-chunk
constexpr int kBinSubs = 4;                          // sub-chunks per chunk
constexpr int kBinChunk = kBinSub * kBinSubs;        // entries per chunk
constexpr int kBinStage = 8192;                      // pairs a chunk stages in LDS (a power of two)
constexpr int kXcds = 8;                             // dies; blocks go to them round-robin

// Renumbers block b of a grid whose first `active` blocks carry work so that
// the live blocks one XCD runs (b = x, x + 8, x + 16, ... < active) take a
// contiguous range of ids; blocks from `active` on keep their ids.
// Neighbouring partitions then share that die's L2, where their partial-line
// writes (strided digit counts, short scatter runs) merge, and the live work
// stays spread over all dies.  A bijection of [0, grid size).
__device__ __forceinline__ int64_t xcd_part(uint32_t b, int64_t active) {
    if ((int64_t)b >= active) return b;
    const uint32_t A = (uint32_t)active;
    const uint32_t x = b % kXcds, i = b / kXcds, q = A / kXcds, r = A % kXcds;
    return (int64_t)x * q + (x < r ? x : r) + i;
}

// per-item 2D gradient record of the backward: d/d(u, v, Qa, Qb, Qc,
// opacity, r, g, b, z) at floats 0-9 of a 64-byte record (one cache line, so
// that a wave's nine gradient atomics for a splat land on one line)
constexpr int kG2 = 16;

// header words (u32) at workspace offset 0
enum Header : int {
    kHdrStatus = 0,
    kHdrPairs = 1,
    kHdrVisible = 2,      // items left after culling (length of the depth order)
    kHdrQueueFwd = 3,     // next heavy-first tile position of the forward blend queue
    kHdrQueueBwd = 4,     // same for the backward blend
    kHdrEntries = 5,      // (item, strip row) entries of the first binning level
    kHdrChunks = 6,       // entry chunks of the second level
    kHdrWords = 16
};

// per camera, computed on the device from the device cameras
struct CamTable {
    int32_t W, H, GX, GY, tile_base;
    int32_t strip_base;   // first global strip id: GY rows of ceil(GX / kStripTiles) strips
    int64_t pix_base;
    double limx, limy;   // guard band: guard * ((0.5 W) / fx), guard * ((0.5 H) / fy)
};

// 64-byte splat record written by the preprocess, gathered by the blends
struct __align__(16) Rec {
    float u_hi, v_hi, u_lo, v_lo;     // projected mean as float32 hi + lo parts
    float w1x, w1y, w2x, w2y;         // whitening rows: q = (w1.d)^2 + (w2.d)^2
    float opacity, r, g, b;
    float z;                          // camera depth
    uint32_t rect_x;                  // px0 | px1 << 16 (inclusive pixel rectangle)
    uint32_t rect_y;                  // py0 | py1 << 16
    int32_t radius;
};
static_assert(sizeof(Rec) == 64, "record layout");

// q = (log2 e / 2) d^T Q d, so that exp(-d^T Q d / 2) = exp2(-q)
constexpr double kHalfLog2e = 0.72134752044448170368;

struct Opts {
    int tile_w, tile_h, batch;
    int ppt, ppt_bwd;
    int schedule;        // SGS_SCHEDULE_GRID or SGS_SCHEDULE_QUEUE (resolved)
    float dilation, guard, alpha_min, alpha_max, t_min;
};

// lobe axis modes (sgs_gaussians.lobe_axes)
enum LobeMode : int { kLobesFree = SGS_LOBES_FREE, kLobesWorld = SGS_LOBES_WORLD, kLobesFrame = SGS_LOBES_FRAME };

struct Params {
    int64_t n;
    int sh_degree, n_lobes;
    int lobe_mode;          // LobeMode
    int n_axes;             // 3-vectors per Gaussian in sg_axes: K (free), 0 (world), 1 (frame)
    int sh_ad0, sh_ad1;     // adaptive SH radius thresholds; both 0 = fixed degree
    // the four colour arrays interleave in one buffer with a common stride
    // (Gaussian g's colour is one run of rec_floats at sh + g * cs_sh);
    // rec_floats may round the record up to whole 16-byte pieces when the
    // stride leaves room
    bool contig;
    int rec_floats;         // elements of the colour type per record
    int colour_type;        // ColourType of the four colour arrays (their pointers
                            // then address elements of that type; strides count them)
    const float* means;
    const float* log_scales;
    const float* quats;
    const float* opacity_logits;
    const float* sh;
    const float* sg_axes;
    const float* sg_log_sharpness;
    const float* sg_amplitudes;
    // floats from one Gaussian's block to the next in each colour array
    int64_t cs_sh, cs_ax, cs_ls, cs_am;
};

struct Workspace {
    uint32_t* header;
    CamTable* cams;
    Rec* records;
    uint32_t* depth_keys;
    uint64_t* tile_rects;
    uint32_t* sort_keys_alt;     // ping-pong for depth keys
    uint32_t* sort_keys_alt2;
    uint32_t* sorted_items;      // final depth order
    uint32_t* sorted_items_alt;
    uint32_t* pair_offsets;
    uint32_t* chunk_start;       // first sorted position of every duplicate chunk
    uint32_t* pair_tiles;
    uint32_t* pair_values;
    uint32_t* pair_tiles_alt;
    uint32_t* pair_values_alt;
    uint32_t* ranges;
    uint32_t* strip_ranges;      // [start, end) of every strip's entries (first level)
    uint4* strip_info;           // per strip: first chunk, chunks, first tile, width | x0 << 16
    uint4* chunk_info;           // per chunk: first entry, end entry, first tile, width | x0 << 16
    uint16_t* chunk_counts;      // per sub-chunk: pairs of each of its strip's tiles
    uint32_t* chunk_offsets;     // per sub-chunk: pairs of the strip's earlier sub-chunks, per tile
    uint32_t* tile_count;        // pairs per tile
    uint32_t* tile_start;        // first pair position of each tile
    uint32_t* tile_keys;         // heavy-first sort key of every tile
    uint32_t* tile_order;        // tiles by decreasing list length (stable)
    float* grad2d;
    float* gx_colour;            // [3][n]: mean gradient through the view direction
    uint32_t* counts;            // radix pass: [256][partitions] digit counts -> offsets
    uint32_t* totals;            // radix pass: [256] digit totals
    uint32_t* pair_counts;       // pairs of each item, in depth order
    uint64_t* sorted_rects;      // tile rectangle of each item, in depth order
    uint64_t* scan_sums;         // per scan block
    double* loss_partial;
    int64_t n_items, n_tiles, n_pixels, capacity;
    int64_t n_strips, chunk_cap;     // strips; chunk table capacity
    int n_cams;
    int cus;                         // compute units of the device (persistent grids)
    int64_t depth_parts, pair_parts, scan_parts, dup_chunks;
    int dup_blocks;              // grid of the duplicate kernel (one block per chunk)
    int strip_passes, strip_bits;
    bool key16;                  // entry strip ids stored as u16 (at most 65536 strips)
};

// the fused Adam step: one entry per parameter array, in sgs_gaussians order
constexpr int kAdamArrays = 8;
struct AdamArrays {
    float* p[kAdamArrays];
    const float* g[kAdamArrays];
    float* m[kAdamArrays];
    float* v[kAdamArrays];
    int64_t count[kAdamArrays];    // elements (packed)
    int64_t width[kAdamArrays];    // floats per Gaussian on the packed side (count: one flat run)
    int64_t pstride[kAdamArrays];  // floats per Gaussian on the parameter side (== width: packed)
    float lr[kAdamArrays];
    float c1[kAdamArrays];         // 1 / (1 - b1^t)
    float c2[kAdamArrays];         // 1 / (1 - b2^t)
    bool on[kAdamArrays];
    float b1, b2, eps;
    float ob1, ob2;                // 1 - b1, 1 - b2, formed in float64 then rounded
};

// launchers (defined in the .hip files)
void launch_adam(const AdamArrays& a, hipStream_t s);
void launch_setup(const Workspace& ws, const sgs_camera* dev_cams, int n_cams, int tile_w, int tile_h,
                  float guard, hipStream_t s);
void launch_preprocess(const Params& p, const sgs_camera* dev_cams, int n_cams, const Opts& o,
                       const Workspace& ws, int hist_blocks, hipStream_t s);
// One stable pass over the digit (key >> shift) & 255.  With `drop_culled`,
// keys equal to 0xFFFFFFFF are removed and the number of kept items is
// written to *kept_out.  digit_bits < 8 declares that the key has no set
// bits above shift + digit_bits (fewer ballots in the ranking).  counted:
// the digit counts of every half partition (kSortTile / 2 items) are already
// in counts[d * 2 parts + h]; the pass then skips its upsweep.  ranges: the
// pass is the last of a tile sort; the tile ranges (cleared beforehand) are
// written from the key changes of its sorted output.
void launch_radix_pass(const uint32_t* keys_in, const uint32_t* vals_in, uint32_t* keys_out,
                       uint32_t* vals_out, const uint32_t* count_ptr, int64_t count_host, int shift,
                       uint32_t* counts, uint32_t* totals, int64_t parts, const uint64_t* rects,
                       uint32_t* pairs_out, uint64_t* rects_out, int64_t n_rects, bool drop_culled,
                       uint32_t* kept_out, hipStream_t s, int digit_bits = kRadixBits,
                       bool counted = false, uint32_t* ranges = nullptr, int64_t n_tiles = 0);
void launch_radix_pass16(const uint16_t* keys_in, const uint32_t* vals_in, uint16_t* keys_out,
                         uint32_t* vals_out, const uint32_t* count_ptr, int64_t count_host, int shift,
                         uint32_t* counts, uint32_t* totals, int64_t parts, hipStream_t s,
                         int digit_bits = kRadixBits, bool counted = false,
                         uint32_t* ranges = nullptr, int64_t n_tiles = 0);
void launch_scan_pairs(const Workspace& ws, hipStream_t s);
void launch_duplicate_counts(const Workspace& ws, int64_t n, hipStream_t s);
// the first tile pass fused with pair generation: scans the duplicate's
// counts, ranks and scatters into (keys_out, vals_out); ranges when it is
// also the last pass
void launch_dup_scatter(const Workspace& ws, int64_t n, uint32_t* keys_out, uint32_t* vals_out,
                        int64_t parts, int digit_bits, uint32_t* ranges, int64_t pair_capacity,
                        hipStream_t s);
// second binning level: the strip-sorted entries (values: positions in the
// depth order) -> pair_values in (tile, depth) order, tile_count, tile_start
// and the tile ranges; pairs past the capacity are dropped
void launch_bin_tiles(const Workspace& ws, const uint32_t* entry_slots, hipStream_t s);
// tile_order = tiles sorted by decreasing list length (one stable 8-bit pass
// over a log-scale length bucket)
void launch_tile_order(const Workspace& ws, int64_t parts, hipStream_t s);
// `queue`: persistent workgroups over tile_order (requires launch_tile_order
// after the ranges of the same forward); otherwise one workgroup per tile
void launch_blend_fwd(const Workspace& ws, const sgs_camera* dev_cams, int n_cams, const Opts& o,
                      const sgs_outputs& out, bool queue, hipStream_t s);
void launch_blend_count(const Workspace& ws, const sgs_camera* dev_cams, int n_cams, const Opts& o,
                        uint64_t* counts, hipStream_t s);
// the backward walk of a finished forward, counting its work events into
// counts[4] (visited, evaluated, blended, reductions); no gradient written
void launch_blend_bwd_count(const Workspace& ws, const sgs_camera* dev_cams, int n_cams,
                            const Opts& o, const sgs_outputs& fwd, uint64_t* counts,
                            hipStream_t s);
// grad_depth / grad_alpha may be NULL (no upstream gradient); with either,
// the blend also adds dL/dz into grad2d row 9
void launch_blend_bwd(const Workspace& ws, const sgs_camera* dev_cams, int n_cams, const Opts& o,
                      const sgs_outputs& fwd, const float* grad_image, const float* grad_depth,
                      const float* grad_alpha, bool queue, hipStream_t s);
// depth_grad: grad2d row 9 (dL/dz per item) holds the depth term
void launch_preprocess_bwd(const Params& p, const sgs_camera* dev_cams, int n_cams, const Opts& o,
                           const Workspace& ws, const sgs_grads& gr, bool depth_grad,
                           hipStream_t s);
void launch_l1(const Workspace& ws, int n_cams, const float* image, const float* target,
               float* grad, double* loss, hipStream_t s);
void launch_read_keys(const Workspace& ws, int64_t count, uint64_t* keys, hipStream_t s);
void launch_fill_u32(uint32_t* p, uint32_t v, int64_t count, hipStream_t s);
// zeroes the 2D gradient records of the visible items
void launch_clear_grad2d(const Workspace& ws, hipStream_t s);

}  // namespace sgs
