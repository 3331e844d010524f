// C-ABI entry points: argument checks, workspace layout, launch sequence.
#include <string.h>

#include <cmath>

#include <array>
#include <atomic>
#include <string>
#include <vector>

#include "common.hpp"

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

#define SGS_HIP(x)                                                                       \
    do {                                                                                 \
        hipError_t e_ = (x);                                                             \
        if (e_ != hipSuccess) return fail(SGS_E_HIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define SGS_LAUNCHED()                                                                   \
    do {                                                                                 \
        hipError_t e_ = hipGetLastError();                                               \
        if (e_ != hipSuccess) return fail(SGS_E_HIP, std::string("kernel launch: ") + hipGetErrorString(e_)); \
    } while (0)

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

struct Plan {
    sgs_layout lay;
    sgs::Opts o;
    int64_t n;
    int n_cams;
    int strip_passes, strip_bits;
    int64_t n_strips, chunk_cap;
    int64_t depth_parts, pair_parts, scan_parts, dup_chunks;
    int pre_blocks, dup_blocks;
    int64_t max_parts;
    // offsets not exported in sgs_layout
    size_t sorted_rects, sort_keys_alt, sort_keys_alt2, sorted_items_alt, chunk_start, pair_tiles_alt,
        pair_values_alt, counts, totals, pair_counts, scan_sums, loss_partial, gx_colour,
        tile_keys, tile_order, strip_ranges, strip_info, chunk_info, chunk_counts, chunk_offsets,
        tile_count, tile_start;
    int64_t tile_parts;   // partitions of the heavy-first tile sort
    // the blends run the queue schedule: requested, and the forward builds
    // the tile order (it does when there are Gaussians and pair capacity)
    bool queue;
};

bool tile_shape_ok(int tw, int th) {
    return (tw == 16 && th == 16) || (tw == 8 && th == 8) || (tw == 16 && th == 8) ||
           (tw == 8 && th == 16) || (tw == 32 && th == 8);
}

int plan(const sgs_gaussians* g, const sgs_camera* cams, int32_t n_cams, const sgs_options* oin,
         int64_t cap, Plan* pl) {
    if (!g) return fail(SGS_E_INVALID, "gaussians is NULL");
    if (g->n < 0) return fail(SGS_E_INVALID, "n < 0");
    if (g->sh_degree < 0 || g->sh_degree > SGS_MAX_SH_DEGREE)
        return fail(SGS_E_INVALID, "sh_degree must be 0..3");
    if (g->n_lobes < 0 || g->n_lobes > SGS_MAX_LOBES)
        return fail(SGS_E_INVALID, "n_lobes must be 0..8");
    if (g->lobe_axes != SGS_LOBES_FREE && g->lobe_axes != SGS_LOBES_WORLD &&
        g->lobe_axes != SGS_LOBES_FRAME)
        return fail(SGS_E_INVALID, "lobe_axes must be SGS_LOBES_FREE, _WORLD or _FRAME");
    if (g->lobe_axes != SGS_LOBES_FREE && g->n_lobes != 3)
        return fail(SGS_E_INVALID, "the orthogonal lobe modes take exactly 3 lobes");
    if (g->sh_adaptive[0] < 0 || g->sh_adaptive[1] < g->sh_adaptive[0])
        return fail(SGS_E_INVALID, "sh_adaptive must satisfy 0 <= [0] <= [1]");
    if (g->colour_dtype != SGS_COLOUR_F32 && g->colour_dtype != SGS_COLOUR_BF16 &&
        g->colour_dtype != SGS_COLOUR_F16)
        return fail(SGS_E_INVALID, "colour_dtype must be SGS_COLOUR_F32, _BF16 or _F16");
    if (g->colour_dtype != SGS_COLOUR_F32 && (g->sh_adaptive[0] | g->sh_adaptive[1]) != 0)
        return fail(SGS_E_INVALID, "half-precision colour storage needs a fixed SH degree");
    if (!cams) return fail(SGS_E_INVALID, "host cameras are NULL");
    if (n_cams < 1 || n_cams > SGS_MAX_CAMERAS) return fail(SGS_E_INVALID, "n_cams must be 1..1024");
    if (cap < 0 || cap >= (int64_t(1) << 30)) return fail(SGS_E_INVALID, "pair_capacity must be in [0, 2^30)");
    sgs::Opts o;
    o.tile_w = oin && oin->tile_w ? oin->tile_w : 16;
    o.tile_h = oin && oin->tile_h ? oin->tile_h : 16;
    if (!tile_shape_ok(o.tile_w, o.tile_h))
        return fail(SGS_E_INVALID, "tile shape must be 16x16, 8x8, 16x8, 8x16 or 32x8");
    const int nt = o.tile_w * o.tile_h;
    // pixels per thread: the block (nt / ppt threads) must be whole waves
    auto ppt_ok = [&](int ppt) {
        if (ppt != 1 && ppt != 2 && ppt != 4) return false;
        if (o.tile_h % ppt != 0 || (nt / ppt) % 64 != 0) return false;
        return !(o.tile_w == 8 && o.tile_h == 8 && ppt != 1) &&
               !((o.tile_w == 16 && o.tile_h == 8) && ppt == 4) &&
               !((o.tile_w == 8 && o.tile_h == 16) && ppt == 4);
    };
    o.ppt = oin && oin->pixels_per_thread ? oin->pixels_per_thread : (ppt_ok(2) ? 2 : 1);
    o.ppt_bwd = oin && oin->pixels_per_thread_bwd ? oin->pixels_per_thread_bwd
                                                   : (ppt_ok(4) ? 4 : (ppt_ok(2) ? 2 : 1));
    if (!ppt_ok(o.ppt) || !ppt_ok(o.ppt_bwd))
        return fail(SGS_E_INVALID, "pixels_per_thread must be 1, 2 or 4 with tile_w*tile_h/ppt a "
                                   "multiple of 64");
    o.batch = oin && oin->batch ? oin->batch : 128;
    if (o.batch < 64 || o.batch % 64 != 0 || o.batch > 1024)
        return fail(SGS_E_INVALID, "batch must be a multiple of 64 in [64, 1024]");
    o.schedule = oin && oin->schedule ? oin->schedule
                                      : (n_cams > 1 ? SGS_SCHEDULE_QUEUE : SGS_SCHEDULE_GRID);
    if (o.schedule != SGS_SCHEDULE_GRID && o.schedule != SGS_SCHEDULE_QUEUE &&
        o.schedule != SGS_SCHEDULE_SLICES)
        return fail(SGS_E_INVALID, "schedule must be 0, SGS_SCHEDULE_GRID, _QUEUE or _SLICES");
    o.dilation = oin && oin->dilation != 0.0f ? oin->dilation : 0.3f;
    o.guard = oin && oin->guard != 0.0f ? oin->guard : 1.3f;
    o.alpha_min = oin && oin->alpha_min != 0.0f ? oin->alpha_min : 1.0f / 255.0f;
    o.alpha_max = oin && oin->alpha_max != 0.0f ? oin->alpha_max : 0.99f;
    o.t_min = oin && oin->t_min != 0.0f ? oin->t_min : 1e-4f;
    if (!(o.alpha_max > 0.0f && o.alpha_max < 1.0f))
        return fail(SGS_E_INVALID, "alpha_max must be in (0, 1)");
    int64_t tiles = 0, pixels = 0, strips = 0;
    for (int c = 0; c < n_cams; ++c) {
        const int W = cams[c].width, H = cams[c].height;
        if (W < 1 || H < 1 || W > SGS_MAX_IMAGE_SIDE || H > SGS_MAX_IMAGE_SIDE)
            return fail(SGS_E_INVALID, "camera width/height must be 1..32767");
        // a non-positive near plane would let depths in (znear, 0] through the
        // 1/z projection (negative depth keys sort behind every positive one)
        if (!(std::isfinite(cams[c].znear) && cams[c].znear > 0.0f))
            return fail(SGS_E_INVALID, "camera znear must be finite and > 0");
        if (!(std::isfinite(cams[c].fx) && cams[c].fx > 0.0f && std::isfinite(cams[c].fy) &&
              cams[c].fy > 0.0f))
            return fail(SGS_E_INVALID, "camera fx and fy must be finite and > 0");
        tiles += cdiv(W, o.tile_w) * cdiv(H, o.tile_h);
        strips += cdiv(H, o.tile_h) * cdiv(cdiv(W, o.tile_w), sgs::kStripTiles);
        pixels += (int64_t)W * H;
    }
    const int64_t n = g->n;
    const int64_t items = n * n_cams;
    if (items >= (int64_t(1) << 30)) return fail(SGS_E_INVALID, "n * n_cams must be < 2^30");
    if (tiles >= (int64_t(1) << 31)) return fail(SGS_E_INVALID, "too many tiles");

    pl->o = o;
    pl->n = n;
    pl->n_cams = n_cams;
    // the first binning level sorts (strip, item) entries by strip id
    int bits = 1;
    while ((int64_t(1) << bits) < strips) ++bits;
    pl->strip_bits = bits;
    pl->strip_passes = (bits + sgs::kRadixBits - 1) / sgs::kRadixBits;
    pl->n_strips = strips;
    // every chunk but a strip's last holds kBinChunk entries, and there are
    // at most as many entries as pairs
    pl->chunk_cap = cdiv(cap, sgs::kBinChunk) + strips;
    pl->depth_parts = cdiv(items, sgs::kSortTile);
    pl->pair_parts = cdiv(cap, sgs::kSortTile);
    pl->scan_parts = cdiv(items, sgs::kScanTile);
    pl->dup_chunks = cdiv(cap, sgs::kDupChunk);
    int64_t pb = cdiv(n, sgs::kPreThreads);
    pl->pre_blocks = (int)(pb < 1 ? 1 : (pb > sgs::kPersistentBlocks ? sgs::kPersistentBlocks : pb));
    int64_t db = pl->dup_chunks;
    // one block per chunk: a chunk's work is a short chain of dependent loads,
    // so many blocks in flight hide it better than a persistent loop
    pl->dup_blocks = (int)(db < 1 ? 1 : (db > (1 << 30) ? (1 << 30) : db));
    pl->tile_parts = cdiv(tiles, sgs::kSortTile);
    pl->max_parts = pl->depth_parts > pl->pair_parts ? pl->depth_parts : pl->pair_parts;
    if (pl->tile_parts > pl->max_parts) pl->max_parts = pl->tile_parts;
    if (2 * pl->pair_parts > pl->max_parts) pl->max_parts = 2 * pl->pair_parts;   // duplicate's counts
    // the queue and slice schedules pop items over the heavy-first tile order
    pl->queue = (o.schedule == SGS_SCHEDULE_QUEUE || o.schedule == SGS_SCHEDULE_SLICES) && n > 0 &&
                cap > 0;

    sgs_layout& L = pl->lay;
    memset(&L, 0, sizeof(L));
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off = align_up(off + bytes);
        return at;
    };
    // header, loss partials and camera table first: their offsets depend on
    // n_cams only, so render_l1 can find them from the cameras alone
    L.header = take(sgs::kHdrWords * 4);
    pl->loss_partial = take(1024 * 8);
    L.cam_table = take((size_t)n_cams * sizeof(sgs::CamTable));
    L.records = take((size_t)items * sizeof(sgs::Rec));
    L.depth_keys = take((size_t)items * 4);
    L.tile_rects = take((size_t)items * 8);
    pl->sort_keys_alt = take((size_t)items * 4);
    pl->sort_keys_alt2 = take((size_t)items * 4);
    L.sorted_items = take((size_t)items * 4);
    pl->sorted_items_alt = take((size_t)items * 4);
    L.pair_offsets = take((size_t)(items + 1) * 4);
    pl->chunk_start = take((size_t)(pl->dup_chunks + 1) * 4);
    L.pair_tiles = take((size_t)cap * 4);
    L.pair_values = take((size_t)cap * 4);
    pl->pair_tiles_alt = take((size_t)cap * 4);
    pl->pair_values_alt = take((size_t)cap * 4);
    L.ranges = take((size_t)tiles * 8);
    pl->tile_keys = take((size_t)tiles * 4);
    pl->tile_order = take((size_t)tiles * 4);
    L.grad2d = take((size_t)items * sgs::kG2 * 4);
    pl->gx_colour = take((size_t)n * 3 * 4);
    pl->counts = take((size_t)pl->max_parts * sgs::kRadix * 4);
    pl->totals = take((size_t)sgs::kRadix * 4);
    pl->pair_counts = take((size_t)items * 4);
    pl->sorted_rects = take((size_t)items * 8);
    pl->scan_sums = take((size_t)(pl->scan_parts + 1) * 16);   // entry sums, then pair sums
    // second binning level (after the sections above, whose offsets then do
    // not move with the pair capacity's chunk tables)
    pl->strip_ranges = take((size_t)strips * 8);
    pl->strip_info = take((size_t)strips * 16);
    pl->tile_count = take((size_t)tiles * 4);
    pl->tile_start = take((size_t)tiles * 4);
    pl->chunk_info = take((size_t)pl->chunk_cap * 16);
    pl->chunk_counts = take((size_t)pl->chunk_cap * sgs::kBinSubs * sgs::kStripTiles * 2);
    pl->chunk_offsets = take((size_t)pl->chunk_cap * sgs::kBinSubs * sgs::kStripTiles * 4);
    L.total_bytes = off;
    L.n_items = items;
    L.n_tiles = tiles;
    L.n_pixels = pixels;
    L.pair_capacity = cap;
    L.n_strips = strips;
    return SGS_OK;
}

// compute units of the current device, queried once per device
int device_cus() {
    static std::atomic<int> cache[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    int v = cache[dev].load();
    if (v > 0) return v;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0)
        v = 256;
    cache[dev].store(v);
    return v;
}

sgs::Workspace bind(const Plan& pl, void* base) {
    char* b = static_cast<char*>(base);
    const sgs_layout& L = pl.lay;
    sgs::Workspace w;
    w.header = reinterpret_cast<uint32_t*>(b + L.header);
    w.cams = reinterpret_cast<sgs::CamTable*>(b + L.cam_table);
    w.records = reinterpret_cast<sgs::Rec*>(b + L.records);
    w.depth_keys = reinterpret_cast<uint32_t*>(b + L.depth_keys);
    w.tile_rects = reinterpret_cast<uint64_t*>(b + L.tile_rects);
    w.sort_keys_alt = reinterpret_cast<uint32_t*>(b + pl.sort_keys_alt);
    w.sort_keys_alt2 = reinterpret_cast<uint32_t*>(b + pl.sort_keys_alt2);
    w.sorted_items = reinterpret_cast<uint32_t*>(b + L.sorted_items);
    w.sorted_items_alt = reinterpret_cast<uint32_t*>(b + pl.sorted_items_alt);
    w.pair_offsets = reinterpret_cast<uint32_t*>(b + L.pair_offsets);
    w.chunk_start = reinterpret_cast<uint32_t*>(b + pl.chunk_start);
    w.pair_tiles = reinterpret_cast<uint32_t*>(b + L.pair_tiles);
    w.pair_values = reinterpret_cast<uint32_t*>(b + L.pair_values);
    w.pair_tiles_alt = reinterpret_cast<uint32_t*>(b + pl.pair_tiles_alt);
    w.pair_values_alt = reinterpret_cast<uint32_t*>(b + pl.pair_values_alt);
    w.ranges = reinterpret_cast<uint32_t*>(b + L.ranges);
    w.strip_ranges = reinterpret_cast<uint32_t*>(b + pl.strip_ranges);
    w.strip_info = reinterpret_cast<uint4*>(b + pl.strip_info);
    w.chunk_info = reinterpret_cast<uint4*>(b + pl.chunk_info);
    w.chunk_counts = reinterpret_cast<uint16_t*>(b + pl.chunk_counts);
    w.chunk_offsets = reinterpret_cast<uint32_t*>(b + pl.chunk_offsets);
    w.tile_count = reinterpret_cast<uint32_t*>(b + pl.tile_count);
    w.tile_start = reinterpret_cast<uint32_t*>(b + pl.tile_start);
    w.tile_keys = reinterpret_cast<uint32_t*>(b + pl.tile_keys);
    w.tile_order = reinterpret_cast<uint32_t*>(b + pl.tile_order);
    w.grad2d = reinterpret_cast<float*>(b + L.grad2d);
    w.gx_colour = reinterpret_cast<float*>(b + pl.gx_colour);
    w.counts = reinterpret_cast<uint32_t*>(b + pl.counts);
    w.totals = reinterpret_cast<uint32_t*>(b + pl.totals);
    w.pair_counts = reinterpret_cast<uint32_t*>(b + pl.pair_counts);
    w.sorted_rects = reinterpret_cast<uint64_t*>(b + pl.sorted_rects);
    w.scan_sums = reinterpret_cast<uint64_t*>(b + pl.scan_sums);
    w.loss_partial = reinterpret_cast<double*>(b + pl.loss_partial);
    w.n_items = L.n_items;
    w.n_tiles = L.n_tiles;
    w.n_pixels = L.n_pixels;
    w.capacity = L.pair_capacity;
    w.depth_parts = pl.depth_parts;
    w.pair_parts = pl.pair_parts;
    w.scan_parts = pl.scan_parts;
    w.dup_chunks = pl.dup_chunks;
    w.dup_blocks = pl.dup_blocks;
    w.strip_passes = pl.strip_passes;
    w.strip_bits = pl.strip_bits;
    w.n_strips = pl.n_strips;
    w.chunk_cap = pl.chunk_cap;
    w.n_cams = pl.n_cams;
    w.cus = device_cus();
    w.key16 = pl.n_strips <= 65536;
    return w;
}

// 3-vectors per Gaussian in sg_axes for the lobe mode
int axis_rows(const sgs_gaussians* g) {
    return g->lobe_axes == SGS_LOBES_FREE ? g->n_lobes : (g->lobe_axes == SGS_LOBES_FRAME ? 1 : 0);
}

sgs::Params params_of(const sgs_gaussians* g) {
    sgs::Params p;
    p.n = g->n;
    p.sh_degree = g->sh_degree;
    p.n_lobes = g->n_lobes;
    p.lobe_mode = g->lobe_axes;
    p.n_axes = axis_rows(g);
    p.sh_ad0 = g->sh_adaptive[0];
    p.sh_ad1 = g->sh_adaptive[1];
    p.means = g->means;
    p.log_scales = g->log_scales;
    p.quats = g->quats;
    p.opacity_logits = g->opacity_logits;
    p.sh = g->sh;
    p.sg_axes = g->sg_axes;
    p.sg_log_sharpness = g->sg_log_sharpness;
    p.sg_amplitudes = g->sg_amplitudes;
    const int64_t nc3 = 3 * (int64_t)(g->sh_degree + 1) * (g->sh_degree + 1), K = g->n_lobes;
    const int64_t A3 = 3 * (int64_t)p.n_axes;
    const int64_t cs = g->colour_stride;
    p.cs_sh = cs > 0 ? cs : nc3;
    p.cs_ax = cs > 0 ? cs : A3;
    p.cs_ls = cs > 0 ? cs : K;
    p.cs_am = cs > 0 ? cs : 3 * K;
    const int64_t rs = nc3 + A3 + 4 * K;
    p.colour_type = g->colour_dtype;
    // bytes per colour element, and elements per 16-byte piece
    const int64_t E = g->colour_dtype == SGS_COLOUR_F32 ? 4 : 2, W16 = 16 / E;
    const char* sh = reinterpret_cast<const char*>(g->sh);
    // the four arrays interleave: one run of rs elements per Gaussian
    p.contig = cs > 0 && (A3 == 0 || reinterpret_cast<const char*>(g->sg_axes) == sh + nc3 * E) &&
               (K == 0 || (reinterpret_cast<const char*>(g->sg_log_sharpness) == sh + (nc3 + A3) * E &&
                           reinterpret_cast<const char*>(g->sg_amplitudes) == sh + (nc3 + A3 + K) * E));
    p.rec_floats = (int)rs;
    // read whole 16-byte pieces when the stride leaves room for the rounding
    const int64_t rs16 = (rs + W16 - 1) / W16 * W16;
    if (p.contig && cs % W16 == 0 && cs >= rs16 && ((uintptr_t)g->sh & 15u) == 0)
        p.rec_floats = (int)rs16;
    return p;
}

int check_params(const sgs_gaussians* g) {
    if (g->n == 0) return SGS_OK;
    if (!g->means || !g->log_scales || !g->quats || !g->opacity_logits || !g->sh)
        return fail(SGS_E_INVALID, "a Gaussian parameter array is NULL");
    if (g->n_lobes > 0 && (!g->sg_log_sharpness || !g->sg_amplitudes))
        return fail(SGS_E_INVALID, "an SG lobe array is NULL");
    if (axis_rows(g) > 0 && !g->sg_axes) return fail(SGS_E_INVALID, "sg_axes is NULL");
    const int64_t nc3 = 3 * (int64_t)(g->sh_degree + 1) * (g->sh_degree + 1);
    if (g->colour_stride < 0 ||
        (g->colour_stride > 0 && (g->colour_stride < nc3 || g->colour_stride < 3 * (int64_t)g->n_lobes ||
                                  g->colour_stride < 3 * (int64_t)axis_rows(g))))
        return fail(SGS_E_INVALID, "colour_stride is below a colour block size");
    return SGS_OK;
}

// ---- stage timing (HIP events between stages, collected on query) ----
constexpr int kFwdEvents = 9;   // 8 forward stages
constexpr int kBwdEvents = 4;   // 3 backward stages
constexpr size_t kMaxTimedCalls = 4096;
const char* const kStageNames[SGS_N_STAGES] = {
    "fwd.setup", "fwd.preprocess", "fwd.depth_sort", "fwd.pair_scan", "fwd.duplicate",
    "fwd.tile_sort", "fwd.tile_order", "fwd.blend", "bwd.clear", "bwd.blend", "bwd.preprocess"};

struct Timing {
    bool on = false;
    std::vector<std::array<hipEvent_t, kFwdEvents>> fwd;
    std::vector<std::array<hipEvent_t, kBwdEvents>> bwd;
    size_t fwd_used = 0, bwd_used = 0;
};
Timing g_timing;

template <size_t E>
hipEvent_t* timing_slot(std::vector<std::array<hipEvent_t, E>>& v, size_t& used) {
    if (!g_timing.on || used >= kMaxTimedCalls) return nullptr;
    if (used == v.size()) {
        std::array<hipEvent_t, E> a;
        for (size_t i = 0; i < E; ++i)
            if (hipEventCreate(&a[i]) != hipSuccess) return nullptr;
        v.push_back(a);
    }
    return v[used++].data();
}

struct Marker {
    hipEvent_t* ev;
    hipStream_t s;
    void mark(int i) {
        if (ev) (void)hipEventRecord(ev[i], s);
    }
};

}  // namespace

extern "C" {

size_t render_workspace_bytes(const sgs_gaussians* g, const sgs_camera* host_cams, int32_t n_cams,
                              const sgs_options* opts, int64_t pair_capacity) {
    Plan pl;
    if (plan(g, host_cams, n_cams, opts, pair_capacity, &pl) != SGS_OK) return 0;
    return pl.lay.total_bytes;
}

int render_layout(const sgs_gaussians* g, const sgs_camera* host_cams, int32_t n_cams,
                  const sgs_options* opts, int64_t pair_capacity, sgs_layout* out) {
    if (!out) return fail(SGS_E_INVALID, "layout output is NULL");
    Plan pl;
    const int rc = plan(g, host_cams, n_cams, opts, pair_capacity, &pl);
    if (rc != SGS_OK) return rc;
    *out = pl.lay;
    return SGS_OK;
}

}  // extern "C"

namespace {

// The forward behind render_forward and render_forward_noalloc.  `timed`:
// record stage events when stage timing is on (creating events allocates,
// which the no-allocation entry point must not do).
int forward_impl(const sgs_gaussians* g, const sgs_camera* host_cams, const sgs_camera* dev_cams,
                 int32_t n_cams, const sgs_options* opts, void* workspace, size_t workspace_bytes,
                 int64_t pair_capacity, const sgs_outputs* outs, int32_t flags,
                 int64_t* pairs_needed, void* stream, bool timed) {
    Plan pl;
    int rc = plan(g, host_cams, n_cams, opts, pair_capacity, &pl);
    if (rc != SGS_OK) return rc;
    if ((rc = check_params(g)) != SGS_OK) return rc;
    if (!dev_cams) return fail(SGS_E_INVALID, "device cameras are NULL");
    if (!workspace) return fail(SGS_E_INVALID, "workspace is NULL");
    if (workspace_bytes < pl.lay.total_bytes) return fail(SGS_E_INVALID, "workspace too small");
    if (!outs || !outs->image || !outs->final_T || !outs->n_contrib)
        return fail(SGS_E_INVALID, "image, final_T and n_contrib outputs are required");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const sgs::Workspace ws = bind(pl, workspace);
    const sgs::Params p = params_of(g);
    const sgs::Opts& o = pl.o;
    (void)hipGetLastError();
    Marker mk{timed ? timing_slot(g_timing.fwd, g_timing.fwd_used) : nullptr, s};

    mk.mark(0);
    sgs::launch_setup(ws, dev_cams, n_cams, o.tile_w, o.tile_h, o.guard, s);   // clears too
    SGS_LAUNCHED();
    mk.mark(1);
    if (pl.n > 0) {
        sgs::launch_preprocess(p, dev_cams, n_cams, o, ws, pl.pre_blocks, s);
        SGS_LAUNCHED();
        mk.mark(2);
        // depth sort of the items: 4 passes, final order in sorted_items; the
        // last pass also lists each item's pair count in sorted order
        const uint32_t* kin[4] = {ws.depth_keys, ws.sort_keys_alt, ws.sort_keys_alt2, ws.sort_keys_alt};
        const uint32_t* vin[4] = {nullptr, ws.sorted_items_alt, ws.sorted_items, ws.sorted_items_alt};
        uint32_t* kout[4] = {ws.sort_keys_alt, ws.sort_keys_alt2, ws.sort_keys_alt, nullptr};
        uint32_t* vout[4] = {ws.sorted_items_alt, ws.sorted_items, ws.sorted_items_alt, ws.sorted_items};
        for (int ps = 0; ps < sgs::kDepthPasses; ++ps) {
            const bool first = ps == 0, last = ps == sgs::kDepthPasses - 1;
            sgs::launch_radix_pass(kin[ps], vin[ps], kout[ps], vout[ps],
                                   first ? nullptr : ws.header + sgs::kHdrVisible, ws.n_items,
                                   ps * sgs::kRadixBits, ws.counts, ws.totals, pl.depth_parts,
                                   last ? ws.tile_rects : nullptr, last ? ws.pair_counts : nullptr,
                                   last ? ws.sorted_rects : nullptr, ws.n_items, first,
                                   ws.header + sgs::kHdrVisible, s);
        }
        SGS_LAUNCHED();
        mk.mark(3);
        sgs::launch_scan_pairs(ws, s);
        SGS_LAUNCHED();
    } else {
        mk.mark(2);
        mk.mark(3);
    }
    mk.mark(4);
    if (flags & SGS_FLAG_CHECK_CAPACITY) {
        uint32_t h[2] = {0, 0};
        SGS_HIP(hipMemcpyAsync(h, ws.header, 8, hipMemcpyDeviceToHost, s));
        SGS_HIP(hipStreamSynchronize(s));
        const uint32_t P = h[sgs::kHdrPairs];
        if (pairs_needed) *pairs_needed = P;
        if (h[sgs::kHdrStatus] & SGS_STATUS_CAMERAS)
            return fail(SGS_E_INVALID, "device cameras disagree with the host cameras' sizes");
        if ((int64_t)P > pair_capacity) {
            if (mk.ev) --g_timing.fwd_used;
            return fail(SGS_E_CAPACITY, "pair capacity " + std::to_string(pair_capacity) +
                                            " < " + std::to_string(P) + " pairs");
        }
    }
    if (pl.n > 0 && pair_capacity > 0) {
        // first level: the duplicate counts the first strip digit of every
        // chunk; the first strip pass generates the entries again and
        // scatters them directly.  The last strip pass leaves the entries in
        // the alternate pair buffers and writes the strip ranges.
        sgs::launch_duplicate_counts(ws, pl.n, s);
        SGS_LAUNCHED();
        mk.mark(5);
        const int L = pl.strip_passes;
        auto out_t = [&](int ps) { return (L - 1 - ps) % 2 == 0 ? ws.pair_tiles_alt : ws.pair_tiles; };
        auto out_v = [&](int ps) { return (L - 1 - ps) % 2 == 0 ? ws.pair_values_alt : ws.pair_values; };
        {
            const int nb = pl.strip_bits < sgs::kRadixBits ? pl.strip_bits : sgs::kRadixBits;
            sgs::launch_dup_scatter(ws, pl.n, out_t(0), out_v(0), pl.pair_parts, nb,
                                    L == 1 ? ws.strip_ranges : nullptr, pair_capacity, s);
        }
        for (int ps = 1; ps < L; ++ps) {
            // strip ids are below 2^strip_bits: the last pass has fewer digit bits
            const int left = pl.strip_bits - ps * sgs::kRadixBits;
            const int nb = left < sgs::kRadixBits ? left : sgs::kRadixBits;
            uint32_t* rng = ps == L - 1 ? ws.strip_ranges : nullptr;
            uint32_t *ti = out_t(ps - 1), *vi = out_v(ps - 1), *to = out_t(ps), *vo = out_v(ps);
            if (ws.key16)
                sgs::launch_radix_pass16(reinterpret_cast<const uint16_t*>(ti), vi,
                                         reinterpret_cast<uint16_t*>(to), vo,
                                         ws.header + sgs::kHdrEntries, pair_capacity,
                                         ps * sgs::kRadixBits, ws.counts, ws.totals, pl.pair_parts, s,
                                         nb, false, rng, ws.n_strips);
            else
                sgs::launch_radix_pass(ti, vi, to, vo, ws.header + sgs::kHdrEntries, pair_capacity,
                                       ps * sgs::kRadixBits, ws.counts, ws.totals, pl.pair_parts,
                                       nullptr, nullptr, nullptr, 0, false, nullptr, s, nb, false,
                                       rng, ws.n_strips);
        }
        // second level: each strip's entries -> its tiles' pairs, in place
        sgs::launch_bin_tiles(ws, ws.pair_values_alt, s);
        SGS_LAUNCHED();
        mk.mark(6);
        if (pl.queue) sgs::launch_tile_order(ws, pl.tile_parts, s);
        SGS_LAUNCHED();
    } else {
        mk.mark(5);
        mk.mark(6);
    }
    mk.mark(7);
    sgs::launch_blend_fwd(ws, dev_cams, n_cams, o, *outs, pl.queue, s);
    SGS_LAUNCHED();
    mk.mark(8);
    return SGS_OK;
}

// Workspace of render_forward_noalloc: one array per device, reserved when
// the code object is loaded and held until the process ends.  Host code
// never passes `scratch` itself (on the host it names a stand-in, not
// device memory): it uses the device address from hipGetSymbolAddress,
// taken once per device.
__device__ __align__(256) unsigned char scratch[SGS_NOALLOC_WORKSPACE_BYTES];
constexpr int kMaxDevices = 64;
std::atomic<void*> g_scratch[kMaxDevices];

}  // namespace

extern "C" {

int render_forward(const sgs_gaussians* g, const sgs_camera* host_cams, const sgs_camera* dev_cams,
                   int32_t n_cams, const sgs_options* opts, void* workspace, size_t workspace_bytes,
                   int64_t pair_capacity, const sgs_outputs* outs, int32_t flags,
                   int64_t* pairs_needed, void* stream) {
    return forward_impl(g, host_cams, dev_cams, n_cams, opts, workspace, workspace_bytes,
                        pair_capacity, outs, flags, pairs_needed, stream, true);
}

int render_forward_noalloc(const sgs_gaussians* g, const sgs_camera* host_cams,
                           const sgs_camera* dev_cams, int32_t n_cams, const sgs_options* opts,
                           int64_t pair_capacity, const sgs_outputs* outs, int32_t flags,
                           int64_t* pairs_needed, void* stream) {
    int dev = -1;
    SGS_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(SGS_E_INVALID, "device index out of range");
    void* base = g_scratch[dev].load();
    if (!base) {
        // first call on this device (current): its copy of the array
        SGS_HIP(hipGetSymbolAddress(&base, HIP_SYMBOL(scratch)));
        if (!base) return fail(SGS_E_HIP, "hipGetSymbolAddress returned no address");
        g_scratch[dev].store(base);
    }
    Plan pl;
    const int rc = plan(g, host_cams, n_cams, opts, pair_capacity, &pl);
    if (rc != SGS_OK) return rc;
    if (pl.lay.total_bytes > (size_t)SGS_NOALLOC_WORKSPACE_BYTES)
        return fail(SGS_E_INVALID, "the workspace needs " + std::to_string(pl.lay.total_bytes) +
                                       " bytes, more than the " +
                                       std::to_string((size_t)SGS_NOALLOC_WORKSPACE_BYTES) +
                                       " bytes of the no-allocation scratch");
    return forward_impl(g, host_cams, dev_cams, n_cams, opts, base, SGS_NOALLOC_WORKSPACE_BYTES,
                        pair_capacity, outs, flags, pairs_needed, stream, false);
}

int render_backward(const sgs_gaussians* g, const sgs_camera* host_cams, const sgs_camera* dev_cams,
                    int32_t n_cams, const sgs_options* opts, void* workspace, size_t workspace_bytes,
                    int64_t pair_capacity, const sgs_outputs* fwd, const float* grad_image,
                    const float* grad_depth, const float* grad_alpha, const sgs_grads* grads,
                    void* stream) {
    Plan pl;
    int rc = plan(g, host_cams, n_cams, opts, pair_capacity, &pl);
    if (rc != SGS_OK) return rc;
    if ((rc = check_params(g)) != SGS_OK) return rc;
    if (!dev_cams || !workspace || !fwd || !fwd->final_T || !fwd->n_contrib || !grad_image || !grads)
        return fail(SGS_E_INVALID, "a required backward argument is NULL");
    if (workspace_bytes < pl.lay.total_bytes) return fail(SGS_E_INVALID, "workspace too small");
    if (g->n > 0 && (!grads->means || !grads->log_scales || !grads->quats ||
                     !grads->opacity_logits || !grads->sh))
        return fail(SGS_E_INVALID, "a gradient output array is NULL");
    if (g->n > 0 && g->n_lobes > 0 && (!grads->sg_log_sharpness || !grads->sg_amplitudes))
        return fail(SGS_E_INVALID, "an SG gradient output array is NULL");
    if (g->n > 0 && axis_rows(g) > 0 && !grads->sg_axes)
        return fail(SGS_E_INVALID, "the sg_axes gradient output is NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const sgs::Workspace ws = bind(pl, workspace);
    const sgs::Params p = params_of(g);
    (void)hipGetLastError();
    if (pl.n == 0) return SGS_OK;
    Marker mk{timing_slot(g_timing.bwd, g_timing.bwd_used), s};
    const bool dg = grad_depth || grad_alpha;
    mk.mark(0);
    // the 64-byte gradient records of the visible items (whole lines); no
    // kernel writes or reads another item's record
    sgs::launch_clear_grad2d(ws, s);
    if (pl.queue) sgs::launch_fill_u32(ws.header + sgs::kHdrQueueBwd, 0u, 1, s);
    mk.mark(1);
    sgs::launch_blend_bwd(ws, dev_cams, n_cams, pl.o, *fwd, grad_image, grad_depth, grad_alpha,
                          pl.queue, s);
    SGS_LAUNCHED();
    mk.mark(2);
    sgs::launch_preprocess_bwd(p, dev_cams, n_cams, pl.o, ws, *grads, dg, s);
    SGS_LAUNCHED();
    mk.mark(3);
    return SGS_OK;
}

int render_l1(const sgs_camera* host_cams, int32_t n_cams, const void* workspace, const float* image,
              const float* target, float* grad_image, double* loss, void* stream) {
    if (!host_cams || n_cams < 1 || n_cams > SGS_MAX_CAMERAS)
        return fail(SGS_E_INVALID, "cameras");
    if (!workspace || !image || !target || !grad_image || !loss)
        return fail(SGS_E_INVALID, "a required L1 argument is NULL");
    sgs_gaussians g0;
    memset(&g0, 0, sizeof(g0));
    Plan pl;
    // only the camera table and the loss partials are used; their offsets do
    // not depend on n, the options or the capacity
    int rc = plan(&g0, host_cams, n_cams, nullptr, 0, &pl);
    if (rc != SGS_OK) return rc;
    sgs::Workspace ws = bind(pl, const_cast<void*>(workspace));
    (void)hipGetLastError();
    sgs::launch_l1(ws, n_cams, image, target, grad_image, loss, static_cast<hipStream_t>(stream));
    SGS_LAUNCHED();
    return SGS_OK;
}

int render_status(const void* workspace, uint32_t* status_bits, int64_t* pairs, void* stream) {
    if (!workspace) return fail(SGS_E_INVALID, "workspace is NULL");
    uint32_t h[2];
    hipStream_t s = static_cast<hipStream_t>(stream);
    SGS_HIP(hipStreamSynchronize(s));
    SGS_HIP(hipMemcpy(h, workspace, 8, hipMemcpyDeviceToHost));
    if (status_bits) *status_bits = h[0];
    if (pairs) *pairs = h[1];
    return SGS_OK;
}

int render_read_keys(const void* workspace, const sgs_layout* layout, int64_t count,
                     uint64_t* keys_out, void* stream) {
    if (!workspace || !layout || !keys_out) return fail(SGS_E_INVALID, "NULL argument");
    if (count < 0 || count > layout->pair_capacity) return fail(SGS_E_INVALID, "count");
    const char* b = static_cast<const char*>(workspace);
    sgs::Workspace ws;
    memset(&ws, 0, sizeof(ws));
    ws.pair_values = reinterpret_cast<uint32_t*>(const_cast<char*>(b) + layout->pair_values);
    ws.ranges = reinterpret_cast<uint32_t*>(const_cast<char*>(b) + layout->ranges);
    ws.depth_keys = reinterpret_cast<uint32_t*>(const_cast<char*>(b) + layout->depth_keys);
    ws.n_items = layout->n_items;
    ws.n_tiles = layout->n_tiles;
    (void)hipGetLastError();
    sgs::launch_read_keys(ws, count, keys_out, static_cast<hipStream_t>(stream));
    SGS_LAUNCHED();
    return SGS_OK;
}

int render_set_timing(int32_t enable) {
    g_timing.on = enable != 0;
    return SGS_OK;
}

int render_stage_times(float* ms_out, int32_t n_out, int32_t* n_calls, int32_t* n_bwd_calls) {
    if (!ms_out || n_out < SGS_N_STAGES) return fail(SGS_E_INVALID, "ms_out needs SGS_N_STAGES entries");
    for (int i = 0; i < SGS_N_STAGES; ++i) ms_out[i] = 0.0f;
    for (size_t c = 0; c < g_timing.fwd_used; ++c) {
        auto& ev = g_timing.fwd[c];
        SGS_HIP(hipEventSynchronize(ev[kFwdEvents - 1]));
        for (int i = 0; i + 1 < kFwdEvents; ++i) {
            float ms = 0.0f;
            SGS_HIP(hipEventElapsedTime(&ms, ev[i], ev[i + 1]));
            ms_out[i] += ms;
        }
    }
    for (size_t c = 0; c < g_timing.bwd_used; ++c) {
        auto& ev = g_timing.bwd[c];
        SGS_HIP(hipEventSynchronize(ev[kBwdEvents - 1]));
        for (int i = 0; i + 1 < kBwdEvents; ++i) {
            float ms = 0.0f;
            SGS_HIP(hipEventElapsedTime(&ms, ev[i], ev[i + 1]));
            ms_out[kFwdEvents - 1 + i] += ms;
        }
    }
    if (n_calls) *n_calls = (int32_t)g_timing.fwd_used;
    if (n_bwd_calls) *n_bwd_calls = (int32_t)g_timing.bwd_used;
    g_timing.fwd_used = g_timing.bwd_used = 0;
    return SGS_OK;
}

const char* render_stage_name(int32_t stage) {
    return (stage >= 0 && stage < SGS_N_STAGES) ? kStageNames[stage] : "";
}

int render_blend_work(const sgs_gaussians* g, const sgs_camera* host_cams, const sgs_camera* dev_cams,
                      int32_t n_cams, const sgs_options* opts, const void* workspace,
                      size_t workspace_bytes, int64_t pair_capacity, uint64_t* counts,
                      void* stream) {
    Plan pl;
    int rc = plan(g, host_cams, n_cams, opts, pair_capacity, &pl);
    if (rc != SGS_OK) return rc;
    if (!dev_cams || !workspace || !counts) return fail(SGS_E_INVALID, "NULL argument");
    if (workspace_bytes < pl.lay.total_bytes) return fail(SGS_E_INVALID, "workspace too small");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const sgs::Workspace ws = bind(pl, const_cast<void*>(workspace));
    (void)hipGetLastError();
    sgs::launch_fill_u32(reinterpret_cast<uint32_t*>(counts), 0u, 6, s);
    sgs::launch_blend_count(ws, dev_cams, n_cams, pl.o, counts, s);
    SGS_LAUNCHED();
    return SGS_OK;
}

int render_blend_bwd_work(const sgs_gaussians* g, const sgs_camera* host_cams,
                          const sgs_camera* dev_cams, int32_t n_cams, const sgs_options* opts,
                          const void* workspace, size_t workspace_bytes, int64_t pair_capacity,
                          const sgs_outputs* fwd, uint64_t* counts, void* stream) {
    Plan pl;
    int rc = plan(g, host_cams, n_cams, opts, pair_capacity, &pl);
    if (rc != SGS_OK) return rc;
    if (!dev_cams || !workspace || !counts || !fwd || !fwd->final_T || !fwd->n_contrib)
        return fail(SGS_E_INVALID, "NULL argument");
    if (workspace_bytes < pl.lay.total_bytes) return fail(SGS_E_INVALID, "workspace too small");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const sgs::Workspace ws = bind(pl, const_cast<void*>(workspace));
    (void)hipGetLastError();
    sgs::launch_fill_u32(reinterpret_cast<uint32_t*>(counts), 0u, 8, s);
    sgs::launch_blend_bwd_count(ws, dev_cams, n_cams, pl.o, *fwd, counts, s);
    SGS_LAUNCHED();
    return SGS_OK;
}

int render_adam_step(const sgs_gaussians* g, const sgs_adam* cfg, const sgs_grads* grads,
                     const sgs_grads* exp_avg, const sgs_grads* exp_avg_sq, void* stream) {
    if (!g || !cfg || !grads || !exp_avg || !exp_avg_sq)
        return fail(SGS_E_INVALID, "a required Adam argument is NULL");
    if (g->n < 0 || g->sh_degree < 0 || g->sh_degree > SGS_MAX_SH_DEGREE || g->n_lobes < 0 ||
        g->n_lobes > SGS_MAX_LOBES)
        return fail(SGS_E_INVALID, "invalid Gaussian form");
    if (g->lobe_axes != SGS_LOBES_FREE && g->lobe_axes != SGS_LOBES_WORLD &&
        g->lobe_axes != SGS_LOBES_FRAME)
        return fail(SGS_E_INVALID, "lobe_axes must be SGS_LOBES_FREE, _WORLD or _FRAME");
    if (cfg->step < 1) return fail(SGS_E_INVALID, "step must be >= 1");
    if (g->colour_dtype != SGS_COLOUR_F32)
        return fail(SGS_E_INVALID, "the Adam step updates float32 parameters only");
    int rc = check_params(g);
    if (rc != SGS_OK) return rc;
    const int64_t n = g->n;
    const int64_t nc3 = 3 * (int64_t)(g->sh_degree + 1) * (g->sh_degree + 1), K = g->n_lobes;
    const int64_t width[sgs::kAdamArrays] = {3 * n, 3 * n, 4 * n, n, nc3, 3 * (int64_t)axis_rows(g), K, 3 * K};
    const bool colour[sgs::kAdamArrays] = {false, false, false, false, true, true, true, true};
    const bool lobe[sgs::kAdamArrays] = {false, false, false, false, false, true, true, true};
    const float* params[sgs::kAdamArrays] = {g->means, g->log_scales, g->quats, g->opacity_logits,
                                             g->sh, g->sg_axes, g->sg_log_sharpness, g->sg_amplitudes};
    auto arrays = [](const sgs_grads* x, float* out[sgs::kAdamArrays]) {
        float* const f[sgs::kAdamArrays] = {x->means, x->log_scales, x->quats, x->opacity_logits,
                                            x->sh, x->sg_axes, x->sg_log_sharpness, x->sg_amplitudes};
        for (int k = 0; k < sgs::kAdamArrays; ++k) out[k] = f[k];
    };
    float *gr[sgs::kAdamArrays], *m[sgs::kAdamArrays], *v[sgs::kAdamArrays];
    arrays(grads, gr);
    arrays(exp_avg, m);
    arrays(exp_avg_sq, v);
    sgs::AdamArrays a;
    memset(&a, 0, sizeof(a));
    const double b1 = cfg->beta1 != 0.0 ? cfg->beta1 : 0.9;
    const double b2 = cfg->beta2 != 0.0 ? cfg->beta2 : 0.999;
    if (!(b1 > 0.0 && b1 < 1.0 && b2 > 0.0 && b2 < 1.0))
        return fail(SGS_E_INVALID, "beta1 and beta2 must be in (0, 1)");
    a.b1 = (float)b1;
    a.b2 = (float)b2;
    a.ob1 = (float)(1.0 - b1);
    a.ob2 = (float)(1.0 - b2);
    a.eps = (float)(cfg->eps != 0.0 ? cfg->eps : 1e-15);
    const int sg0 = cfg->sg_start > 1 ? cfg->sg_start : 1;
    for (int k = 0; k < sgs::kAdamArrays; ++k) {
        if (!(cfg->lr[k] >= 0.0f)) return fail(SGS_E_INVALID, "learning rates must be >= 0");
        const int64_t count = colour[k] ? n * width[k] : width[k];
        const int t = lobe[k] ? cfg->step - sg0 + 1 : cfg->step;
        a.on[k] = count > 0 && cfg->lr[k] > 0.0f && t >= 1;
        if (!a.on[k]) continue;
        if (!params[k] || !gr[k] || !m[k] || !v[k])
            return fail(SGS_E_INVALID, "a parameter, gradient or moment array is NULL");
        a.p[k] = const_cast<float*>(params[k]);
        a.g[k] = gr[k];
        a.m[k] = m[k];
        a.v[k] = v[k];
        a.count[k] = count;
        // geometry rows and packed colour arrays are flat runs
        const int64_t cs = g->colour_stride;
        a.width[k] = colour[k] ? width[k] : count;
        a.pstride[k] = colour[k] && cs > 0 ? cs : a.width[k];
        a.lr[k] = cfg->lr[k];
        a.c1[k] = (float)(1.0 / (1.0 - std::pow(b1, (double)t)));
        a.c2[k] = (float)(1.0 / (1.0 - std::pow(b2, (double)t)));
    }
    (void)hipGetLastError();
    sgs::launch_adam(a, static_cast<hipStream_t>(stream));
    SGS_LAUNCHED();
    return SGS_OK;
}

const char* render_last_error(void) { return g_err.c_str(); }

}  // extern "C"
