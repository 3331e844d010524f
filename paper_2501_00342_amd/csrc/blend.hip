// Tile compositing, forward and backward, and the L1 loss.
//
// One workgroup per tile (TW x TH pixels, PPT pixels per thread, stacked in
// one column so that the column test and the x-terms of the power are
// shared; a wave owns a compact block of rows).  The tile's sorted
// Gaussians are streamed through LDS in batches: each thread gathers 64-byte
// records, turns them into tile-relative entries and all pixels of the tile
// read them back.  Forward
// (the compositing of the Preliminaries section, front to back in depth):
//   alpha = min(alpha_max, opacity * exp(-d^T Q d / 2)),  skip alpha < alpha_min,
//   stop before T (1 - alpha) < T_min,  C += alpha T rgb,  T *= 1 - alpha.
// exp(-d^T Q d / 2) is evaluated as exp2(-q), q = (w1.d)^2 + (w2.d)^2 with
// whitening rows from the preprocess (one v_exp_f32, no conic cancellation).
// Early exit: a wave skips the LDS loop once its 64 pixels are done and
// the workgroup leaves when all pixels are done (__syncthreads_count).
// Tile order, two schedules:
//   grid   one workgroup per tile; consecutive workgroup ids go to different
//          XCDs, so block b is mapped to a contiguous run of tiles per XCD
//          to share L2 lines of records;
//   queue  a persistent grid (as many workgroups as fit on the chip at once)
//          pops tiles from an atomic counter over a heavy-first tile order
//          (tiles sorted by decreasing list length), so that the longest
//          tiles start first and the short ones fill the tail.
//
// Backward: the same tile walk back to front from the saved final T and
// n_contrib, recomputing alpha with the same instructions, T_j =
// T_{j+1} / (1 - alpha_j).  Per-Gaussian 2D gradients are summed over a
// thread's pixels, then across the wave (lane swaps and DPP), and added with
// one float atomic per value per wave.  Depth and accumulated alpha may
// carry upstream gradients too (then the splat depth z gets one).

#include "common.hpp"
#include "occupancy.hpp"

namespace sgs {

struct __align__(16) Entry {
    float4 a;   // ux, vy, w1x, w1y   (ux = (x0 - u_hi) - u_lo, tile-relative)
    float4 b;   // w2x, w2y, opacity, z
    float4 c;   // r, g, b, item (as bits)
    uint2 m;    // column mask, row mask of the pixel rectangle inside the tile
};

__device__ __forceinline__ uint32_t span_mask(int lo, int hi, int n) {
    if (hi < 0 || lo > n - 1) return 0u;
    lo = lo < 0 ? 0 : lo;
    hi = hi > n - 1 ? n - 1 : hi;
    return (2u << hi) - (1u << lo);
}

__device__ __forceinline__ Entry make_entry(const Rec* __restrict__ recs, uint32_t item, int x0,
                                            int y0, int TW, int TH) {
    const float4* src = reinterpret_cast<const float4*>(recs + item);
    const float4 r0 = src[0], r1 = src[1], r2 = src[2], r3 = src[3];
    Entry e;
    e.a.x = ((float)x0 - r0.x) - r0.z;
    e.a.y = ((float)y0 - r0.y) - r0.w;
    e.a.z = r1.x;
    e.a.w = r1.y;
    e.b.x = r1.z;
    e.b.y = r1.w;
    e.b.z = r2.x;
    e.b.w = r3.x;
    e.c.x = r2.y;
    e.c.y = r2.z;
    e.c.z = r2.w;
    e.c.w = __uint_as_float(item);
    const uint32_t rx = __float_as_uint(r3.y), ry = __float_as_uint(r3.z);
    e.m.x = span_mask((int)(rx & 0xFFFF) - x0, (int)(rx >> 16) - x0, TW);
    e.m.y = span_mask((int)(ry & 0xFFFF) - y0, (int)(ry >> 16) - y0, TH);
    return e;
}

// alpha of one splat at one pixel; identical instructions in both passes.
// The x-terms w1x*dx and w2x*dx are shared by the pixels of one column.
struct Eval {
    float y1, y2, E, alpha;
};

__device__ __forceinline__ Eval eval_splat(const Entry& e, float t1, float t2, float dy,
                                           float amax) {
    Eval v;
    v.y1 = fmaf(e.a.w, dy, t1);
    v.y2 = fmaf(e.b.y, dy, t2);
    const float q = fmaf(v.y2, v.y2, v.y1 * v.y1);
    v.E = __builtin_amdgcn_exp2f(-q);
    v.alpha = fminf(amax, e.b.z * v.E);
    return v;
}

// blockIdx -> tile: XCD x = b % 8 receives a contiguous run of tiles
__device__ __forceinline__ int64_t xcd_tile(int64_t b, int64_t n_tiles) {
    const int64_t q = n_tiles / 8, r = n_tiles % 8;
    const int64_t x = b % 8, k = b / 8;
    return x * q + (x < r ? x : r) + k;
}

__device__ __forceinline__ int find_camera(const CamTable* cams, int n_cams, int64_t tile) {
    int lo = 0, hi = n_cams - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (cams[mid].tile_base <= tile) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// entry for list position `pos`; an out-of-range item yields an empty mask
__device__ __forceinline__ Entry load_entry(const Workspace& ws, int64_t pos, int x0, int y0, int TW,
                                            int TH) {
    const uint32_t item = ws.pair_values[pos];
    if (item < (uint64_t)ws.n_items) return make_entry(ws.records, item, x0, y0, TW, TH);
    Entry e = {};
    e.c.w = __uint_as_float(0u);
    return e;
}

// Thread t of a TW x TH tile with PPT pixels per thread owns column t % TW
// and the PPT consecutive rows from (t / TW) * PPT, so that a wave covers a
// compact TW x (64 / TW) * PPT block and small splats touch few waves.
// SLICED: the workgroup is one wave and owns slice `slice` of the tile (the
// pixels wave `slice` of a whole-tile workgroup would own); it streams the
// tile's list on its own, so no wave waits on another's pixels.
template <int TW, int TH, int PPT, bool COUNT, bool SLICED>
__device__ __forceinline__ void fwd_tile(const Workspace& ws, const sgs_camera* __restrict__ cams,
                                         int n_cams, const Opts& o, const sgs_outputs& out,
                                         int batch, int64_t tile, int slice, Entry* s_e, int* s_cam,
                                         unsigned long long& visited,
                                         unsigned long long& evaluated,
                                         unsigned long long& blended) {
    constexpr int NT = SLICED ? 64 : TW * TH / PPT;   // threads of the workgroup
    const int tid = threadIdx.x;
    const int vtid = (SLICED ? slice * 64 : 0) + tid;  // thread of the whole-tile layout
    if (tid == 0) *s_cam = find_camera(ws.cams, n_cams, tile);
    __syncthreads();
    const int cam = *s_cam;
    const CamTable ct = ws.cams[cam];
    const int lt = (int)(tile - ct.tile_base);
    const int tx = lt % ct.GX, ty = lt / ct.GX;
    const int x0 = tx * TW, y0 = ty * TH;
    const int lx = vtid % TW, ry = (vtid / TW) * PPT;   // rows ry .. ry + PPT - 1
    const uint32_t start = ws.ranges[2 * tile];
    const uint32_t end = (int64_t)ws.ranges[2 * tile + 1] <= ws.capacity ? ws.ranges[2 * tile + 1] : start;
    const uint32_t colbit = 1u << lx;
    const float lxf = (float)lx;
    const float amin = o.alpha_min, amax = o.alpha_max, tmin = o.t_min;

    float T[PPT], C0[PPT], C1[PPT], C2[PPT], D[PPT];
    int n[PPT];
    uint32_t live = 0;   // bit k: pixel k still blending
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        T[k] = 1.0f;
        C0[k] = C1[k] = C2[k] = D[k] = 0.0f;
        n[k] = 0;
        if (x0 + lx < ct.W && y0 + ry + k < ct.H) live |= 1u << k;
    }
    for (uint32_t bs = start; bs < end; bs += batch) {
        if (__syncthreads_count(live != 0) == 0) break;
        const int cnt = (int)((end - bs) < (uint32_t)batch ? (end - bs) : (uint32_t)batch);
        for (int k = tid; k < cnt; k += NT)
            s_e[k] = load_entry(ws, (int64_t)bs + k, x0, y0, TW, TH);
        __syncthreads();
        // the loop exits are wave-uniform: a thread whose pixels are all done
        // stays in it with every pixel skipped by its live bit, instead of a
        // divergent exit whose bookkeeping costs VALU on every entry
        if (__any(live != 0u)) {
            for (int j = 0; j < cnt; ++j) {
                const Entry e = s_e[j];
                if (COUNT && live) ++visited;   // per thread: its pixels share the column work
                // nested tests rather than `continue`: no exit flag to track
                if (e.m.x & colbit) {
                    const float dx = lxf + e.a.x;
                    const float t1 = e.a.z * dx, t2 = e.b.x * dx;
                    // bit k: pixel k still blends and lies in the splat's rows
                    const uint32_t take = (e.m.y >> ry) & live;
#pragma unroll
                    for (int k = 0; k < PPT; ++k) {
                        if ((take >> k) & 1u) {
                            if (COUNT) ++evaluated;
                            const Eval v = eval_splat(e, t1, t2, (float)(ry + k) + e.a.y, amax);
                            if (!(v.alpha < amin)) {
                                const float Tn = T[k] * (1.0f - v.alpha);
                                if (Tn < tmin) {
                                    live &= ~(1u << k);
                                } else {
                                    const float w = v.alpha * T[k];
                                    C0[k] = fmaf(w, e.c.x, C0[k]);
                                    C1[k] = fmaf(w, e.c.y, C1[k]);
                                    C2[k] = fmaf(w, e.c.z, C2[k]);
                                    D[k] = fmaf(w, e.b.w, D[k]);
                                    T[k] = Tn;
                                    n[k] = (int)(bs - start) + j + 1;
                                    if (COUNT) ++blended;
                                }
                            }
                        }
                    }
                }
                if (!__any(live != 0u)) break;
            }
        }
    }
    if (COUNT) return;
    const int64_t W = ct.W, H = ct.H;
    const sgs_camera& c = cams[cam];
    float* img = out.image + 3 * ct.pix_base;
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const int px = x0 + lx, py = y0 + ry + k;
        if (px >= ct.W || py >= ct.H) continue;
        const int64_t pix = (int64_t)py * W + px;
        img[pix] = C0[k] + T[k] * c.bg[0];
        img[W * H + pix] = C1[k] + T[k] * c.bg[1];
        img[2 * W * H + pix] = C2[k] + T[k] * c.bg[2];
        if (out.depth) out.depth[ct.pix_base + pix] = D[k];
        if (out.alpha) out.alpha[ct.pix_base + pix] = 1.0f - T[k];
        out.final_T[ct.pix_base + pix] = T[k];
        out.n_contrib[ct.pix_base + pix] = n[k];
    }
}

// next tile of the queue schedule, or -1 once the queue is drained; every
// thread of the workgroup gets the same answer.  The leading barrier keeps
// the previous tile's LDS reads ahead of the next tile's writes.
// With S slices per tile the queue holds S items per tile, consecutive in
// the heavy-first order; *slice receives the item's slice.
template <int S>
__device__ __forceinline__ int64_t pop_tile(const Workspace& ws, uint32_t* counter,
                                            uint32_t* s_next, int* slice) {
    __syncthreads();
    if (threadIdx.x == 0) *s_next = atomicAdd(counter, 1u);
    __syncthreads();
    const uint32_t item = *s_next;
    if ((int64_t)item >= ws.n_tiles * S) return -1;
    *slice = (int)(item % S);
    const uint32_t t = ws.tile_order[item / S];
    return (int64_t)t < ws.n_tiles ? (int64_t)t : -1;
}

// schedule: SGS_SCHEDULE_GRID (one workgroup per tile), _QUEUE (persistent
// whole-tile workgroups) or _SLICES (persistent one-wave workgroups, one
// slice of a tile per item)
template <int TW, int TH, int PPT, bool COUNT, int SCHED>
__global__ void __launch_bounds__(SCHED == SGS_SCHEDULE_SLICES ? 64 : TW * TH / PPT)
k_blend_fwd(Workspace ws, const sgs_camera* __restrict__ cams, int n_cams, Opts o,
            sgs_outputs out, int batch, unsigned long long* counts) {
    extern __shared__ __align__(16) Entry s_e[];
    __shared__ int s_cam;
    __shared__ uint32_t s_next;
    if (ws.header[kHdrStatus] & SGS_STATUS_CAMERAS) return;
    constexpr bool SL = SCHED == SGS_SCHEDULE_SLICES;
    constexpr int S = SL ? TW * TH / PPT / 64 : 1;   // slices per tile
    unsigned long long visited = 0, evaluated = 0, blended = 0;
    if (SCHED != SGS_SCHEDULE_GRID) {
        for (;;) {
            int slice = 0;
            const int64_t tile = pop_tile<S>(ws, ws.header + kHdrQueueFwd, &s_next, &slice);
            if (tile < 0) break;
            fwd_tile<TW, TH, PPT, COUNT, SL>(ws, cams, n_cams, o, out, batch, tile, slice, s_e,
                                             &s_cam, visited, evaluated, blended);
        }
    } else {
        fwd_tile<TW, TH, PPT, COUNT, false>(ws, cams, n_cams, o, out, batch,
                                            xcd_tile(blockIdx.x, ws.n_tiles), 0, s_e, &s_cam,
                                            visited, evaluated, blended);
    }
    if (COUNT) {
        __shared__ unsigned long long s_cnt[3];
        __syncthreads();
        if (threadIdx.x == 0) s_cnt[0] = s_cnt[1] = s_cnt[2] = 0ull;
        __syncthreads();
        atomicAdd(&s_cnt[0], visited);
        atomicAdd(&s_cnt[1], evaluated);
        atomicAdd(&s_cnt[2], blended);
        __syncthreads();
        if (threadIdx.x == 0) {
            atomicAdd(&counts[0], s_cnt[0]);
            atomicAdd(&counts[1], s_cnt[1]);
            atomicAdd(&counts[2], s_cnt[2]);
        }
    }
}

// ---------------------------------------------------------------------------
// backward
// ---------------------------------------------------------------------------

template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_add(float v) {
    const int s = __builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, 0xF, false);
    return v + __int_as_float(s);
}

__device__ __forceinline__ float2 swap16(float a, float b) {
    // rows of 16 lanes: odd rows of a <-> even rows of b
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false,
                                                    false);
    return make_float2(__uint_as_float(r[0]), __uint_as_float(r[1]));
}

__device__ __forceinline__ float2 swap32(float a, float b) {
    // upper 32 lanes of a <-> lower 32 lanes of b
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false,
                                                    false);
    return make_float2(__uint_as_float(r[0]), __uint_as_float(r[1]));
}

// Sums of NV (9 or 10) per-lane values over the wave, scattered over the
// rows (a reduce-scatter: two halving steps with the gfx950 lane-swap
// instructions, then a row reduction of three values with DPP, 28 VALU
// instead of 54 for nine full reductions).  Afterwards every lane of row r
// (lanes 16 r .. 16 r + 15) holds in x[i] the total of value 4 i + 2 q + h,
// q = r & 1, h = r >> 1 (values NV .. 11 are zero).
template <int NV>
__device__ __forceinline__ void wave_sum(const float v[NV], float x[3]) {
    static_assert(NV >= 9 && NV <= 10, "two halving steps and three row sums cover 9-12 values");
    float w[5];
#pragma unroll
    for (int j = 0; j < 5; ++j) {
        const float2 t = swap32(v[2 * j], 2 * j + 1 < NV ? v[2 * j + 1] : 0.0f);
        w[j] = t.x + t.y;   // lanes 0-31: value 2j, lanes 32-63: value 2j + 1
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const float2 t = swap16(w[2 * i], 2 * i + 1 < 5 ? w[2 * i + 1] : 0.0f);
        x[i] = t.x + t.y;   // even rows: w[2i], odd rows: w[2i + 1]
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        float y = dpp_add<0xB1, 0xF>(x[i]);   // quad_perm [1,0,3,2]
        y = dpp_add<0x4E, 0xF>(y);            // quad_perm [2,3,0,1]
        y = dpp_add<0x124, 0xF>(y);           // row_ror:4
        x[i] = dpp_add<0x128, 0xF>(y);        // row_ror:8
    }
}

// Upstream gradients of the backward: the image, and (DG) the depth and the
// accumulated alpha (either may be NULL: zero).
struct Upstream {
    const float* image;
    const float* depth;
    const float* alpha;
};

// DG: the depth D = sum alpha T z and accumulated alpha A = 1 - T_final
// have upstream gradients too.  With gD, gA the pixel's gradients of D and
// A, the scalar carried back to front becomes gC.S + gD D_behind - gA T_f
// (dA/dalpha_j = T_f / (1 - alpha_j)), each splat's front term adds gD z,
// and dL/dz = gD alpha T is a tenth 2D gradient.
// Work events of one backward walk (COUNT): list entries visited per
// thread, (pixel, entry) pairs whose alpha is recomputed, pairs that carry
// a gradient (alpha >= alpha_min), and wave reductions (one per wave and
// entry that some lane's pixels touch: one reduce-scatter and one atomic
// instruction of 9 or 10 lanes).
struct BwdWork {
    unsigned long long visited, evaluated, blended, reductions;
};

// SLICED: as in the forward, a one-wave workgroup owns one slice of the
// tile and walks back from the slice's own largest n_contrib.
template <int TW, int TH, int PPT, bool DG, bool COUNT, bool SLICED>
__device__ __forceinline__ void bwd_tile(const Workspace& ws, const sgs_camera* __restrict__ cams,
                                         int n_cams, const Opts& o, const sgs_outputs& fwd,
                                         const Upstream& up, int batch,
                                         int64_t tile, int slice, Entry* s_e, int* s_cam,
                                         int* s_maxn, BwdWork& work) {
    constexpr int NT = SLICED ? 64 : TW * TH / PPT;   // threads of the workgroup
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int vtid = (SLICED ? slice * 64 : 0) + tid;  // thread of the whole-tile layout
    if (tid == 0) {
        *s_cam = find_camera(ws.cams, n_cams, tile);
        *s_maxn = 0;
    }
    __syncthreads();
    const int cam = *s_cam;
    const CamTable ct = ws.cams[cam];
    const int lt = (int)(tile - ct.tile_base);
    const int tx = lt % ct.GX, ty = lt / ct.GX;
    const int x0 = tx * TW, y0 = ty * TH;
    const int lx = vtid % TW, ry = (vtid / TW) * PPT;   // rows ry .. ry + PPT - 1
    const uint32_t start = ws.ranges[2 * tile];
    const int64_t len = (int64_t)ws.ranges[2 * tile + 1] <= ws.capacity
                            ? (int64_t)ws.ranges[2 * tile + 1] - start : 0;
    const uint32_t colbit = 1u << lx;
    const float lxf = (float)lx;
    const float amin = o.alpha_min, amax = o.alpha_max;
    const sgs_camera& c = cams[cam];
    const int64_t W = ct.W, H = ct.H;
    const float* gi = up.image + 3 * ct.pix_base;

    // SG: dL/dC . S, S = colour composited behind the current splat (only its
    // product with the pixel's upstream gradient is needed); with DG also
    // gD D_behind - gA T_f
    float T[PPT], g0[PPT], g1[PPT], g2[PPT], SG[PPT], gD[PPT];
    int nc[PPT];
    int my_max = 0;
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const int px = x0 + lx, py = y0 + ry + k;
        T[k] = 1.0f;
        g0[k] = g1[k] = g2[k] = gD[k] = 0.0f;
        float gA = 0.0f;
        nc[k] = 0;
        if (px < ct.W && py < ct.H) {
            const int64_t pix = (int64_t)py * W + px;
            T[k] = fwd.final_T[ct.pix_base + pix];
            nc[k] = fwd.n_contrib[ct.pix_base + pix];
            if (!COUNT) {
                g0[k] = gi[pix];
                g1[k] = gi[W * H + pix];
                g2[k] = gi[2 * W * H + pix];
            }
            if (DG) {
                if (up.depth) gD[k] = up.depth[ct.pix_base + pix];
                if (up.alpha) gA = up.alpha[ct.pix_base + pix];
            }
        }
        if (nc[k] > len) nc[k] = (int)len;
        SG[k] = T[k] * (c.bg[0] * g0[k] + c.bg[1] * g1[k] + c.bg[2] * g2[k]);
        if (DG) SG[k] -= gA * T[k];
        my_max = nc[k] > my_max ? nc[k] : my_max;
    }
    if (my_max > 0) atomicMax(s_maxn, my_max);
    __syncthreads();
    const int maxn = *s_maxn;
    const int64_t M = ws.n_items;
    float* G = ws.grad2d;
    const float inv_k = (float)(1.0 / kHalfLog2e);

    for (int be = maxn; be > 0; be -= batch) {
        const int bb = be - batch > 0 ? be - batch : 0;
        const int cnt = be - bb;
        __syncthreads();
        for (int k = tid; k < cnt; k += NT)
            s_e[k] = load_entry(ws, (int64_t)start + bb + k, x0, y0, TW, TH);
        __syncthreads();
        for (int j = cnt - 1; j >= 0; --j) {
            const Entry e = s_e[j];
            const int pos = bb + j;
            // per pixel only the moments of dL/dp over the splat's offsets
            // d = (dx, dy) are summed: m1 = sum dLdp dx, m2 = sum dLdp dy,
            // m3 = sum dLdp dx^2, m4 = sum dLdp dx dy, m5 = sum dLdp dy^2.
            // The mean and conic gradients are linear in them (dp/du =
            // (Q d)_x, dp/dQa = -dx^2 / 2, ...) and are formed once per wave
            // reduction.
            float m1 = 0.f, m2 = 0.f, m3 = 0.f, m4 = 0.f, m5 = 0.f, v_s = 0.f;
            float v_r = 0.f, v_g = 0.f, v_b = 0.f, v_z = 0.f;
            bool contrib = false;
            if (COUNT) ++work.visited;
            if (e.m.x & colbit) {
                const float dx = lxf + e.a.x;
                const float t1 = e.a.z * dx, t2 = e.b.x * dx;
#pragma unroll
                for (int k = 0; k < PPT; ++k) {
                    // nested tests rather than `continue`: no exit flag to track
                    if (pos < nc[k] && ((e.m.y >> (ry + k)) & 1u)) {
                        if (COUNT) ++work.evaluated;
                        const float dy = (float)(ry + k) + e.a.y;
                        const Eval v = eval_splat(e, t1, t2, dy, amax);
                        if (!(v.alpha < amin)) {
                            contrib = true;
                            if (COUNT) {
                                ++work.blended;
                            } else {
                                // 1 / (1 - alpha) with v_rcp_f32 (1 ulp; 1 - alpha >= 1 - alpha_max)
                                const float iom = __builtin_amdgcn_rcpf(1.0f - v.alpha);
                                T[k] = T[k] * iom;
                                const float w = v.alpha * T[k];
                                v_r = fmaf(w, g0[k], v_r);
                                v_g = fmaf(w, g1[k], v_g);
                                v_b = fmaf(w, g2[k], v_b);
                                float cg = e.c.x * g0[k] + e.c.y * g1[k] + e.c.z * g2[k];
                                if (DG) {
                                    cg = fmaf(e.b.w, gD[k], cg);   // + z gD
                                    v_z = fmaf(w, gD[k], v_z);      // dL/dz = alpha T gD
                                }
                                const float sg = SG[k];
                                const float dLda = T[k] * cg - sg * iom;
                                SG[k] = fmaf(w, cg, SG[k]);
                                if (e.b.z * v.E <= amax) {
                                    v_s = fmaf(dLda, v.E, v_s);
                                    const float dLdp = dLda * v.alpha;
                                    m1 = fmaf(dLdp, dx, m1);
                                    m2 = fmaf(dLdp, dy, m2);
                                    const float px_ = dLdp * dx;
                                    m3 = fmaf(px_, dx, m3);
                                    m4 = fmaf(px_, dy, m4);
                                    m5 = fmaf(dLdp * dy, dy, m5);
                                }
                            }
                        }
                    }
                }
            }
            if (COUNT) {
                if (__any(contrib) && lane == 0) ++work.reductions;
            } else if (__any(contrib)) {
                constexpr int NV = DG ? 10 : 9;
                const float vals[10] = {m1, m2, m3, m4, m5, v_s, v_r, v_g, v_b, v_z};
                float x[3];
                wave_sum<NV>(vals, x);
                // row r holds the totals of values ch, 4 + ch and 8 + ch,
                // ch = 2 (r & 1) + (r >> 1): the moments sit in rows 0-3 of
                // x[0] and row 0 of x[1]
                auto lane_f = [](float v, int l) {
                    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
                };
                const float s1 = lane_f(x[0], 0), s2 = lane_f(x[0], 32);
                const float s3 = lane_f(x[0], 16), s4 = lane_f(x[0], 48);
                const float s5 = lane_f(x[1], 0);
                // Q k = w1 w1^T + w2 w2^T (whitening rows), k = 1 / inv_k
                const float qa = fmaf(e.a.z, e.a.z, e.b.x * e.b.x);
                const float qb = fmaf(e.a.z, e.a.w, e.b.x * e.b.y);
                const float qc = fmaf(e.a.w, e.a.w, e.b.y * e.b.y);
                const float g_u = inv_k * fmaf(qa, s1, qb * s2);
                const float g_v = inv_k * fmaf(qb, s1, qc * s2);
                // the entry is the same in every lane: its address is scalar
                const int64_t item =
                    __builtin_amdgcn_readfirstlane(__float_as_uint(e.c.w));
                float* gi = G + item * kG2;
                // lane 15 of row r adds channel ch (u, Qa, v, Qb for rows
                // 0-3), lane 14 channel 4 + ch (Qc, r, sigma, g) and, in the
                // rows with ch < NV - 8, lane 13 channel 8 + ch (b, z) -- NV
                // lanes of one atomic instruction, all on the item's 64-byte
                // gradient record (channel order: u, v, Qa, Qb, Qc, sigma,
                // r, g, b, z)
                const int r = lane >> 4, sel = 15 - (lane & 15);
                const int ch = 2 * (r & 1) + (r >> 1);
                if (sel < 2 || (sel == 2 && ch < NV - 8)) {
                    const float c0 = r == 0 ? g_u : (r == 1 ? -0.5f * s3 : (r == 2 ? g_v : -s4));
                    const float c1 = r == 0 ? -0.5f * s5 : x[1];
                    const int chan = sel == 0 ? ch : (sel == 1 ? 4 + ch : 8 + ch);
                    unsafeAtomicAdd(gi + chan, sel == 0 ? c0 : (sel == 1 ? c1 : x[2]));
                }
            }
        }
    }
}

// waves per SIMD asked of the compiler for the backward: 7 without the
// depth/alpha terms (72 VGPRs, a few cold spills: 530 against 573 us on
// the 3M frame at the natural 74 VGPRs and 6 waves), 6 with them
template <bool DG>
struct BwdWaves {
    static constexpr int value = DG ? 6 : 7;
};

template <int TW, int TH, int PPT, int SCHED, bool DG, bool COUNT>
__global__ void __launch_bounds__(SCHED == SGS_SCHEDULE_SLICES ? 64 : TW * TH / PPT)
__attribute__((amdgpu_waves_per_eu(BwdWaves<DG>::value)))
k_blend_bwd(Workspace ws, const sgs_camera* __restrict__ cams, int n_cams, Opts o,
            sgs_outputs fwd, Upstream up, int batch, unsigned long long* counts) {
    extern __shared__ __align__(16) Entry s_e[];
    __shared__ int s_cam;
    __shared__ int s_maxn;
    __shared__ uint32_t s_next;
    if (ws.header[kHdrStatus] & SGS_STATUS_CAMERAS) return;
    constexpr bool SL = SCHED == SGS_SCHEDULE_SLICES;
    constexpr int S = SL ? TW * TH / PPT / 64 : 1;   // slices per tile
    BwdWork work = {0ull, 0ull, 0ull, 0ull};
    if (SCHED != SGS_SCHEDULE_GRID) {
        for (;;) {
            int slice = 0;
            const int64_t tile = pop_tile<S>(ws, ws.header + kHdrQueueBwd, &s_next, &slice);
            if (tile < 0) break;
            bwd_tile<TW, TH, PPT, DG, COUNT, SL>(ws, cams, n_cams, o, fwd, up, batch, tile, slice,
                                                 s_e, &s_cam, &s_maxn, work);
        }
    } else {
        bwd_tile<TW, TH, PPT, DG, COUNT, false>(ws, cams, n_cams, o, fwd, up, batch,
                                                xcd_tile(blockIdx.x, ws.n_tiles), 0, s_e, &s_cam,
                                                &s_maxn, work);
    }
    if (COUNT) {
        __shared__ unsigned long long s_cnt[4];
        __syncthreads();
        if (threadIdx.x < 4) s_cnt[threadIdx.x] = 0ull;
        __syncthreads();
        atomicAdd(&s_cnt[0], work.visited);
        atomicAdd(&s_cnt[1], work.evaluated);
        atomicAdd(&s_cnt[2], work.blended);
        atomicAdd(&s_cnt[3], work.reductions);
        __syncthreads();
        if (threadIdx.x < 4) atomicAdd(&counts[threadIdx.x], s_cnt[threadIdx.x]);
    }
}

// ---------------------------------------------------------------------------

static unsigned grid_of(int64_t resident, int64_t items) {
    const int64_t g = resident < 1 || resident > items ? items : resident;
    return (unsigned)g;
}

// sched: the schedule the plan resolved (SGS_SCHEDULE_GRID, _QUEUE or _SLICES)
template <int TW, int TH, int PPT>
static void launch_fwd_t(const Workspace& ws, const sgs_camera* cams, int n_cams, const Opts& o,
                         const sgs_outputs& out, int sched, hipStream_t s) {
    const size_t lds = (size_t)o.batch * sizeof(Entry);
    constexpr int NT = TW * TH / PPT;
    if (sched == SGS_SCHEDULE_SLICES) {
        auto k = k_blend_fwd<TW, TH, PPT, false, SGS_SCHEDULE_SLICES>;
        const int64_t items = ws.n_tiles * (NT / 64);
        hipLaunchKernelGGL(k, dim3(grid_of(resident_blocks(k, 64, lds), items)), dim3(64), lds, s,
                           ws, cams, n_cams, o, out, o.batch, nullptr);
    } else if (sched == SGS_SCHEDULE_QUEUE) {
        auto k = k_blend_fwd<TW, TH, PPT, false, SGS_SCHEDULE_QUEUE>;
        hipLaunchKernelGGL(k, dim3(grid_of(resident_blocks(k, NT, lds), ws.n_tiles)), dim3(NT), lds,
                           s, ws, cams, n_cams, o, out, o.batch, nullptr);
    } else {
        hipLaunchKernelGGL((k_blend_fwd<TW, TH, PPT, false, SGS_SCHEDULE_GRID>),
                           dim3((unsigned)ws.n_tiles), dim3(NT), lds, s, ws, cams, n_cams, o, out,
                           o.batch, nullptr);
    }
}

template <int TW, int TH, int PPT>
static void launch_count_t(const Workspace& ws, const sgs_camera* cams, int n_cams, const Opts& o,
                           uint64_t* counts, hipStream_t s) {
    const size_t lds = (size_t)o.batch * sizeof(Entry);
    sgs_outputs none = {};
    hipLaunchKernelGGL((k_blend_fwd<TW, TH, PPT, true, SGS_SCHEDULE_GRID>), dim3((unsigned)ws.n_tiles),
                       dim3(TW * TH / PPT), lds, s, ws, cams, n_cams, o, none, o.batch,
                       reinterpret_cast<unsigned long long*>(counts));
}

template <int TW, int TH, int PPT, bool DG>
static void launch_bwd_dg(const Workspace& ws, const sgs_camera* cams, int n_cams, const Opts& o,
                          const sgs_outputs& fwd, const Upstream& up, int sched, hipStream_t s) {
    const size_t lds = (size_t)o.batch * sizeof(Entry);
    constexpr int NT = TW * TH / PPT;
    if (sched == SGS_SCHEDULE_SLICES) {
        auto k = k_blend_bwd<TW, TH, PPT, SGS_SCHEDULE_SLICES, DG, false>;
        const int64_t items = ws.n_tiles * (NT / 64);
        hipLaunchKernelGGL(k, dim3(grid_of(resident_blocks(k, 64, lds), items)), dim3(64), lds, s,
                           ws, cams, n_cams, o, fwd, up, o.batch, nullptr);
    } else if (sched == SGS_SCHEDULE_QUEUE) {
        auto k = k_blend_bwd<TW, TH, PPT, SGS_SCHEDULE_QUEUE, DG, false>;
        hipLaunchKernelGGL(k, dim3(grid_of(resident_blocks(k, NT, lds), ws.n_tiles)), dim3(NT), lds,
                           s, ws, cams, n_cams, o, fwd, up, o.batch, nullptr);
    } else {
        hipLaunchKernelGGL((k_blend_bwd<TW, TH, PPT, SGS_SCHEDULE_GRID, DG, false>),
                           dim3((unsigned)ws.n_tiles), dim3(NT), lds, s, ws, cams, n_cams, o, fwd,
                           up, o.batch, nullptr);
    }
}

template <int TW, int TH, int PPT>
static void launch_bwd_count_t(const Workspace& ws, const sgs_camera* cams, int n_cams,
                               const Opts& o, const sgs_outputs& fwd, uint64_t* counts,
                               hipStream_t s) {
    const size_t lds = (size_t)o.batch * sizeof(Entry);
    const Upstream none = {nullptr, nullptr, nullptr};
    hipLaunchKernelGGL((k_blend_bwd<TW, TH, PPT, SGS_SCHEDULE_GRID, false, true>),
                       dim3((unsigned)ws.n_tiles), dim3(TW * TH / PPT), lds, s, ws, cams, n_cams, o,
                       fwd, none, o.batch, reinterpret_cast<unsigned long long*>(counts));
}

template <int TW, int TH, int PPT>
static void launch_bwd_t(const Workspace& ws, const sgs_camera* cams, int n_cams, const Opts& o,
                         const sgs_outputs& fwd, const Upstream& up, int sched, hipStream_t s) {
    if (up.depth || up.alpha)
        launch_bwd_dg<TW, TH, PPT, true>(ws, cams, n_cams, o, fwd, up, sched, s);
    else
        launch_bwd_dg<TW, TH, PPT, false>(ws, cams, n_cams, o, fwd, up, sched, s);
}

// supported (tile, pixels per thread): the block is a whole number of waves
#define SGS_TILE_SWITCH(F, PPT_FWD, ...)                                             \
    if (o.tile_w == 16 && o.tile_h == 16 && PPT_FWD == 1) F<16, 16, 1>(__VA_ARGS__);   \
    else if (o.tile_w == 16 && o.tile_h == 16 && PPT_FWD == 2) F<16, 16, 2>(__VA_ARGS__); \
    else if (o.tile_w == 16 && o.tile_h == 16 && PPT_FWD == 4) F<16, 16, 4>(__VA_ARGS__); \
    else if (o.tile_w == 8 && o.tile_h == 8) F<8, 8, 1>(__VA_ARGS__);                 \
    else if (o.tile_w == 16 && o.tile_h == 8 && PPT_FWD == 2) F<16, 8, 2>(__VA_ARGS__);   \
    else if (o.tile_w == 16 && o.tile_h == 8) F<16, 8, 1>(__VA_ARGS__);               \
    else if (o.tile_w == 8 && o.tile_h == 16 && PPT_FWD == 2) F<8, 16, 2>(__VA_ARGS__);   \
    else if (o.tile_w == 8 && o.tile_h == 16) F<8, 16, 1>(__VA_ARGS__);               \
    else if (o.tile_w == 32 && o.tile_h == 8 && PPT_FWD == 2) F<32, 8, 2>(__VA_ARGS__);   \
    else if (o.tile_w == 32 && o.tile_h == 8 && PPT_FWD == 4) F<32, 8, 4>(__VA_ARGS__);   \
    else if (o.tile_w == 32 && o.tile_h == 8) F<32, 8, 1>(__VA_ARGS__);

void launch_blend_fwd(const Workspace& ws, const sgs_camera* dev_cams, int n_cams, const Opts& o,
                      const sgs_outputs& out, bool queue, hipStream_t s) {
    if (ws.n_tiles <= 0) return;
    const int sched = queue ? o.schedule : SGS_SCHEDULE_GRID;
    SGS_TILE_SWITCH(launch_fwd_t, o.ppt, ws, dev_cams, n_cams, o, out, sched, s)
}

void launch_blend_count(const Workspace& ws, const sgs_camera* dev_cams, int n_cams, const Opts& o,
                        uint64_t* counts, hipStream_t s) {
    if (ws.n_tiles <= 0) return;
    SGS_TILE_SWITCH(launch_count_t, o.ppt, ws, dev_cams, n_cams, o, counts, s)
}

void launch_blend_bwd_count(const Workspace& ws, const sgs_camera* dev_cams, int n_cams,
                            const Opts& o, const sgs_outputs& fwd, uint64_t* counts,
                            hipStream_t s) {
    if (ws.n_tiles <= 0) return;
    SGS_TILE_SWITCH(launch_bwd_count_t, o.ppt_bwd, ws, dev_cams, n_cams, o, fwd, counts, s)
}

void launch_blend_bwd(const Workspace& ws, const sgs_camera* dev_cams, int n_cams, const Opts& o,
                      const sgs_outputs& fwd, const float* grad_image, const float* grad_depth,
                      const float* grad_alpha, bool queue, hipStream_t s) {
    if (ws.n_tiles <= 0) return;
    const Upstream up = {grad_image, grad_depth, grad_alpha};
    const int sched = queue ? o.schedule : SGS_SCHEDULE_GRID;
    SGS_TILE_SWITCH(launch_bwd_t, o.ppt_bwd, ws, dev_cams, n_cams, o, fwd, up, sched, s)
}

// ---------------------------------------------------------------------------
// L1 loss: L = sum_k mean_{3 H_k W_k} |img - tgt|, grad = sign / (3 H_k W_k)
// ---------------------------------------------------------------------------

constexpr int kL1Blocks = 1024;

__global__ void __launch_bounds__(256)
k_l1(Workspace ws, int n_cams, const float* __restrict__ img, const float* __restrict__ tgt,
     float* __restrict__ grad, double* partial) {
    __shared__ double s_sum[256];
    double acc = 0.0;
    const int64_t total = ws.n_pixels;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < total;
         p += (int64_t)gridDim.x * blockDim.x) {
        int lo = 0, hi = n_cams - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (ws.cams[mid].pix_base <= p) lo = mid; else hi = mid - 1;
        }
        const CamTable ct = ws.cams[lo];
        const int64_t wh = (int64_t)ct.W * ct.H;
        const int64_t local = p - ct.pix_base;
        const float inv = (float)(1.0 / (3.0 * (double)wh));
        double part = 0.0;
        for (int ch = 0; ch < 3; ++ch) {
            const int64_t idx = 3 * ct.pix_base + ch * wh + local;
            const float d = img[idx] - tgt[idx];
            grad[idx] = d > 0.0f ? inv : (d < 0.0f ? -inv : 0.0f);
            part += fabs((double)d);
        }
        acc += part / (3.0 * (double)wh);
    }
    s_sum[threadIdx.x] = acc;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) s_sum[threadIdx.x] += s_sum[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = s_sum[0];
}

__global__ void __launch_bounds__(256) k_l1_final(const double* partial, int n, double* loss) {
    __shared__ double s_sum[256];
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) acc += partial[i];
    s_sum[threadIdx.x] = acc;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) s_sum[threadIdx.x] += s_sum[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = s_sum[0];
}

void launch_l1(const Workspace& ws, int n_cams, const float* image, const float* target,
               float* grad, double* loss, hipStream_t s) {
    hipLaunchKernelGGL(k_l1, dim3(kL1Blocks), dim3(256), 0, s, ws, n_cams, image, target, grad,
                       ws.loss_partial);
    hipLaunchKernelGGL(k_l1_final, dim3(1), dim3(256), 0, s, ws.loss_partial, kL1Blocks, loss);
}

}  // namespace sgs
