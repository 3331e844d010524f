/*
 * sgsplat.h — C ABI of the MI355X SG-Splatting rasteriser (libsgsplat.so).
 *
 * The library renders 3D Gaussians whose view-dependent colour is low-degree
 * spherical harmonics plus K spherical-Gaussian lobes (SG-Splatting, arXiv
 * 2501.00342: Methods, eqs. 4-9) with the tile-based Gaussian-splatting
 * rasteriser the method builds on (Preliminaries: EWA projection, then
 * alpha blending of the depth-sorted splats), forward and backward, on one
 * AMD gfx950 GPU.
 *
 * Conventions shared by every entry point
 *   - All array pointers marked "device" are HIP device pointers owned by the
 *     caller.  The library allocates no device memory: every buffer it needs
 *     lives in a caller-provided workspace sized by render_workspace_bytes().
 *   - Geometry arrays (means, log_scales, quats, opacity_logits) are
 *     component-major (SoA): component c of Gaussian g is at [c * n + g].
 *     Colour arrays are Gaussian-major: Gaussian g's block starts at
 *     g * colour_stride floats (colour_stride 0 = packed), and inside it SH
 *     coefficients are [(deg+1)^2][3] (l-major, then m = -l..l, then the
 *     channel r, g, b), lobe axes and amplitudes [K][3], log-sharpness [K].
 *     See struct sgs_gaussians.
 *   - Quaternions are (w, x, y, z).  Raw parameters cross the ABI; the
 *     library applies scale = exp(log_scale), opacity = sigmoid(logit),
 *     sharpness = exp(log_sharpness) and normalises q and each lobe axis.
 *   - Colour of a Gaussian seen along the unit direction d from the camera
 *     centre to its mean: rgb = max(0, 0.5 + sum_lm sh_lm Y_lm(d)
 *     + sum_k a_k exp(lambda_k (d . mu_k - 1)))   (eq. 5 per lobe, eq. 9).
 *     Real SH with the Condon-Shortley phase.  K = 0 with degree 3 is the
 *     plain degree-3 SH form (eq. 4).
 *   - Cameras: pinhole, OpenCV axes, x_cam = R x_world + t, pixel (i, j)
 *     sampled at integer coordinates (i, j).  znear, fx and fy must be
 *     finite and > 0 (host cameras: SGS_E_INVALID; device cameras: status
 *     bit SGS_STATUS_CAMERAS, and no image is written).
 *   - Several cameras render in one call ("batched views"): their pixels are
 *     packed camera after camera.  Camera k's image is the (3, H_k, W_k)
 *     block starting at float offset 3 * pix_base_k of `image`, and its
 *     depth / final_T / n_contrib are the (H_k, W_k) blocks starting at
 *     pix_base_k, with pix_base_k = sum_{j<k} W_j H_j.
 *   - Every entry point returns an sgs_status; on a non-zero return
 *     render_last_error() gives a message (thread-local).  No exception
 *     crosses the ABI.  Work is enqueued on `stream` (a hipStream_t); the
 *     calls do not synchronise unless stated.
 */
#ifndef SGSPLAT_H
#define SGSPLAT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum sgs_status {
    SGS_OK = 0,
    SGS_E_INVALID = 1,   /* bad argument: NULL pointer, size, degree, tile shape, workspace */
    SGS_E_CAPACITY = 2,  /* more (tile, Gaussian) pairs than the workspace holds */
    SGS_E_HIP = 3        /* a HIP runtime call failed */
} sgs_status;

#define SGS_MAX_SH_DEGREE 3
#define SGS_MAX_LOBES 8
#define SGS_MAX_CAMERAS 1024
#define SGS_MAX_IMAGE_SIDE 32767

/* Gaussian parameters (device, float32).  n may be 0.
 * The geometry, which every Gaussian needs for culling, is component-major
 * (one contiguous row per component: coalesced over all n).  The colour,
 * which only Gaussians that survive culling need, is Gaussian-major: each
 * colour array holds one block per Gaussian, so a culled Gaussian's colour
 * is never read.  Block g of an array starts at g * colour_stride floats
 * (colour_stride 0: the array's own block size, i.e. packed).  With
 * colour_stride = 3 (deg+1)^2 + 7 K and the four arrays at offsets 0,
 * 3 (deg+1)^2, 3 (deg+1)^2 + 3 K and 3 (deg+1)^2 + 4 K of one buffer, a
 * Gaussian's whole colour is one contiguous record, which the rasteriser
 * fetches with the fewest cache lines (there, with colour_stride a multiple
 * of 4, the record may be read rounded up to whole 16-byte pieces: the
 * buffer must then span n * colour_stride floats from `sh`).  The axis
 * block holds A 3-vectors: A = K (free lobes), 1 (frame) or 0 (world);
 * record offsets then read 3 (deg+1)^2 + 3 A etc. in place of 3 K. */
typedef struct sgs_gaussians {
    int64_t n;
    int32_t sh_degree;               /* 0..3 */
    int32_t n_lobes;                 /* K, 0..SGS_MAX_LOBES */
    const float* means;              /* [3][n]   world position X (eq. 2)        */
    const float* log_scales;         /* [3][n]   log of the scale vector s (eq. 3) */
    const float* quats;              /* [4][n]   rotation q, (w,x,y,z) (eq. 3)     */
    const float* opacity_logits;     /* [n]      logit of opacity sigma            */
    const float* sh;                 /* [n][(deg+1)^2][3] SH coefficients (eq. 4)  */
    const float* sg_axes;            /* [n][A][3] lobe axis mu, any length (eq. 5), or the
                                        frame parameters (lobe_axes below) */
    const float* sg_log_sharpness;   /* [n][K]   log of lobe sharpness lambda      */
    const float* sg_amplitudes;      /* [n][K][3] lobe RGB amplitude alpha          */
    int64_t colour_stride;           /* floats between consecutive blocks of each colour
                                        array; 0 = packed; else >= every block size and a
                                        multiple of 4 gives 16-byte fetches */
    int32_t lobe_axes;               /* how the lobe axes are given (SGS_LOBES_*):
                                        FREE  sg_axes [n][K][3], one axis per lobe (eq. 5);
                                        WORLD K = 3 lobes on the fixed world axes (1,0,0),
                                              (0,1,0), (0,0,1); sg_axes unused, may be NULL
                                              (eqs. 7-8; Experiments, Implementation);
                                        FRAME K = 3 mutually orthogonal lobes on the columns
                                              of the rotation of the unit quaternion
                                              (1, w)/|(1, w)|, sg_axes [n][1][3] holding w
                                              (eq. 8; Methods, Multi-Axis Orthogonal
                                              Gaussians: 3 parameters for the frame) */
    int32_t sh_adaptive[2];          /* adaptive SH degree by projected radius r (pixels,
                                        the 3-sigma radius): degree 0 where r <= [0], at
                                        most 1 where r <= [1], else sh_degree (Methods,
                                        Mixing Spherical Harmonics and Spherical
                                        Gaussians).  {0, 0} = every Gaussian uses
                                        sh_degree; else 0 <= [0] <= [1]. */
    int32_t colour_dtype;            /* element type of the four colour arrays (sh, sg_axes,
                                        sg_log_sharpness, sg_amplitudes): SGS_COLOUR_F32, or
                                        SGS_COLOUR_BF16 / SGS_COLOUR_F16 storage (their
                                        pointers then address 2-byte elements and
                                        colour_stride counts elements; the arithmetic stays
                                        float32, and those types need sh_adaptive {0, 0}).
                                        The storage side of the compact model (Experiments,
                                        Table 3). */
} sgs_gaussians;

#define SGS_COLOUR_F32 0
#define SGS_COLOUR_BF16 1
#define SGS_COLOUR_F16 2

#define SGS_LOBES_FREE 0
#define SGS_LOBES_WORLD 1
#define SGS_LOBES_FRAME 2

/* Gradient outputs, same shapes as sgs_gaussians (device, float32), every
 * array packed (the colour arrays Gaussian-major with colour_stride 0).
 * Every array is overwritten (not accumulated).  Arrays of zero size may be
 * NULL. */
typedef struct sgs_grads {
    float* means;
    float* log_scales;
    float* quats;
    float* opacity_logits;
    float* sh;
    float* sg_axes;
    float* sg_log_sharpness;
    float* sg_amplitudes;
} sgs_grads;

/* One pinhole camera (host and device copies share this layout). */
typedef struct sgs_camera {
    int32_t width, height;           /* 1..SGS_MAX_IMAGE_SIDE */
    float R[9];                      /* world -> camera rotation, row-major */
    float t[3];                      /* world -> camera translation */
    float fx, fy, cx, cy;            /* focal lengths and principal point, pixels */
    float znear;                     /* Gaussians with camera depth <= znear are culled */
    float bg[3];                     /* background colour, added as T_final * bg */
} sgs_camera;

/* Rasteriser options.  Zero-initialised fields take the defaults given. */
typedef struct sgs_options {
    int32_t tile_w, tile_h;          /* 16x16 (default), 8x8, 16x8, 8x16, 32x8 */
    int32_t batch;                   /* LDS batch depth: a multiple of the block size, <= 1024;
                                        0 = 128 */
    float dilation;                  /* added to both diagonal entries of the 2D covariance (0.3) */
    float guard;                     /* guard band on the projection Jacobian, x tan(fov/2) (1.3) */
    float alpha_min;                 /* splats with alpha < alpha_min are skipped (1/255) */
    float alpha_max;                 /* alpha is clamped to alpha_max (0.99) */
    float t_min;                     /* blending stops before T would fall below t_min (1e-4) */
    int32_t pixels_per_thread;       /* forward blend: 1, 2 or 4 pixels per thread (0 = 2); the
                                        block, tile_w*tile_h/ppt threads, must be whole waves */
    int32_t pixels_per_thread_bwd;   /* backward blend, same rule (0 = 4 where allowed) */
    int32_t schedule;                /* tile schedule of both blends: SGS_SCHEDULE_GRID (one
                                        workgroup per tile), SGS_SCHEDULE_QUEUE (persistent
                                        workgroups popping tiles heavy-first from an atomic
                                        counter), SGS_SCHEDULE_SLICES (persistent one-wave
                                        workgroups popping (tile, slice) items heavy-first: a
                                        slice is the pixels one wave of a whole-tile workgroup
                                        owns, and each slice streams the tile's list on its
                                        own); 0 = queue for several cameras, grid for one.
                                        The image does not depend on it. */
} sgs_options;

#define SGS_SCHEDULE_GRID 1
#define SGS_SCHEDULE_QUEUE 2
#define SGS_SCHEDULE_SLICES 3

/* Forward outputs (device, packed over cameras as described above). */
typedef struct sgs_outputs {
    float* image;                    /* [3][H][W] per camera: C + T_final * bg */
    float* depth;                    /* [H][W] sum alpha T z (may be NULL)     */
    float* final_T;                  /* [H][W] transmittance after the last blended splat */
    int32_t* n_contrib;              /* [H][W] 1 + position in the tile list of the last
                                        blended splat, 0 if none */
    float* alpha;                    /* [H][W] accumulated alpha sum alpha_i T_i = 1 - T_final
                                        (may be NULL) */
} sgs_outputs;

/* Byte offsets of the workspace sections, for inspection by tests. */
typedef struct sgs_layout {
    size_t total_bytes;
    size_t header;          /* u32[16]: [0] status bits, [1] pair count P, [2] visible
                               items, [3] forward and [4] backward tile-queue counters,
                               [5] first-level (strip, item) entries, [6] second-level
                               entry chunks */
    size_t cam_table;       /* per camera: int32 W,H,GX,GY,tile_base,strip_base;
                               int64 pix_base; f64 guard limits */
    size_t records;         /* per (camera, Gaussian) item: 64-byte splat record */
    size_t depth_keys;      /* u32 per item: bits of float32 depth, 0xFFFFFFFF if culled */
    size_t tile_rects;      /* u64 per item: tx0 | tx1<<16 | ty0<<32 | ty1<<48; 0 pairs if culled */
    size_t sorted_items;    /* u32 per item: items in ascending (depth key, item) order */
    size_t pair_offsets;    /* u32 per item: exclusive scan, in sorted order, of each
                               item's (strip, item) entries: tile rows times strip
                               columns (a strip: SGS_STRIP_TILES consecutive tiles of a
                               row) of its tile rectangle */
    size_t pair_tiles;      /* binning scratch, capacity entries: strip ids of the
                               first level (u16 when n_strips <= 65536, else u32); the
                               tile of a sorted pair is the one whose range holds it */
    size_t pair_values;     /* u32 per pair: item = camera * n + g, in blend order
                               (tile ascending, then depth key, then item) */
    size_t ranges;          /* u32[2] per global tile: [start, end), (0,0) if empty */
    size_t grad2d;          /* per item a 64-byte record of f32: d/d(u, v, Qa, Qb, Qc,
                               opacity, r, g, b, z) at floats 0-9 (z only when depth or
                               alpha had a gradient), floats 10-15 unused; written for
                               the items the forward kept visible, others unspecified */
    int64_t n_items;        /* n_cams * n */
    int64_t n_tiles;        /* total tiles over all cameras */
    int64_t n_pixels;       /* total pixels over all cameras */
    int64_t pair_capacity;
    int64_t n_strips;       /* row strips over all cameras: per camera, tile rows
                               times ceil(tiles per row / SGS_STRIP_TILES) */
} sgs_layout;

#define SGS_STRIP_TILES 64   /* tiles per row strip of the first binning level */

#define SGS_STATUS_CAPACITY 1u   /* header[0] bit: P exceeded pair_capacity; pairs truncated */
#define SGS_STATUS_CAMERAS  2u   /* header[0] bit: a device camera is invalid or disagrees
                                    with the host cameras' sizes; the blends write nothing */

#define SGS_FLAG_CHECK_CAPACITY 1 /* render_forward: read P on the host after binning */

/*
 * render_workspace_bytes / render_layout
 *   Size (and section offsets) of the workspace for n Gaussians, the given
 *   host cameras (sizes fix the layout; znear, fx, fy are validated) and
 *   options, holding up to
 *   pair_capacity (tile, Gaussian) pairs (< 2^30).  Returns 0 (or
 *   SGS_E_INVALID from render_layout) on invalid arguments.
 */
size_t render_workspace_bytes(const sgs_gaussians* g, const sgs_camera* host_cams,
                              int32_t n_cams, const sgs_options* opts,
                              int64_t pair_capacity);
int render_layout(const sgs_gaussians* g, const sgs_camera* host_cams, int32_t n_cams,
                  const sgs_options* opts, int64_t pair_capacity, sgs_layout* out);

/*
 * render_forward — the forward pass (preprocess, binning, sort, tile ranges,
 * front-to-back compositing).  Paper: Preliminaries (eqs. 2-3 and the EWA
 * projection; depth-sorted splats composited front to back), colour eqs. 4-9.
 *   g           Gaussian parameters (device arrays).
 *   host_cams   n_cams cameras in host memory: fix launch geometry/layout.
 *   dev_cams    the same cameras in device memory: what the kernels read
 *               (poses may change between calls without re-planning).
 *   workspace   device buffer of workspace_bytes >= render_workspace_bytes().
 *               Holds records, pairs and ranges that render_backward reuses:
 *               keep it untouched between a forward and its backward.
 *   outs        packed outputs (device).
 *   flags       SGS_FLAG_CHECK_CAPACITY: synchronise after binning, and if
 *               P > pair_capacity return SGS_E_CAPACITY with *pairs_needed
 *               = P and no image written.  Without it nothing synchronises:
 *               pairs beyond capacity are dropped on the device and status
 *               bit SGS_STATUS_CAPACITY is set (read with render_status).
 *   pairs_needed  optional host pointer, receives P when the flag is set.
 * Camera counts 1..SGS_MAX_CAMERAS; n = 0 renders the background.
 */
int render_forward(const sgs_gaussians* g, const sgs_camera* host_cams,
                   const sgs_camera* dev_cams, int32_t n_cams, const sgs_options* opts,
                   void* workspace, size_t workspace_bytes, int64_t pair_capacity,
                   const sgs_outputs* outs, int32_t flags, int64_t* pairs_needed,
                   void* stream);

/*
 * render_forward_noalloc — render_forward for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation.  Same arguments and results as
 * render_forward, except that the workspace is the library's own
 * no-allocation scratch: a static device array of
 * SGS_NOALLOC_WORKSPACE_BYTES per GPU, reserved when the library's code is
 * loaded on that GPU and held until the process ends.  The call allocates
 * nothing (no hipMalloc, no events: stage timing does not record it).
 *   - The current device must be the one the stream and the buffers live
 *     on; the first call on a device looks up that device's copy of the
 *     array.
 *   - SGS_E_INVALID when render_workspace_bytes() for these arguments
 *     exceeds SGS_NOALLOC_WORKSPACE_BYTES (fewer Gaussians, cameras or
 *     pairs fit).
 *   - Every call on one GPU shares the array, which keeps the last call's
 *     contents (every section the forward reads is written or cleared by
 *     its own kernels first).  Calls that overlap on one GPU (other
 *     streams or threads) race: serialise them.  No render_backward can
 *     follow: its workspace is not exposed.
 */
#define SGS_NOALLOC_WORKSPACE_BYTES (64ull << 20)
int render_forward_noalloc(const sgs_gaussians* g, const sgs_camera* host_cams,
                           const sgs_camera* dev_cams, int32_t n_cams, const sgs_options* opts,
                           int64_t pair_capacity, const sgs_outputs* outs, int32_t flags,
                           int64_t* pairs_needed, void* stream);

/*
 * render_backward — gradients of a scalar loss L w.r.t. every raw
 * parameter, given dL/dimage (device, packed like `image`): the exact
 * derivative of what render_forward computes.  Paper: Preliminaries (the
 * front-to-back compositing C = sum_i c_i a_i prod_{j<i} (1 - a_j) over the
 * depth-sorted splats, a_i from the EWA-projected density of eqs. 2-3),
 * and the colour model of eqs. 4-9 (SH basis, SG lobes a exp(lambda (d.mu
 * - 1)), their sum).  Walks each tile back to front from the saved final
 * transmittance and contributor count, recomputing each alpha, reduces the
 * nine 2D gradients per splat (mean, conic, opacity, rgb), then applies the
 * chain rule through the preprocess to the raw parameters (means through
 * the projection, the EWA Jacobian and the view direction; log-scales and
 * the quaternion through Sigma = R S S^T R^T; the opacity logit; SH
 * coefficients; lobe axes through their normalisation, log-sharpness and
 * amplitudes).  Arguments as render_forward; `workspace` and `fwd` must be
 * those of the matching forward (same g, cameras, options, capacity) and
 * untouched since.  grad_image: dL/dimage (device, packed like `image`).
 * grad_depth, grad_alpha: dL/ddepth and dL/dalpha (device, packed like
 * `depth`; either may be NULL = zero): depth D = sum alpha_i T_i z_i and
 * accumulated alpha A = 1 - T_final then pass gradients to every splat's
 * alpha, and D to its camera depth z (hence to the mean).  `grads`: every
 * array is overwritten (packed layout).  Returns SGS_E_INVALID on a NULL
 * required pointer or a too-small workspace; otherwise enqueues and
 * returns SGS_OK.
 */
int render_backward(const sgs_gaussians* g, const sgs_camera* host_cams,
                    const sgs_camera* dev_cams, int32_t n_cams, const sgs_options* opts,
                    void* workspace, size_t workspace_bytes, int64_t pair_capacity,
                    const sgs_outputs* fwd, const float* grad_image, const float* grad_depth,
                    const float* grad_alpha, const sgs_grads* grads, void* stream);

/*
 * render_l1 — L = sum over cameras of mean_{3 H W} |image - target| and
 * dL/dimage = sign(image - target) / (3 H_k W_k) (sign(0) = 0).
 * image, target, grad_image: packed like `image` (device).  loss: one
 * device double.  Uses the camera table of the workspace of the forward.
 */
int render_l1(const sgs_camera* host_cams, int32_t n_cams, const void* workspace,
              const float* image, const float* target, float* grad_image,
              double* loss, void* stream);

/* render_status — synchronises `stream` and returns header[0] of the
 * workspace (SGS_STATUS_* bits); *pairs receives P when non-NULL. */
int render_status(const void* workspace, uint32_t* status_bits, int64_t* pairs, void* stream);

/* render_read_keys — writes the sorted 64-bit keys (tile << 32 | depth
 * bits) of the first `count` pairs of a finished forward into keys_out
 * (device u64[count]); for parity tests. */
int render_read_keys(const void* workspace, const sgs_layout* layout, int64_t count,
                     uint64_t* keys_out, void* stream);

/*
 * Stage timing.  render_set_timing(1) makes render_forward / render_backward
 * record HIP events between their stages on the call's stream (no host
 * synchronisation is added).  render_stage_times() waits for the recorded
 * events, returns in ms_out[s] the summed milliseconds of stage s over all
 * calls recorded since the previous query, in *n_calls the number of
 * forward calls summed, and forgets them.  Stages are numbered 0..
 * SGS_N_STAGES-1 and named by render_stage_name().  The timing state is
 * per process and not thread-safe.
 */
#define SGS_N_STAGES 11
int render_set_timing(int32_t enable);
int render_stage_times(float* ms_out, int32_t n_out, int32_t* n_calls, int32_t* n_bwd_calls);
const char* render_stage_name(int32_t stage);

/*
 * render_blend_work — re-walks the tiles of a finished forward (same
 * workspace, cameras, options and outputs) and counts the list entries
 * visited by each thread while one of its pixels still blends (counts[0];
 * a thread owns pixels_per_thread pixels of one column and tests the
 * column once per entry), over all pixels the entries whose pixel
 * rectangle holds the pixel, i.e. whose alpha is evaluated (counts[1]), and
 * the entries that blend into the pixel: alpha at least alpha_min and the
 * pixel not stopped by them (counts[2]).  counts: device u64[3],
 * overwritten.  For roofline figures; not part of the render.
 */
int render_blend_work(const sgs_gaussians* g, const sgs_camera* host_cams,
                      const sgs_camera* dev_cams, int32_t n_cams, const sgs_options* opts,
                      const void* workspace, size_t workspace_bytes, int64_t pair_capacity,
                      uint64_t* counts, void* stream);

/*
 * render_blend_bwd_work — walks the tiles of a finished forward back to
 * front as render_backward's blend does (same workspace, cameras, options;
 * fwd: the forward's outputs, of which final_T and n_contrib are read) and
 * counts its work events into counts (device u64[4], overwritten): list
 * entries visited per thread (every thread of a tile visits the entries
 * before the tile's largest n_contrib), (pixel, entry) pairs whose alpha is
 * recomputed (entry before the pixel's n_contrib, pixel inside the splat's
 * rectangle), the pairs among them with alpha >= alpha_min (the pairs that
 * carry a gradient: the blended pairs of the forward), and wave reductions
 * (one per wave and entry that one of the wave's pairs carries: one
 * reduce-scatter and one atomic instruction).  Uses the grid schedule and
 * options.ppt_bwd.  For roofline figures; writes no gradient.
 */
int render_blend_bwd_work(const sgs_gaussians* g, const sgs_camera* host_cams,
                          const sgs_camera* dev_cams, int32_t n_cams, const sgs_options* opts,
                          const void* workspace, size_t workspace_bytes, int64_t pair_capacity,
                          const sgs_outputs* fwd, uint64_t* counts, void* stream);

/*
 * Fused Adam step over every parameter array (the optimiser of the training
 * the rasteriser serves; paper: Experiments, Implementation — the 3D-GS
 * learning rates, and the SG lobes introduced after the first 2,000
 * iterations with learning rate 0.0025).
 *   lr[8]      learning rate per array, in sgs_gaussians order: means,
 *              log_scales, quats, opacity_logits, sh, sg_axes,
 *              sg_log_sharpness, sg_amplitudes (0 leaves an array untouched).
 *   step       1-based iteration of this update (Adam's t for the arrays
 *              that train from the start).
 *   sg_start   the lobe arrays (sg_axes, sg_log_sharpness, sg_amplitudes)
 *              stay untouched, moments included, while step < sg_start; from
 *              there their own t = step - sg_start + 1.  0 or 1: from the start.
 */
typedef struct sgs_adam {
    float lr[8];
    double beta1, beta2, eps;        /* 0 = 0.9, 0.999, 1e-15 (the 3D-GS optimiser's eps); double, so
                                        that 1 - beta is formed before rounding to float32 */
    int32_t step;
    int32_t sg_start;
} sgs_adam;

/*
 * render_adam_step — one Adam update, in float32, of every parameter array
 * of `g` in place (its arrays must be writable device memory, in the
 * layout sgs_gaussians describes, colour_stride included):
 *   m = b1 m + (1 - b1) grad,  v = b2 v + (1 - b2) grad^2,
 *   p -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
 * grads: the gradients render_backward wrote (packed).  exp_avg,
 * exp_avg_sq: the first and second moments, packed like the gradients,
 * caller-owned, zero before the first step (device).  One launch; no
 * allocation, no synchronisation.  SGS_E_INVALID on a NULL array that the
 * form needs, step < 1, a learning rate < 0, or colour_dtype other than
 * SGS_COLOUR_F32 (the update is float32 in place).
 */
int render_adam_step(const sgs_gaussians* g, const sgs_adam* cfg, const sgs_grads* grads,
                     const sgs_grads* exp_avg, const sgs_grads* exp_avg_sq, void* stream);

/* render_last_error — message for the last non-zero return on this thread. */
const char* render_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SGSPLAT_H */
