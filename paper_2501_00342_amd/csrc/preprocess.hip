// Forward preprocess: one thread per Gaussian, all cameras.
//
// Per Gaussian and camera (SG-Splatting Preliminaries and Methods):
//   covariance Sigma = R S S^T R^T from the quaternion and scales (eq. 3),
//   EWA projection Sigma' = J W Sigma W^T J^T + dilation I, the 3-sigma
//   radius, the integer pixel and tile rectangles, the depth key, and the
//   colour of eq. 9: low-degree SH (eq. 4, optionally of a degree chosen by
//   the projected radius) plus K SG lobes (eq. 5-7) on free axes, the world
//   axes or a per-Gaussian orthonormal frame (eq. 8).
//
// This file is compiled with -ffp-contract=off: the values that decide
// integers (cull, radius, rectangles, depth key) follow one fixed sequence
// of IEEE float64 operations, sums left to right, no fused multiply-add.
// The colour is image-path only and runs in float32 (explicit fmaf); the
// culling tests on the colour parameters look only at the inputs.
//
// Memory: every parameter array is read once with unit-stride (coalesced)
// loads; outputs are one 64-byte record, a depth key and a packed tile
// rectangle per (camera, Gaussian).
#include "common.hpp"
#include "colour.hpp"

namespace sgs {

struct Geo {
    bool visible;
    double xc0, xc1, z;
    double A, B, C, det, lam1;
    double u, v;
    int radius, px0, px1, py0, py1;
};

__device__ __forceinline__ bool finite_d(double x) { return isfinite(x); }

// Fixed-order float64 key path.  Every line is one rounding step as written.
__device__ __forceinline__ Geo project(const double X[3], const double ls[3], const double q[4],
                                       const sgs_camera& cam, const CamTable& ct, const Opts& o) {
    Geo r;
    const double R0 = cam.R[0], R1 = cam.R[1], R2 = cam.R[2];
    const double R3 = cam.R[3], R4 = cam.R[4], R5 = cam.R[5];
    const double R6 = cam.R[6], R7 = cam.R[7], R8 = cam.R[8];
    const double fx = cam.fx, fy = cam.fy, cx = cam.cx, cy = cam.cy;
    const int W = cam.width, H = cam.height;
    // camera-space mean
    const double xc0 = ((R0 * X[0] + R1 * X[1]) + R2 * X[2]) + (double)cam.t[0];
    const double xc1 = ((R3 * X[0] + R4 * X[1]) + R5 * X[2]) + (double)cam.t[1];
    const double z = ((R6 * X[0] + R7 * X[1]) + R8 * X[2]) + (double)cam.t[2];
    r.xc0 = xc0;
    r.xc1 = xc1;
    r.z = z;
    // activations
    const double s0 = exp(ls[0]), s1 = exp(ls[1]), s2 = exp(ls[2]);
    const double qn = sqrt(((q[0] * q[0] + q[1] * q[1]) + q[2] * q[2]) + q[3] * q[3]);
    const double iq = 1.0 / qn;
    const double w = q[0] * iq, x = q[1] * iq, y = q[2] * iq, zq = q[3] * iq;
    // rotation of the unit quaternion, then M3 = R diag(s)
    const double r00 = 1.0 - 2.0 * (y * y + zq * zq), r01 = 2.0 * (x * y - w * zq), r02 = 2.0 * (x * zq + w * y);
    const double r10 = 2.0 * (x * y + w * zq), r11 = 1.0 - 2.0 * (x * x + zq * zq), r12 = 2.0 * (y * zq - w * x);
    const double r20 = 2.0 * (x * zq - w * y), r21 = 2.0 * (y * zq + w * x), r22 = 1.0 - 2.0 * (x * x + y * y);
    const double m00 = r00 * s0, m01 = r01 * s1, m02 = r02 * s2;
    const double m10 = r10 * s0, m11 = r11 * s1, m12 = r12 * s2;
    const double m20 = r20 * s0, m21 = r21 * s1, m22 = r22 * s2;
    // Jacobian of the perspective map, evaluated inside the guard band
    const double iz = 1.0 / z;
    const double xn = xc0 * iz;
    const double yn = xc1 * iz;
    const double limx = ct.limx, limy = ct.limy;   // guard * ((0.5 W) / fx), per camera
    const double xnc = fmin(fmax(xn, -limx), limx);
    const double ync = fmin(fmax(yn, -limy), limy);
    const double J00 = fx * iz;
    const double J02 = -(fx * xnc) * iz;
    const double J11 = fy * iz;
    const double J12 = -(fy * ync) * iz;
    // T2 = J W (2x3)
    const double t00 = J00 * R0 + J02 * R6, t01 = J00 * R1 + J02 * R7, t02 = J00 * R2 + J02 * R8;
    const double t10 = J11 * R3 + J12 * R6, t11 = J11 * R4 + J12 * R7, t12 = J11 * R5 + J12 * R8;
    // M = T2 M3 (2x3); Sigma' = M M^T + dilation I
    const double a0 = (t00 * m00 + t01 * m10) + t02 * m20;
    const double a1 = (t00 * m01 + t01 * m11) + t02 * m21;
    const double a2 = (t00 * m02 + t01 * m12) + t02 * m22;
    const double b0 = (t10 * m00 + t11 * m10) + t12 * m20;
    const double b1 = (t10 * m01 + t11 * m11) + t12 * m21;
    const double b2 = (t10 * m02 + t11 * m12) + t12 * m22;
    const double pp = (a0 * a0 + a1 * a1) + a2 * a2;
    const double qq = (b0 * b0 + b1 * b1) + b2 * b2;
    const double bb = (a0 * b0 + a1 * b1) + a2 * b2;
    const double dil = o.dilation;
    const double A = pp + dil;
    const double C = qq + dil;
    const double B = bb;
    // det = AC - B^2 through the Lagrange identity |a x b|^2 = |a|^2|b|^2 - (a.b)^2
    const double cx_ = a1 * b2 - a2 * b1;
    const double cy_ = a2 * b0 - a0 * b2;
    const double cz_ = a0 * b1 - a1 * b0;
    const double det = (((cx_ * cx_ + cy_ * cy_) + cz_ * cz_) + dil * (pp + qq)) + dil * dil;
    const double h = (A - C) * 0.5;
    const double lam1 = (A + C) * 0.5 + sqrt(h * h + B * B);
    const double rad = ceil(3.0 * sqrt(lam1));
    const double u = fx * xn + cx;
    const double v = fy * yn + cy;
    const double lox = ceil(u - rad), hix = floor(u + rad);
    const double loy = ceil(v - rad), hiy = floor(v + rad);
    r.A = A;
    r.B = B;
    r.C = C;
    r.det = det;
    r.lam1 = lam1;
    r.u = u;
    r.v = v;
    bool vis = (z > (double)cam.znear) && finite_d(A) && finite_d(B) && finite_d(C) &&
               finite_d(det) && finite_d(lam1) && finite_d(u) && finite_d(v);
    vis = vis && lox <= (double)(W - 1) && hix >= 0.0 && loy <= (double)(H - 1) && hiy >= 0.0;
    r.visible = vis;
    // clamped into the image whether visible or not (equal to the plain
    // max/min for visible Gaussians), so every conversion is in range
    const double wm = (double)(W - 1), hm = (double)(H - 1);
    r.radius = (int)fmin(rad, 1.0e9);
    r.px0 = (int)fmin(fmax(lox, 0.0), wm);
    r.px1 = (int)fmax(fmin(hix, wm), 0.0);
    r.py0 = (int)fmin(fmax(loy, 0.0), hm);
    r.py1 = (int)fmax(fmin(hiy, hm), 0.0);
    return r;
}

// A block takes tiles of kPreTile consecutive Gaussians, one per thread.
// The float64 geometry comes first; the lanes of a wave whose Gaussians are
// visible in a camera then gather their colour records into the wave's LDS
// buffer together (once per tile, at the first camera that sees each), so
// culled Gaussians never fetch colour and the waves need no barrier.  The
// next tile's geometry is loaded into registers while this tile computes,
// so only the colour gather's latency is exposed per tile.  The colour is
// evaluated from LDS, so the geometry's and the colour's registers are never
// live together.
template <int DEG, int KMAX, int LM, bool AD, int CT>
__global__ void __launch_bounds__(kPreTile)
k_preprocess(Params p, const sgs_camera* __restrict__ cams, int n_cams, Opts o, Workspace ws) {
    constexpr int NC = (DEG + 1) * (DEG + 1);
    // record bound: the largest record rounded up to whole 16-byte pieces (a
    // record is read in 16-byte pieces only when its stride leaves that room)
    constexpr int MAXROWS = (3 * NC + 3 * AxisRows<LM, KMAX>::value + 4 * KMAX + 3) & ~3;
    constexpr int WAVES = kPreTile / 64;
    __shared__ __align__(16) float s_rec[WAVES][64 * (MAXROWS > 0 ? MAXROWS : 1)];
    __shared__ int64_t s_g[WAVES][64];
    const int64_t n = p.n;
    const int tid = threadIdx.x, wave = tid >> 6;
    const int RS = p.rec_floats;
    float* rec = s_rec[wave];
    // device cameras that disagree with the plan (status bit set by the
    // setup kernel): every item is culled, so no tile id outside the planned
    // range reaches binning
    const bool cams_ok = (ws.header[kHdrStatus] & SGS_STATUS_CAMERAS) == 0;
    // geometry of this thread's Gaussian in the next tile: 3 + 3 + 4 + 1 floats
    float nxt[11];
    auto load_geometry = [&](int64_t base) {
        const int64_t g0 = base + tid;
        const int64_t g = g0 < n ? g0 : n - 1;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            nxt[c] = p.means[c * n + g];
            nxt[3 + c] = p.log_scales[c * n + g];
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) nxt[6 + c] = p.quats[c * n + g];
        nxt[10] = p.opacity_logits[g];
    };
    if ((int64_t)blockIdx.x * kPreTile < n) load_geometry((int64_t)blockIdx.x * kPreTile);
    for (int64_t base = (int64_t)blockIdx.x * kPreTile; base < n;
         base += (int64_t)gridDim.x * kPreTile) {
        const int64_t g0 = base + tid;
        const bool active = g0 < n;
        const int64_t g = active ? g0 : n - 1;
        double X[3], ls[3], q[4];
        bool finite = true;
        for (int c = 0; c < 3; ++c) {
            X[c] = nxt[c];
            ls[c] = nxt[3 + c];
            finite = finite && finite_d(X[c]) && finite_d(ls[c]);
        }
        for (int c = 0; c < 4; ++c) {
            q[c] = nxt[6 + c];
            finite = finite && finite_d(q[c]);
        }
        const float logit = nxt[10];
        finite = finite && isfinite(logit);
        const float opacity = 1.0f / (1.0f + fast_exp(-logit));
        const int64_t next = base + (int64_t)gridDim.x * kPreTile;
        if (next < n) load_geometry(next);

        int slot = -1;    // this lane's colour record in the wave's buffer
        int used = 0;     // records gathered by the wave in this tile (uniform)
        for (int ci = 0; ci < n_cams; ++ci) {
            const sgs_camera& cam = cams[ci];
            const CamTable ct = ws.cams[ci];
            const int64_t item = (int64_t)ci * n + g;
            const Geo geo = project(X, ls, q, cam, ct, o);
            bool vis = active && finite && geo.visible && cams_ok;
            const int got = gather_colour<3 * NC, CT>(p, g, vis && slot < 0, used, rec, s_g[wave], &slot);
            used += got;
            // this wave's direct loads have landed (it reads only its own buffer)
            if (got) __builtin_amdgcn_s_waitcnt(0);
            float rgb[3] = {0.0f, 0.0f, 0.0f};
            if (vis) {
                float d[3], dist;
                view_dir(X, cam, d, &dist);
                const char* r = reinterpret_cast<const char*>(rec) + slot * RS * ColourElem<CT>::bytes;
                const int K = p.n_lobes, A3 = 3 * p.n_axes;
                vis = colour_eval<DEG, KMAX, LM>(
                    [&](int l, int c) { return colour_at<CT>(r, 3 * l + c); },
                    [&](int k, int j) { return colour_at<CT>(r, 3 * NC + 3 * k + j); },
                    [&](int k) { return colour_at<CT>(r, 3 * NC + A3 + k); },
                    [&](int k, int c) { return colour_at<CT>(r, 3 * NC + A3 + K + 3 * k + c); }, K,
                    AD ? sh_used<DEG>(p, geo.radius) : NC, d[0], d[1], d[2], rgb);
            }
            if (!active) continue;
            uint32_t key = 0xFFFFFFFFu;
            uint64_t trect = 1;  // tx0 = 1 > tx1 = 0: no pairs
            if (vis) {
                const int TW = o.tile_w, TH = o.tile_h;
                const int tx0 = geo.px0 / TW, tx1 = geo.px1 / TW;
                const int ty0 = geo.py0 / TH, ty1 = geo.py1 / TH;
                trect = (uint64_t)tx0 | ((uint64_t)tx1 << 16) | ((uint64_t)ty0 << 32) |
                        ((uint64_t)ty1 << 48);
                const float zf = (float)geo.z;
                key = __float_as_uint(zf);
                // whitening of the conic Q = Sigma'^-1 along its eigenvectors
                const double A = geo.A, B = geo.B, C = geo.C;
                const double il1 = 1.0 / geo.lam1;
                const double lam2 = geo.det * il1;
                double v0, v1;
                if (A >= C) {
                    v0 = geo.lam1 - C;
                    v1 = B;
                } else {
                    v0 = B;
                    v1 = geo.lam1 - A;
                }
                // eigenvector of lambda_1 (difference in float64, normalised in float32)
                float f0 = (float)v0, f1 = (float)v1;
                const float fn2 = f0 * f0 + f1 * f1;
                if (fn2 > 0.0f) {
                    const float ivn = rsqrtf(fn2);
                    f0 *= ivn;
                    f1 *= ivn;
                } else {
                    f0 = 1.0f;
                    f1 = 0.0f;
                }
                const float k1 = sqrtf((float)(kHalfLog2e * il1));
                const float k2 = sqrtf((float)(kHalfLog2e / lam2));
                const float u_hi = (float)geo.u, v_hi = (float)geo.v;
                float4* dst = reinterpret_cast<float4*>(ws.records + item);
                // layout of Rec: u_hi v_hi u_lo v_lo | w1 w2 | opacity rgb | z rect_x rect_y radius
                dst[0] = make_float4(u_hi, v_hi, (float)(geo.u - (double)u_hi),
                                     (float)(geo.v - (double)v_hi));
                dst[1] = make_float4(f0 * k1, f1 * k1, -f1 * k2, f0 * k2);
                dst[2] = make_float4(opacity, fmaxf(rgb[0], 0.0f), fmaxf(rgb[1], 0.0f),
                                     fmaxf(rgb[2], 0.0f));
                dst[3] = make_float4(zf, __uint_as_float((uint32_t)geo.px0 | ((uint32_t)geo.px1 << 16)),
                                     __uint_as_float((uint32_t)geo.py0 | ((uint32_t)geo.py1 << 16)),
                                     __int_as_float(geo.radius));
            }
            ws.depth_keys[item] = key;
            ws.tile_rects[item] = trect;
        }
    }
}

template <int KMAX, int LM>
static void launch_pre_k(const Params& p, const sgs_camera* dev_cams, int n_cams, const Opts& o,
                         const Workspace& ws, dim3 grid, hipStream_t s) {
    const dim3 block(kPreTile);
    // adaptive SH degree is its own instantiation: with a fixed degree the
    // coefficient loops keep a compile-time bound
    const bool ad = (p.sh_ad0 | p.sh_ad1) != 0;
    // colour element type: float32, or bfloat16 / float16 storage (those
    // with a fixed SH degree only; the host checks)
#define SGS_PRE(D, A, C) hipLaunchKernelGGL((k_preprocess<D, KMAX, LM, A, C>), grid, block, 0, s, p, dev_cams, n_cams, o, ws)
#define SGS_PRE_T(D)                                                                       \
    if (p.colour_type == kColourBF16) SGS_PRE(D, false, kColourBF16);                      \
    else if (p.colour_type == kColourF16) SGS_PRE(D, false, kColourF16);                   \
    else if (ad && D > 0) SGS_PRE(D, (D > 0), kColourF32);                                 \
    else SGS_PRE(D, false, kColourF32)
    switch (p.sh_degree) {
        case 0: SGS_PRE_T(0); break;
        case 1: SGS_PRE_T(1); break;
        case 2: SGS_PRE_T(2); break;
        default: SGS_PRE_T(3); break;
    }
#undef SGS_PRE_T
#undef SGS_PRE
}

void launch_preprocess(const Params& p, const sgs_camera* dev_cams, int n_cams, const Opts& o,
                       const Workspace& ws, int hist_blocks, hipStream_t s) {
    (void)hist_blocks;
    // persistent: up to 16 blocks of two waves per CU
    const int64_t tiles = (p.n + kPreTile - 1) / kPreTile;
    const dim3 grid((unsigned)(tiles < 4096 ? (tiles < 1 ? 1 : tiles) : 4096));
    // the orthogonal modes have exactly three lobes (checked on the host)
    if (p.lobe_mode == kLobesWorld) launch_pre_k<3, kLobesWorld>(p, dev_cams, n_cams, o, ws, grid, s);
    else if (p.lobe_mode == kLobesFrame) launch_pre_k<3, kLobesFrame>(p, dev_cams, n_cams, o, ws, grid, s);
    else if (p.n_lobes == 0) launch_pre_k<0, kLobesFree>(p, dev_cams, n_cams, o, ws, grid, s);
    else if (p.n_lobes <= 4) launch_pre_k<4, kLobesFree>(p, dev_cams, n_cams, o, ws, grid, s);
    else launch_pre_k<SGS_MAX_LOBES, kLobesFree>(p, dev_cams, n_cams, o, ws, grid, s);
}

}  // namespace sgs
