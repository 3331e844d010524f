// Backward preprocess: chain rule from the per-item 2D gradients to every
// raw parameter, one thread per Gaussian summing over cameras, in two
// kernels so that neither holds both live sets (no register spills):
//
//   k_colour_bwd<DEG, KMAX, LM> (float32): colour eq. 9 -> SH coefficients
//     (eq. 4; only those of the degree each camera used), SG amplitude,
//     log-sharpness and axis (eq. 5) or frame parameters (eq. 8), and the part of the
//     mean's gradient that flows through the view direction; the latter is
//     left in a [3][n] scratch row of the workspace.
//   k_geom_bwd (float64): conic Q = Sigma'^-1 -> Sigma' (dQ = -Q dSigma' Q),
//     Sigma' = M M^T + dilation I with M = J W R S (eq. 3 and the EWA step),
//     J and the projected mean -> camera-space mean (no derivative through
//     the guard clamp where it is active), opacity sigmoid, scale exp and
//     quaternion normalisation; adds the colour part of the mean gradient.
// Both write their outputs once (no atomics, no accumulation across calls).
#include "colour.hpp"

namespace sgs {

__device__ __forceinline__ bool item_visible(const Workspace& ws, int64_t item) {
    const uint64_t tr = ws.tile_rects[item];
    return (int)((tr >> 16) & 0xFFFF) >= (int)(tr & 0xFFFF);
}

// A block takes tiles of kPreTile consecutive Gaussians, one per thread; the
// lanes of a wave whose Gaussians are visible in some camera gather their
// colour records into the wave's LDS buffer (as the forward preprocess
// does).  The
// gradients then go through LDS as one record per Gaussian, so that the
// block writes each gradient array's Gaussian-major tile region (contiguous)
// with consecutive threads on consecutive floats; a Gaussian no camera sees
// gets zeros.
// waves per SIMD asked of the compiler: 4 up to 40 colour rows (no spills
// there); larger forms keep their natural register count
template <int DEG, int KMAX, int LM>
struct ColourBwdWaves {
    static constexpr int rows = 3 * (DEG + 1) * (DEG + 1) + 3 * AxisRows<LM, KMAX>::value + 4 * KMAX;
    static constexpr int value = rows <= 40 ? 4 : (rows <= 48 ? 3 : 1);
};

template <int DEG, int KMAX, int LM, bool AD, int CT>
__global__ void __launch_bounds__(kPreTile)
__attribute__((amdgpu_waves_per_eu(ColourBwdWaves<DEG, KMAX, LM>::value)))
k_colour_bwd(Params p, const sgs_camera* __restrict__ cams, int n_cams, Workspace ws,
             sgs_grads gr, float* __restrict__ gx_colour) {
    constexpr int NC = (DEG + 1) * (DEG + 1);
    constexpr int AMAX = AxisRows<LM, KMAX>::value;
    // record bound: SH, axis rows, sharpness and amplitudes, rounded up to
    // whole 16-byte pieces
    constexpr int MAXROWS = (3 * NC + 3 * AMAX + 4 * KMAX + 3) & ~3;
    // gradient records: an odd stride keeps a wave's record writes on
    // distinct banks
    constexpr int SG = (MAXROWS % 2 == 0) ? MAXROWS + 1 : MAXROWS;
    constexpr int WAVES = kPreTile / 64;
    // first the waves' colour record buffers (64 records each), then the
    // gradient records of the tile
    __shared__ __align__(16) float s_buf[kPreTile * SG];
    __shared__ int64_t s_g[WAVES][64];
    const int64_t n = p.n;
    const int64_t M = ws.n_items;
    const int K = p.n_lobes;
    const int tid = threadIdx.x, wave = tid >> 6;
    const int RS = p.rec_floats;
    const int A3 = LM == kLobesFree ? 3 * K : 3 * AMAX;   // axis floats (3 per free lobe)
    float* crec = s_buf + wave * 64 * MAXROWS;
    // this thread's Gaussian in the next tile: its mean and the first
    // camera's rectangle, loaded while this tile computes (only where the
    // registers allow it without spilling)
    constexpr bool PF = ColourBwdWaves<DEG, KMAX, LM>::value >= 4;
    float nX[3];
    uint64_t nrect;
    auto load = [&](int64_t b) {
        const int64_t gg = b + tid < n ? b + tid : n - 1;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            nX[c] = p.means[c * n + gg];
        }
        nrect = ws.tile_rects[gg];
    };
    if (PF && (int64_t)blockIdx.x * kPreTile < n) load((int64_t)blockIdx.x * kPreTile);
    for (int64_t base = (int64_t)blockIdx.x * kPreTile; base < n;
         base += (int64_t)gridDim.x * kPreTile) {
        __syncthreads();   // the previous tile's records are written out
        const int64_t g = base + tid;
        const bool active = g < n;
        if (!PF) load(base);
        const double X[3] = {nX[0], nX[1], nX[2]};
        const uint64_t rect0 = nrect;
        if (PF && base + (int64_t)gridDim.x * kPreTile < n) load(base + (int64_t)gridDim.x * kPreTile);
        float gsh[NC][3];
        float gamp[KMAX + 1][3], gax[AMAX + 1][3], glsh[KMAX + 1];
#pragma unroll
        for (int l = 0; l < NC; ++l) gsh[l][0] = gsh[l][1] = gsh[l][2] = 0.0f;
#pragma unroll
        for (int k = 0; k < KMAX + 1; ++k) {
            glsh[k] = 0.0f;
            gamp[k][0] = gamp[k][1] = gamp[k][2] = 0.0f;
        }
#pragma unroll
        for (int a = 0; a < AMAX + 1; ++a) gax[a][0] = gax[a][1] = gax[a][2] = 0.0f;
        float gX[3] = {0.0f, 0.0f, 0.0f};
        const int64_t gc = active ? g : n - 1;
        int slot = -1, used = 0;
        for (int ci = 0; ci < n_cams; ++ci) {
            const int64_t item = (int64_t)ci * n + gc;
            const uint64_t tr = PF && ci == 0 ? rect0 : ws.tile_rects[item];
            const bool vis = active && (int)((tr >> 16) & 0xFFFF) >= (int)(tr & 0xFFFF);
            // with registers to spare, issued before the gather's wait
            // (only a visible item's gradient record is read)
            float grgb[3] = {0.0f, 0.0f, 0.0f};
            if constexpr (PF) {
                if (vis) {
#pragma unroll
                    for (int c = 0; c < 3; ++c) grgb[c] = ws.grad2d[item * kG2 + 6 + c];
                }
            }
            const int got = gather_colour<3 * NC, CT>(p, gc, vis && slot < 0, used, crec, s_g[wave], &slot);
            used += got;
            if (got) __builtin_amdgcn_s_waitcnt(0);
            if (!vis) continue;
            if constexpr (!PF) {
#pragma unroll
                for (int c = 0; c < 3; ++c) grgb[c] = ws.grad2d[item * kG2 + 6 + c];
            }
            const char* r = reinterpret_cast<const char*>(crec) + slot * RS * ColourElem<CT>::bytes;
            float d[3], dist;
            view_dir(X, cams[ci], d, &dist);
            float gd[3];
            // adaptive SH: the degree this camera used, from the item's radius
            const int ncu = AD ? sh_used<DEG>(p, ws.records[item].radius) : NC;
            colour_bwd_eval<DEG, KMAX, LM>(
                [&](int l, int c) { return colour_at<CT>(r, 3 * l + c); },
                [&](int k, int j) { return colour_at<CT>(r, 3 * NC + 3 * k + j); },
                [&](int k) { return colour_at<CT>(r, 3 * NC + A3 + k); },
                [&](int k, int c) { return colour_at<CT>(r, 3 * NC + A3 + K + 3 * k + c); }, K, ncu, d[0], d[1],
                d[2], grgb, gsh, gamp, gax, glsh, gd);
            // through d = (X - c) / |X - c|: (I - d d^T) / |X - c|
            const float dd = d[0] * gd[0] + d[1] * gd[1] + d[2] * gd[2];
            const float inv = 1.0f / dist;
#pragma unroll
            for (int c = 0; c < 3; ++c) gX[c] += (gd[c] - d[c] * dd) * inv;
        }
        if (active)
#pragma unroll
            for (int c = 0; c < 3; ++c) gx_colour[c * n + g] = gX[c];
        __syncthreads();   // every wave is done with its colour records
        // record layout with AMAX axis and KMAX lobe slots (compile-time
        // offsets): SH rows, then axis rows at 3 NC + 3 a + c, log-sharpness
        // at 3 NC + 3 AMAX + k, amplitudes at 3 NC + 3 AMAX + KMAX + 3 k + c;
        // slots past the live counts hold zeros
        float* rec = s_buf + tid * SG;
#pragma unroll
        for (int l = 0; l < NC; ++l)
#pragma unroll
            for (int c = 0; c < 3; ++c) rec[3 * l + c] = gsh[l][c];
#pragma unroll
        for (int a = 0; a < AMAX; ++a)
#pragma unroll
            for (int c = 0; c < 3; ++c) rec[3 * NC + 3 * a + c] = gax[a][c];
#pragma unroll
        for (int k = 0; k < KMAX; ++k) {
#pragma unroll
            for (int c = 0; c < 3; ++c) rec[3 * NC + 3 * AMAX + KMAX + 3 * k + c] = gamp[k][c];
            rec[3 * NC + 3 * AMAX + k] = glsh[k];
        }
        __syncthreads();
        // array with S floats per Gaussian at record offset R: the tile's
        // region is `count * S` consecutive floats from Gaussian `base`
        const int count = n - base < kPreTile ? (int)(n - base) : kPreTile;
        auto write_out = [&](float* dst, int S, int R) {
            if (S <= 0) return;
            dst += base * S;
            const float inv_s = 1.0f / (float)S;
            for (int e = tid; e < count * S; e += kPreTile) {
                // e / S through the reciprocal: (e + 0.5) / S is at least
                // 0.5 / S from an integer, far above the rounding error
                const int j = (int)(((float)e + 0.5f) * inv_s);
                dst[e] = s_buf[j * SG + R + (e - j * S)];
            }
        };
        write_out(gr.sh, 3 * NC, 0);
        if (K > 0) {
            write_out(gr.sg_axes, A3, 3 * NC);
            write_out(gr.sg_log_sharpness, K, 3 * NC + 3 * AMAX);
            write_out(gr.sg_amplitudes, 3 * K, 3 * NC + 3 * AMAX + KMAX);
        }
    }
}

__global__ void __launch_bounds__(kPreThreads)
k_geom_bwd(Params p, const sgs_camera* __restrict__ cams, int n_cams, Opts o, Workspace ws,
           sgs_grads gr, const float* __restrict__ gx_colour, bool depth_grad) {
    const int64_t n = p.n;
    const int64_t M = ws.n_items;
    const double dil = o.dilation;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    // inputs of this thread's next Gaussian, loaded while the current one
    // computes: geometry, the colour part of the mean's gradient, the first
    // camera's rectangle and, when that camera sees it, its 2D gradients
    // (u, v, Qa, Qb, Qc, sigma, z).  The rectangles are loaded one Gaussian
    // further ahead, so that the gradient record is fetched only for a
    // visible item without waiting for its rectangle.
    struct In {
        float X[3], ls[3], q[4], logit, gxc[3];
        uint64_t rect0;
        float g0[7];
    };
    auto load = [&](int64_t g, In& in) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            in.X[c] = p.means[c * n + g];
            in.ls[c] = p.log_scales[c * n + g];
            in.gxc[c] = gx_colour[c * n + g];
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) in.q[c] = p.quats[c * n + g];
        in.logit = p.opacity_logits[g];
    };
    auto load_g2 = [&](int64_t g, uint64_t rect, In& in) {
#pragma unroll
        for (int c = 0; c < 7; ++c) in.g0[c] = 0.0f;
        in.rect0 = rect;
        if ((int)((rect >> 16) & 0xFFFF) >= (int)(rect & 0xFFFF)) {   // visible
            const float* r0 = ws.grad2d + g * kG2;
            const float4 a = *reinterpret_cast<const float4*>(r0);
            const float2 b = *reinterpret_cast<const float2*>(r0 + 4);
            in.g0[0] = a.x; in.g0[1] = a.y; in.g0[2] = a.z; in.g0[3] = a.w;
            in.g0[4] = b.x; in.g0[5] = b.y;
            in.g0[6] = depth_grad ? r0[9] : 0.0f;
        }
    };
    In cur;
    int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t rect_n = 1ull;   // the rectangle of this thread's next Gaussian (1: no pairs)
    if (g < n) {
        load(g, cur);
        load_g2(g, ws.tile_rects[g], cur);
        if (g + stride < n) rect_n = ws.tile_rects[g + stride];
    }
    for (; g < n; g += stride) {
        In nxt;
        if (g + stride < n) {
            load(g + stride, nxt);
            load_g2(g + stride, rect_n, nxt);
        }
        if (g + 2 * stride < n) rect_n = ws.tile_rects[g + 2 * stride];
        const float* g0 = cur.g0;
        double gX[3] = {0.0, 0.0, 0.0}, gls[3] = {0.0, 0.0, 0.0}, gq[4] = {0.0, 0.0, 0.0, 0.0};
        double glogit = 0.0;
        const double X[3] = {cur.X[0], cur.X[1], cur.X[2]};
        const double s[3] = {exp((double)cur.ls[0]), exp((double)cur.ls[1]), exp((double)cur.ls[2])};
        const double q[4] = {cur.q[0], cur.q[1], cur.q[2], cur.q[3]};
        const double iq = 1.0 / sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
        const double w = q[0] * iq, x = q[1] * iq, y = q[2] * iq, z = q[3] * iq;
        const double Rq[3][3] = {
            {1.0 - 2.0 * (y * y + z * z), 2.0 * (x * y - w * z), 2.0 * (x * z + w * y)},
            {2.0 * (x * y + w * z), 1.0 - 2.0 * (x * x + z * z), 2.0 * (y * z - w * x)},
            {2.0 * (x * z - w * y), 2.0 * (y * z + w * x), 1.0 - 2.0 * (x * x + y * y)}};
        const double sig = 1.0 / (1.0 + exp(-(double)cur.logit));
        bool any = false;
        for (int ci = 0; ci < n_cams; ++ci) {
            const int64_t item = (int64_t)ci * n + g;
            const uint64_t tr = ci == 0 ? cur.rect0 : ws.tile_rects[item];
            if ((int)((tr >> 16) & 0xFFFF) < (int)(tr & 0xFFFF)) continue;   // not visible
            any = true;
            const sgs_camera& cam = cams[ci];
            const CamTable ct = ws.cams[ci];
            float g2d[7];
#pragma unroll
            for (int c = 0; c < 6; ++c) g2d[c] = ci == 0 ? g0[c] : ws.grad2d[item * kG2 + c];
            g2d[6] = ci == 0 ? g0[6] : (depth_grad ? ws.grad2d[item * kG2 + 9] : 0.0f);
            const double gu = g2d[0], gv = g2d[1];
            // depth z = x_cam[2] carries dL/dz from the blend when depth or
            // alpha had an upstream gradient
            const double gzd = depth_grad ? (double)g2d[6] : 0.0;
            const double gQa = g2d[2], gQb = g2d[3];
            const double gQc = g2d[4];
            glogit += (double)g2d[5] * sig * (1.0 - sig);
            const double fx = cam.fx, fy = cam.fy;
            double xc[3];
            for (int i = 0; i < 3; ++i)
                xc[i] = (double)cam.R[3 * i] * X[0] + (double)cam.R[3 * i + 1] * X[1] +
                        (double)cam.R[3 * i + 2] * X[2] + (double)cam.t[i];
            const double iz = 1.0 / xc[2];
            const double xn = xc[0] * iz, yn = xc[1] * iz;
            const bool clx = xn < -ct.limx || xn > ct.limx;
            const bool cly = yn < -ct.limy || yn > ct.limy;
            const double xnc = fmin(fmax(xn, -ct.limx), ct.limx);
            const double ync = fmin(fmax(yn, -ct.limy), ct.limy);
            const double J00 = fx * iz, J02 = -(fx * xnc) * iz;
            const double J11 = fy * iz, J12 = -(fy * ync) * iz;
            // T2 = J W
            double T2[2][3];
            for (int k = 0; k < 3; ++k) {
                T2[0][k] = J00 * (double)cam.R[k] + J02 * (double)cam.R[6 + k];
                T2[1][k] = J11 * (double)cam.R[3 + k] + J12 * (double)cam.R[6 + k];
            }
            // M = T2 R diag(s)
            double Mm[2][3];
            for (int i = 0; i < 2; ++i)
                for (int a = 0; a < 3; ++a)
                    Mm[i][a] = (T2[i][0] * Rq[0][a] + T2[i][1] * Rq[1][a] + T2[i][2] * Rq[2][a]) * s[a];
            const double pp = Mm[0][0] * Mm[0][0] + Mm[0][1] * Mm[0][1] + Mm[0][2] * Mm[0][2];
            const double qq = Mm[1][0] * Mm[1][0] + Mm[1][1] * Mm[1][1] + Mm[1][2] * Mm[1][2];
            const double A = pp + dil, C = qq + dil;
            const double B = Mm[0][0] * Mm[1][0] + Mm[0][1] * Mm[1][1] + Mm[0][2] * Mm[1][2];
            const double crx = Mm[0][1] * Mm[1][2] - Mm[0][2] * Mm[1][1];
            const double cry = Mm[0][2] * Mm[1][0] - Mm[0][0] * Mm[1][2];
            const double crz = Mm[0][0] * Mm[1][1] - Mm[0][1] * Mm[1][0];
            const double det = crx * crx + cry * cry + crz * crz + dil * (pp + qq) + dil * dil;
            const double id2 = 1.0 / (det * det);
            // conic -> Sigma'
            const double gA = (-C * C * gQa + B * C * gQb - B * B * gQc) * id2;
            const double gC = (-B * B * gQa + A * B * gQb - A * A * gQc) * id2;
            const double gB = (2.0 * B * C * gQa - (A * C + B * B) * gQb + 2.0 * A * B * gQc) * id2;
            // Sigma' = M M^T + dil I -> M
            double gM[2][3];
            for (int a = 0; a < 3; ++a) {
                gM[0][a] = 2.0 * gA * Mm[0][a] + gB * Mm[1][a];
                gM[1][a] = gB * Mm[0][a] + 2.0 * gC * Mm[1][a];
            }
            // M[i][a] = (T2 R)[i][a] s[a]: to log s, to R (then q), to T2 (then J)
            double gR[3][3], gT2[2][3] = {{0, 0, 0}, {0, 0, 0}};
            for (int a = 0; a < 3; ++a) {
                gls[a] += gM[0][a] * Mm[0][a] + gM[1][a] * Mm[1][a];
                const double ga0 = gM[0][a] * s[a], ga1 = gM[1][a] * s[a];
                for (int m = 0; m < 3; ++m) {
                    gR[m][a] = T2[0][m] * ga0 + T2[1][m] * ga1;
                    gT2[0][m] += ga0 * Rq[m][a];
                    gT2[1][m] += ga1 * Rq[m][a];
                }
            }
            gq[0] += 2.0 * (-z * gR[0][1] + y * gR[0][2] + z * gR[1][0] - x * gR[1][2] -
                            y * gR[2][0] + x * gR[2][1]);
            gq[1] += 2.0 * (y * gR[0][1] + z * gR[0][2] + y * gR[1][0] - 2.0 * x * gR[1][1] -
                            w * gR[1][2] + z * gR[2][0] + w * gR[2][1] - 2.0 * x * gR[2][2]);
            gq[2] += 2.0 * (-2.0 * y * gR[0][0] + x * gR[0][1] + w * gR[0][2] + x * gR[1][0] +
                            z * gR[1][2] - w * gR[2][0] + z * gR[2][1] - 2.0 * y * gR[2][2]);
            gq[3] += 2.0 * (-2.0 * z * gR[0][0] - w * gR[0][1] + x * gR[0][2] + w * gR[1][0] -
                            2.0 * z * gR[1][1] + y * gR[1][2] + x * gR[2][0] + y * gR[2][1]);
            // T2 = J W -> J entries
            double gJ00 = 0, gJ02 = 0, gJ11 = 0, gJ12 = 0;
            for (int k = 0; k < 3; ++k) {
                gJ00 += gT2[0][k] * (double)cam.R[k];
                gJ02 += gT2[0][k] * (double)cam.R[6 + k];
                gJ11 += gT2[1][k] * (double)cam.R[3 + k];
                gJ12 += gT2[1][k] * (double)cam.R[6 + k];
            }
            // J and (u, v) -> camera-space mean
            const double iz2 = iz * iz;
            double g0 = gu * fx * iz, g1 = gv * fy * iz;
            double g2 = -(gJ00 * fx + gJ11 * fy) * iz2 - (gu * fx * xc[0] + gv * fy * xc[1]) * iz2 + gzd;
            if (clx) {
                g2 += gJ02 * fx * xnc * iz2;
            } else {
                g0 += -gJ02 * fx * iz2;
                g2 += 2.0 * gJ02 * fx * xc[0] * iz2 * iz;
            }
            if (cly) {
                g2 += gJ12 * fy * ync * iz2;
            } else {
                g1 += -gJ12 * fy * iz2;
                g2 += 2.0 * gJ12 * fy * xc[1] * iz2 * iz;
            }
            for (int j = 0; j < 3; ++j)
                gX[j] += (double)cam.R[j] * g0 + (double)cam.R[3 + j] * g1 + (double)cam.R[6 + j] * g2;
        }
        const double dq = w * gq[0] + x * gq[1] + y * gq[2] + z * gq[3];
        const double qh[4] = {w, x, y, z};
        for (int c = 0; c < 3; ++c) {
            gr.means[c * n + g] = (float)(gX[c] + (any ? (double)cur.gxc[c] : 0.0));
            gr.log_scales[c * n + g] = (float)gls[c];
        }
        for (int c = 0; c < 4; ++c) gr.quats[c * n + g] = (float)((gq[c] - qh[c] * dq) * iq);
        gr.opacity_logits[g] = (float)glogit;
        cur = nxt;
    }
}

void launch_preprocess_bwd(const Params& p, const sgs_camera* dev_cams, int n_cams, const Opts& o,
                           const Workspace& ws, const sgs_grads& gr, bool depth_grad,
                           hipStream_t s) {
    if (p.n <= 0) return;
    int64_t blocks = (p.n + kPreThreads - 1) / kPreThreads;
    if (blocks > 4096) blocks = 4096;
    dim3 grid((unsigned)blocks), block(kPreThreads);
    float* gxc = ws.gx_colour;
    const int64_t tiles = (p.n + kPreTile - 1) / kPreTile;
    const dim3 cgrid((unsigned)(tiles < 4096 ? tiles : 4096)), cblock(kPreTile);
    // adaptive SH degree is its own instantiation (compile-time loop bounds
    // otherwise)
    const bool ad = (p.sh_ad0 | p.sh_ad1) != 0 && p.sh_degree > 0;
#define SGS_COLOUR_BWD1(D, K, LM, A, C)                                                        \
    hipLaunchKernelGGL((k_colour_bwd<D, K, LM, A, C>), cgrid, cblock, 0, s, p, dev_cams, n_cams, \
                       ws, gr, gxc)
    // colour element type: bfloat16 / float16 storage only with a fixed SH
    // degree (the host checks)
#define SGS_COLOUR_BWD(D, K, LM)                                                               \
    if (p.colour_type == kColourBF16) SGS_COLOUR_BWD1(D, K, LM, false, kColourBF16);           \
    else if (p.colour_type == kColourF16) SGS_COLOUR_BWD1(D, K, LM, false, kColourF16);        \
    else if (ad) SGS_COLOUR_BWD1(D, K, LM, (D > 0), kColourF32);                               \
    else SGS_COLOUR_BWD1(D, K, LM, false, kColourF32)
#define SGS_COLOUR_BWD_K(D)                                                                    \
    if (p.lobe_mode == kLobesWorld) SGS_COLOUR_BWD(D, 3, kLobesWorld);                         \
    else if (p.lobe_mode == kLobesFrame) SGS_COLOUR_BWD(D, 3, kLobesFrame);                    \
    else if (p.n_lobes == 0) SGS_COLOUR_BWD(D, 0, kLobesFree);                                 \
    else if (p.n_lobes <= 4) SGS_COLOUR_BWD(D, 4, kLobesFree);                                 \
    else SGS_COLOUR_BWD(D, 8, kLobesFree)
    switch (p.sh_degree) {
        case 0: SGS_COLOUR_BWD_K(0); break;
        case 1: SGS_COLOUR_BWD_K(1); break;
        case 2: SGS_COLOUR_BWD_K(2); break;
        default: SGS_COLOUR_BWD_K(3); break;
    }
#undef SGS_COLOUR_BWD_K
#undef SGS_COLOUR_BWD
#undef SGS_COLOUR_BWD1
    hipLaunchKernelGGL(k_geom_bwd, grid, block, 0, s, p, dev_cams, n_cams, o, ws, gr, gxc, depth_grad);
}

}  // namespace sgs
