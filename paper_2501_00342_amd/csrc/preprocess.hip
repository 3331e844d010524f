// Forward preprocess: one thread per Gaussian, all cameras.
//
// Per Gaussian and camera (SG-Splatting Preliminaries and Methods):
//   covariance Sigma = R S S^T R^T from the quaternion and scales (eq. 3),
//   EWA projection Sigma' = J W Sigma W^T J^T + dilation I, the 3-sigma
//   radius, the integer pixel and tile rectangles, the depth key, and the
//   colour of eq. 9: low-degree SH (eq. 4) plus K SG lobes (eq. 5-7).
//
// This file is compiled with -ffp-contract=off: the values that decide
// integers (cull, radius, rectangles, depth key) follow one fixed sequence
// of IEEE float64 operations, sums left to right, no fused multiply-add.
//
// Memory: every parameter array is read once with unit-stride (coalesced)
// loads; outputs are one 64-byte record, a depth key and a packed tile
// rectangle per (camera, Gaussian).  The depth-key digit histograms for the
// depth sort are accumulated here in LDS (no extra pass over the keys).
#include "common.hpp"
#include "sh_basis.hpp"

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
                                       const sgs_camera& cam, const Opts& o) {
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
    const double w = q[0] / qn, x = q[1] / qn, y = q[2] / qn, zq = q[3] / qn;
    // rotation of the unit quaternion, then M3 = R diag(s)
    const double r00 = 1.0 - 2.0 * (y * y + zq * zq), r01 = 2.0 * (x * y - w * zq), r02 = 2.0 * (x * zq + w * y);
    const double r10 = 2.0 * (x * y + w * zq), r11 = 1.0 - 2.0 * (x * x + zq * zq), r12 = 2.0 * (y * zq - w * x);
    const double r20 = 2.0 * (x * zq - w * y), r21 = 2.0 * (y * zq + w * x), r22 = 1.0 - 2.0 * (x * x + y * y);
    const double m00 = r00 * s0, m01 = r01 * s1, m02 = r02 * s2;
    const double m10 = r10 * s0, m11 = r11 * s1, m12 = r12 * s2;
    const double m20 = r20 * s0, m21 = r21 * s1, m22 = r22 * s2;
    // Jacobian of the perspective map, evaluated inside the guard band
    const double xn = xc0 / z;
    const double yn = xc1 / z;
    const double limx = (double)o.guard * ((0.5 * W) / fx);
    const double limy = (double)o.guard * ((0.5 * H) / fy);
    const double xnc = fmin(fmax(xn, -limx), limx);
    const double ync = fmin(fmax(yn, -limy), limy);
    const double J00 = fx / z;
    const double J02 = -(fx * xnc) / z;
    const double J11 = fy / z;
    const double J12 = -(fy * ync) / z;
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
    if (vis) {
        r.radius = (int)rad;
        r.px0 = (int)fmax(lox, 0.0);
        r.px1 = (int)fmin(hix, (double)(W - 1));
        r.py0 = (int)fmax(loy, 0.0);
        r.py1 = (int)fmin(hiy, (double)(H - 1));
    } else {
        r.radius = r.px0 = r.px1 = r.py0 = r.py1 = 0;
    }
    return r;
}

template <int DEG>
__global__ void __launch_bounds__(kPreThreads)
k_preprocess(Params p, const sgs_camera* __restrict__ cams, int n_cams, Opts o, Workspace ws) {
    constexpr int NC = (DEG + 1) * (DEG + 1);
    __shared__ uint32_t hist[kDepthPasses][kRadix];
    for (int i = threadIdx.x; i < kDepthPasses * kRadix; i += blockDim.x) (&hist[0][0])[i] = 0;
    __syncthreads();

    const int64_t n = p.n;
    const int K = p.n_lobes;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n;
         g += (int64_t)gridDim.x * blockDim.x) {
        double X[3], ls[3], q[4];
        bool finite = true;
        for (int c = 0; c < 3; ++c) {
            X[c] = p.means[c * n + g];
            ls[c] = p.log_scales[c * n + g];
            finite = finite && finite_d(X[c]) && finite_d(ls[c]);
        }
        for (int c = 0; c < 4; ++c) {
            q[c] = p.quats[c * n + g];
            finite = finite && finite_d(q[c]);
        }
        const double logit = p.opacity_logits[g];
        finite = finite && finite_d(logit);
        float shc[NC][3];
        for (int l = 0; l < NC; ++l)
            for (int c = 0; c < 3; ++c) {
                shc[l][c] = p.sh[((int64_t)l * 3 + c) * n + g];
                finite = finite && isfinite(shc[l][c]);
            }
        for (int k = 0; k < K; ++k) {
            for (int c = 0; c < 3; ++c) {
                finite = finite && isfinite(p.sg_axes[((int64_t)k * 3 + c) * n + g]) &&
                         isfinite(p.sg_amplitudes[((int64_t)k * 3 + c) * n + g]);
            }
            finite = finite && isfinite(p.sg_log_sharpness[(int64_t)k * n + g]);
        }
        const double opacity = 1.0 / (1.0 + exp(-logit));

        for (int ci = 0; ci < n_cams; ++ci) {
            const sgs_camera& cam = cams[ci];
            const int64_t item = (int64_t)ci * n + g;
            Geo geo = project(X, ls, q, cam, o);
            bool vis = finite && geo.visible;
            double rgb[3] = {0.0, 0.0, 0.0};
            if (vis) {
                // view direction: camera centre -> mean, c = -R^T t
                const double cc0 = -(((double)cam.R[0] * cam.t[0] + (double)cam.R[3] * cam.t[1]) + (double)cam.R[6] * cam.t[2]);
                const double cc1 = -(((double)cam.R[1] * cam.t[0] + (double)cam.R[4] * cam.t[1]) + (double)cam.R[7] * cam.t[2]);
                const double cc2 = -(((double)cam.R[2] * cam.t[0] + (double)cam.R[5] * cam.t[1]) + (double)cam.R[8] * cam.t[2]);
                double d0 = X[0] - cc0, d1 = X[1] - cc1, d2 = X[2] - cc2;
                const double dn = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
                d0 /= dn;
                d1 /= dn;
                d2 /= dn;
                double Y[NC];
                sh_eval<DEG>(d0, d1, d2, Y);
                for (int c = 0; c < 3; ++c) {
                    double acc = 0.5;
                    for (int l = 0; l < NC; ++l) acc += (double)shc[l][c] * Y[l];
                    rgb[c] = acc;
                }
                for (int k = 0; k < K; ++k) {
                    double m0 = p.sg_axes[((int64_t)k * 3 + 0) * n + g];
                    double m1 = p.sg_axes[((int64_t)k * 3 + 1) * n + g];
                    double m2 = p.sg_axes[((int64_t)k * 3 + 2) * n + g];
                    const double mn = sqrt(m0 * m0 + m1 * m1 + m2 * m2);
                    const double lam = exp((double)p.sg_log_sharpness[(int64_t)k * n + g]);
                    const double e = exp(lam * ((d0 * m0 + d1 * m1 + d2 * m2) / mn - 1.0));
                    for (int c = 0; c < 3; ++c)
                        rgb[c] += (double)p.sg_amplitudes[((int64_t)k * 3 + c) * n + g] * e;
                }
                vis = finite_d(rgb[0]) && finite_d(rgb[1]) && finite_d(rgb[2]);
            }
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
                const double lam2 = geo.det / geo.lam1;
                double e0, e1;
                if (A >= C) {
                    e0 = geo.lam1 - C;
                    e1 = B;
                } else {
                    e0 = B;
                    e1 = geo.lam1 - A;
                }
                double en = sqrt(e0 * e0 + e1 * e1);
                if (!(en > 0.0)) {
                    e0 = 1.0;
                    e1 = 0.0;
                    en = 1.0;
                }
                e0 /= en;
                e1 /= en;
                const double k1 = sqrt(kHalfLog2e / geo.lam1);
                const double k2 = sqrt(kHalfLog2e / lam2);
                Rec rec;
                rec.u_hi = (float)geo.u;
                rec.v_hi = (float)geo.v;
                rec.u_lo = (float)(geo.u - (double)rec.u_hi);
                rec.v_lo = (float)(geo.v - (double)rec.v_hi);
                rec.w1x = (float)(e0 * k1);
                rec.w1y = (float)(e1 * k1);
                rec.w2x = (float)(-e1 * k2);
                rec.w2y = (float)(e0 * k2);
                rec.opacity = (float)opacity;
                rec.r = (float)fmax(rgb[0], 0.0);
                rec.g = (float)fmax(rgb[1], 0.0);
                rec.b = (float)fmax(rgb[2], 0.0);
                rec.z = zf;
                rec.rect_x = (uint32_t)geo.px0 | ((uint32_t)geo.px1 << 16);
                rec.rect_y = (uint32_t)geo.py0 | ((uint32_t)geo.py1 << 16);
                rec.radius = geo.radius;
                float4* dst = reinterpret_cast<float4*>(ws.records + item);
                const float4* src = reinterpret_cast<const float4*>(&rec);
                dst[0] = src[0];
                dst[1] = src[1];
                dst[2] = src[2];
                dst[3] = src[3];
            }
            ws.depth_keys[item] = key;
            ws.tile_rects[item] = trect;
            atomicAdd(&hist[0][key & 0xFF], 1u);
            atomicAdd(&hist[1][(key >> 8) & 0xFF], 1u);
            atomicAdd(&hist[2][(key >> 16) & 0xFF], 1u);
            atomicAdd(&hist[3][key >> 24], 1u);
        }
    }
    __syncthreads();
    uint32_t* row = ws.hist_partial + (int64_t)blockIdx.x * kDepthPasses * kRadix;
    for (int i = threadIdx.x; i < kDepthPasses * kRadix; i += blockDim.x) row[i] = (&hist[0][0])[i];
}

void launch_preprocess(const Params& p, const sgs_camera* dev_cams, int n_cams, const Opts& o,
                       const Workspace& ws, int hist_blocks, hipStream_t s) {
    dim3 grid(hist_blocks), block(kPreThreads);
    switch (p.sh_degree) {
        case 0: hipLaunchKernelGGL(k_preprocess<0>, grid, block, 0, s, p, dev_cams, n_cams, o, ws); break;
        case 1: hipLaunchKernelGGL(k_preprocess<1>, grid, block, 0, s, p, dev_cams, n_cams, o, ws); break;
        case 2: hipLaunchKernelGGL(k_preprocess<2>, grid, block, 0, s, p, dev_cams, n_cams, o, ws); break;
        default: hipLaunchKernelGGL(k_preprocess<3>, grid, block, 0, s, p, dev_cams, n_cams, o, ws); break;
    }
}

}  // namespace sgs
