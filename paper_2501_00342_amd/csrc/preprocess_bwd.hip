// Backward preprocess: one thread per Gaussian, summing over cameras.
//
// Input: the 2D gradients of each (camera, Gaussian) item w.r.t. the
// projected mean (u, v), the conic Q = Sigma'^-1 (Qa, Qb, Qc), the opacity
// and the clamped colour.  Output: gradients of every raw parameter,
// written once (no atomics).  The chain rule runs through
//   conic -> Sigma' (dQ = -Q dSigma' Q),
//   Sigma' = M M^T + dilation I, M = J W R S   (eq. 3 and the EWA step),
//   J and (u, v) -> camera-space mean (no derivative through the guard
//   clamp where it is active),
//   colour eq. 9 -> SH coefficients (eq. 4), SG amplitude, sharpness and
//   axis (eq. 5), and the view direction -> mean,
//   activations exp / sigmoid and the normalisations of q and mu.
// Float64 arithmetic: the kernel is bound by memory traffic.
#include "common.hpp"
#include "sh_basis.hpp"

namespace sgs {

template <int DEG>
__global__ void __launch_bounds__(kPreThreads)
k_preprocess_bwd(Params p, const sgs_camera* __restrict__ cams, int n_cams, Opts o, Workspace ws,
                 sgs_grads gr) {
    constexpr int NC = (DEG + 1) * (DEG + 1);
    const int64_t n = p.n;
    const int K = p.n_lobes;
    const int64_t M = ws.n_items;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n;
         g += (int64_t)gridDim.x * blockDim.x) {
        double X[3], ls[3], q[4];
        for (int c = 0; c < 3; ++c) {
            X[c] = p.means[c * n + g];
            ls[c] = p.log_scales[c * n + g];
        }
        for (int c = 0; c < 4; ++c) q[c] = p.quats[c * n + g];
        const double logit = p.opacity_logits[g];
        const double sig = 1.0 / (1.0 + exp(-logit));
        const double s[3] = {exp(ls[0]), exp(ls[1]), exp(ls[2])};
        const double qn = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
        const double w = q[0] / qn, x = q[1] / qn, y = q[2] / qn, z = q[3] / qn;
        const double Rq[3][3] = {
            {1.0 - 2.0 * (y * y + z * z), 2.0 * (x * y - w * z), 2.0 * (x * z + w * y)},
            {2.0 * (x * y + w * z), 1.0 - 2.0 * (x * x + z * z), 2.0 * (y * z - w * x)},
            {2.0 * (x * z - w * y), 2.0 * (y * z + w * x), 1.0 - 2.0 * (x * x + y * y)}};
        double M3[3][3];
        for (int i = 0; i < 3; ++i)
            for (int a = 0; a < 3; ++a) M3[i][a] = Rq[i][a] * s[a];

        // accumulators (sum over cameras)
        double gX[3] = {0, 0, 0}, gls[3] = {0, 0, 0}, gq[4] = {0, 0, 0, 0}, glogit = 0.0;
        float gsh[NC][3];
        for (int l = 0; l < NC; ++l) gsh[l][0] = gsh[l][1] = gsh[l][2] = 0.0f;
        float gamp[SGS_MAX_LOBES][3], gax[SGS_MAX_LOBES][3], glsh[SGS_MAX_LOBES];
#pragma unroll
        for (int k = 0; k < SGS_MAX_LOBES; ++k) {
            glsh[k] = 0.0f;
            for (int c = 0; c < 3; ++c) gamp[k][c] = gax[k][c] = 0.0f;
        }

        for (int ci = 0; ci < n_cams; ++ci) {
            const int64_t item = (int64_t)ci * n + g;
            const uint64_t tr = ws.tile_rects[item];
            if ((int)((tr >> 16) & 0xFFFF) < (int)(tr & 0xFFFF)) continue;   // culled
            const sgs_camera& cam = cams[ci];
            const double g2[9] = {ws.grad2d[0 * M + item], ws.grad2d[1 * M + item],
                                  ws.grad2d[2 * M + item], ws.grad2d[3 * M + item],
                                  ws.grad2d[4 * M + item], ws.grad2d[5 * M + item],
                                  ws.grad2d[6 * M + item], ws.grad2d[7 * M + item],
                                  ws.grad2d[8 * M + item]};
            double Rc[3][3];
            for (int i = 0; i < 3; ++i)
                for (int k = 0; k < 3; ++k) Rc[i][k] = cam.R[3 * i + k];
            const double fx = cam.fx, fy = cam.fy;
            double xc[3];
            for (int i = 0; i < 3; ++i)
                xc[i] = Rc[i][0] * X[0] + Rc[i][1] * X[1] + Rc[i][2] * X[2] + (double)cam.t[i];

            // ---- opacity
            glogit += g2[5] * sig * (1.0 - sig);

            // ---- colour
            double cc[3];
            for (int j = 0; j < 3; ++j)
                cc[j] = -(Rc[0][j] * cam.t[0] + Rc[1][j] * cam.t[1] + Rc[2][j] * cam.t[2]);
            double dv[3] = {X[0] - cc[0], X[1] - cc[1], X[2] - cc[2]};
            const double dist = sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
            const double d[3] = {dv[0] / dist, dv[1] / dist, dv[2] / dist};
            double Y[NC];
            sh_eval<DEG, double>(d[0], d[1], d[2], Y);
            double raw[3];
            for (int c = 0; c < 3; ++c) {
                double acc = 0.5;
                for (int l = 0; l < NC; ++l) acc += (double)p.sh[((int64_t)l * 3 + c) * n + g] * Y[l];
                raw[c] = acc;
            }
            double lam[SGS_MAX_LOBES], ek[SGS_MAX_LOBES], cosk[SGS_MAX_LOBES], mlen[SGS_MAX_LOBES];
#pragma unroll
            for (int k = 0; k < SGS_MAX_LOBES; ++k) {
                if (k >= K) break;
                const double m0 = p.sg_axes[((int64_t)k * 3 + 0) * n + g];
                const double m1 = p.sg_axes[((int64_t)k * 3 + 1) * n + g];
                const double m2 = p.sg_axes[((int64_t)k * 3 + 2) * n + g];
                mlen[k] = sqrt(m0 * m0 + m1 * m1 + m2 * m2);
                lam[k] = exp((double)p.sg_log_sharpness[(int64_t)k * n + g]);
                cosk[k] = (d[0] * m0 + d[1] * m1 + d[2] * m2) / mlen[k];
                ek[k] = cosk[k] - 1.0 == 0.0 ? 1.0 : exp(lam[k] * (cosk[k] - 1.0));
                for (int c = 0; c < 3; ++c)
                    raw[c] += (double)p.sg_amplitudes[((int64_t)k * 3 + c) * n + g] * ek[k];
            }
            const double grgb[3] = {raw[0] >= 0.0 ? g2[6] : 0.0, raw[1] >= 0.0 ? g2[7] : 0.0,
                                    raw[2] >= 0.0 ? g2[8] : 0.0};
            for (int l = 0; l < NC; ++l)
                for (int c = 0; c < 3; ++c) gsh[l][c] += (float)(grgb[c] * Y[l]);
            double gd[3] = {0, 0, 0};
            {
                double gx[NC], gy[NC], gz[NC];
                sh_grad<DEG>(d[0], d[1], d[2], gx, gy, gz);
                for (int l = 0; l < NC; ++l) {
                    double cl = 0.0;
                    for (int c = 0; c < 3; ++c) cl += grgb[c] * (double)p.sh[((int64_t)l * 3 + c) * n + g];
                    gd[0] += cl * gx[l];
                    gd[1] += cl * gy[l];
                    gd[2] += cl * gz[l];
                }
            }
#pragma unroll
            for (int k = 0; k < SGS_MAX_LOBES; ++k) {
                if (k >= K) break;
                double sk = 0.0;
                for (int c = 0; c < 3; ++c) {
                    const int64_t ia = ((int64_t)k * 3 + c) * n + g;
                    gamp[k][c] += (float)(grgb[c] * ek[k]);
                    sk += grgb[c] * (double)p.sg_amplitudes[ia];
                }
                sk *= ek[k];
                glsh[k] += (float)(sk * (cosk[k] - 1.0) * lam[k]);
                const double mu[3] = {p.sg_axes[((int64_t)k * 3 + 0) * n + g] / mlen[k],
                                      p.sg_axes[((int64_t)k * 3 + 1) * n + g] / mlen[k],
                                      p.sg_axes[((int64_t)k * 3 + 2) * n + g] / mlen[k]};
                const double gm[3] = {sk * lam[k] * d[0], sk * lam[k] * d[1], sk * lam[k] * d[2]};
                const double dot = mu[0] * gm[0] + mu[1] * gm[1] + mu[2] * gm[2];
                for (int c = 0; c < 3; ++c) {
                    gax[k][c] += (float)((gm[c] - mu[c] * dot) / mlen[k]);
                    gd[c] += sk * lam[k] * mu[c];
                }
            }
            {
                const double dd = d[0] * gd[0] + d[1] * gd[1] + d[2] * gd[2];
                for (int c = 0; c < 3; ++c) gX[c] += (gd[c] - d[c] * dd) / dist;
            }

            // ---- geometry: recompute the forward chain
            const double zc = xc[2];
            const double xn = xc[0] / zc, yn = xc[1] / zc;
            const double limx = (double)o.guard * ((0.5 * cam.width) / fx);
            const double limy = (double)o.guard * ((0.5 * cam.height) / fy);
            const bool clx = xn < -limx || xn > limx;
            const bool cly = yn < -limy || yn > limy;
            const double xnc = fmin(fmax(xn, -limx), limx);
            const double ync = fmin(fmax(yn, -limy), limy);
            const double J[2][3] = {{fx / zc, 0.0, -(fx * xnc) / zc}, {0.0, fy / zc, -(fy * ync) / zc}};
            double T2[2][3], Mm[2][3];
            for (int i = 0; i < 2; ++i)
                for (int k = 0; k < 3; ++k)
                    T2[i][k] = J[i][0] * Rc[0][k] + J[i][1] * Rc[1][k] + J[i][2] * Rc[2][k];
            for (int i = 0; i < 2; ++i)
                for (int a = 0; a < 3; ++a)
                    Mm[i][a] = T2[i][0] * M3[0][a] + T2[i][1] * M3[1][a] + T2[i][2] * M3[2][a];
            const double dil = o.dilation;
            const double pp = Mm[0][0] * Mm[0][0] + Mm[0][1] * Mm[0][1] + Mm[0][2] * Mm[0][2];
            const double qq = Mm[1][0] * Mm[1][0] + Mm[1][1] * Mm[1][1] + Mm[1][2] * Mm[1][2];
            const double A = pp + dil, C = qq + dil;
            const double B = Mm[0][0] * Mm[1][0] + Mm[0][1] * Mm[1][1] + Mm[0][2] * Mm[1][2];
            const double crx = Mm[0][1] * Mm[1][2] - Mm[0][2] * Mm[1][1];
            const double cry = Mm[0][2] * Mm[1][0] - Mm[0][0] * Mm[1][2];
            const double crz = Mm[0][0] * Mm[1][1] - Mm[0][1] * Mm[1][0];
            const double det = crx * crx + cry * cry + crz * crz + dil * (pp + qq) + dil * dil;
            // conic -> Sigma'
            const double gQa = g2[2], gQb = g2[3], gQc = g2[4];
            const double d2 = det * det;
            const double gA = (-C * C * gQa + B * C * gQb - B * B * gQc) / d2;
            const double gC = (-B * B * gQa + A * B * gQb - A * A * gQc) / d2;
            const double gB = (2.0 * B * C * gQa - (A * C + B * B) * gQb + 2.0 * A * B * gQc) / d2;
            // Sigma' = M M^T + dil I
            double gM[2][3];
            for (int a = 0; a < 3; ++a) {
                gM[0][a] = 2.0 * gA * Mm[0][a] + gB * Mm[1][a];
                gM[1][a] = gB * Mm[0][a] + 2.0 * gC * Mm[1][a];
            }
            // M = T2 M3
            double gT2[2][3], gM3[3][3];
            for (int i = 0; i < 2; ++i)
                for (int k = 0; k < 3; ++k)
                    gT2[i][k] = gM[i][0] * M3[k][0] + gM[i][1] * M3[k][1] + gM[i][2] * M3[k][2];
            for (int k = 0; k < 3; ++k)
                for (int a = 0; a < 3; ++a) gM3[k][a] = T2[0][k] * gM[0][a] + T2[1][k] * gM[1][a];
            // M3 = Rq diag(s)
            double gR[3][3];
            for (int i = 0; i < 3; ++i)
                for (int a = 0; a < 3; ++a) gR[i][a] = gM3[i][a] * s[a];
            for (int a = 0; a < 3; ++a)
                gls[a] += (gM3[0][a] * Rq[0][a] + gM3[1][a] * Rq[1][a] + gM3[2][a] * Rq[2][a]) * s[a];
            const double gw = 2.0 * (-z * gR[0][1] + y * gR[0][2] + z * gR[1][0] - x * gR[1][2] -
                                     y * gR[2][0] + x * gR[2][1]);
            const double gxq = 2.0 * (y * gR[0][1] + z * gR[0][2] + y * gR[1][0] - 2.0 * x * gR[1][1] -
                                      w * gR[1][2] + z * gR[2][0] + w * gR[2][1] - 2.0 * x * gR[2][2]);
            const double gyq = 2.0 * (-2.0 * y * gR[0][0] + x * gR[0][1] + w * gR[0][2] + x * gR[1][0] +
                                      z * gR[1][2] - w * gR[2][0] + z * gR[2][1] - 2.0 * y * gR[2][2]);
            const double gzq = 2.0 * (-2.0 * z * gR[0][0] - w * gR[0][1] + x * gR[0][2] + w * gR[1][0] -
                                      2.0 * z * gR[1][1] + y * gR[1][2] + x * gR[2][0] + y * gR[2][1]);
            gq[0] += gw;
            gq[1] += gxq;
            gq[2] += gyq;
            gq[3] += gzq;
            // T2 = J W -> J
            double gJ[2][3];
            for (int i = 0; i < 2; ++i)
                for (int m = 0; m < 3; ++m)
                    gJ[i][m] = gT2[i][0] * Rc[m][0] + gT2[i][1] * Rc[m][1] + gT2[i][2] * Rc[m][2];
            // J, (u, v) -> camera-space mean
            const double z2 = zc * zc;
            double gxc[3] = {0.0, 0.0, 0.0};
            gxc[2] += gJ[0][0] * (-fx / z2) + gJ[1][1] * (-fy / z2);
            if (clx) {
                gxc[2] += gJ[0][2] * (fx * xnc / z2);
            } else {
                gxc[0] += gJ[0][2] * (-fx / z2);
                gxc[2] += gJ[0][2] * (2.0 * fx * xc[0] / (z2 * zc));
            }
            if (cly) {
                gxc[2] += gJ[1][2] * (fy * ync / z2);
            } else {
                gxc[1] += gJ[1][2] * (-fy / z2);
                gxc[2] += gJ[1][2] * (2.0 * fy * xc[1] / (z2 * zc));
            }
            const double gu = g2[0], gv = g2[1];
            gxc[0] += gu * fx / zc;
            gxc[1] += gv * fy / zc;
            gxc[2] += -gu * fx * xc[0] / z2 - gv * fy * xc[1] / z2;
            for (int j = 0; j < 3; ++j) gX[j] += Rc[0][j] * gxc[0] + Rc[1][j] * gxc[1] + Rc[2][j] * gxc[2];
        }

        // quaternion normalisation: (I - q q^T) / |q|
        const double qh[4] = {w, x, y, z};
        const double dq = qh[0] * gq[0] + qh[1] * gq[1] + qh[2] * gq[2] + qh[3] * gq[3];
        for (int c = 0; c < 3; ++c) {
            gr.means[c * n + g] = (float)gX[c];
            gr.log_scales[c * n + g] = (float)gls[c];
        }
        for (int c = 0; c < 4; ++c) gr.quats[c * n + g] = (float)((gq[c] - qh[c] * dq) / qn);
        gr.opacity_logits[g] = (float)glogit;
        for (int l = 0; l < NC; ++l)
            for (int c = 0; c < 3; ++c) gr.sh[((int64_t)l * 3 + c) * n + g] = gsh[l][c];
#pragma unroll
        for (int k = 0; k < SGS_MAX_LOBES; ++k) {
            if (k >= K) break;
            for (int c = 0; c < 3; ++c) {
                gr.sg_axes[((int64_t)k * 3 + c) * n + g] = gax[k][c];
                gr.sg_amplitudes[((int64_t)k * 3 + c) * n + g] = gamp[k][c];
            }
            gr.sg_log_sharpness[(int64_t)k * n + g] = glsh[k];
        }
    }
}

void launch_preprocess_bwd(const Params& p, const sgs_camera* dev_cams, int n_cams, const Opts& o,
                           const Workspace& ws, const sgs_grads& gr, hipStream_t s) {
    if (p.n <= 0) return;
    int64_t blocks = (p.n + kPreThreads - 1) / kPreThreads;
    if (blocks > 4096) blocks = 4096;
    dim3 grid((unsigned)blocks), block(kPreThreads);
    switch (p.sh_degree) {
        case 0: hipLaunchKernelGGL(k_preprocess_bwd<0>, grid, block, 0, s, p, dev_cams, n_cams, o, ws, gr); break;
        case 1: hipLaunchKernelGGL(k_preprocess_bwd<1>, grid, block, 0, s, p, dev_cams, n_cams, o, ws, gr); break;
        case 2: hipLaunchKernelGGL(k_preprocess_bwd<2>, grid, block, 0, s, p, dev_cams, n_cams, o, ws, gr); break;
        default: hipLaunchKernelGGL(k_preprocess_bwd<3>, grid, block, 0, s, p, dev_cams, n_cams, o, ws, gr); break;
    }
}

}  // namespace sgs
