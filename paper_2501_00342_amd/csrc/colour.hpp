// Colour of eq. 9 in float32 and its derivative, shared by the forward
// preprocess and the colour backward: rgb = 0.5 + SH(d) + sum_k a_k
// exp(lambda_k (d.mu_k - 1)) with lambda = exp(log-sharpness) and mu the
// normalised lobe axis (eqs. 4, 5, 9).
#pragma once

#include "common.hpp"
#include "sh_basis.hpp"

namespace sgs {

__device__ __forceinline__ float fast_exp(float x) { return __builtin_amdgcn_exp2f(x * 1.44269504088896341f); }

// colour of eq. 9 in float32: 0.5 + SH(d) + sum_k a_k exp(lambda_k (d.mu_k - 1)),
// reading the parameters through accessors: sh(l, c), axis(k, j),
// lsh(k) (log-sharpness) and amp(k, c).  Returns false when a colour
// parameter is non-finite or a lobe axis has zero length (the Gaussian is
// culled).  KMAX >= n_lobes bounds the unrolled lobe loop.
template <int DEG, int KMAX, typename SH, typename AX, typename LS, typename AM>
__device__ __forceinline__ bool colour_eval(SH sh, AX axis, LS lsh, AM amp, int n_lobes, float d0,
                                            float d1, float d2, float rgb[3]) {
    constexpr int NC = (DEG + 1) * (DEG + 1);
    bool ok = true;
    float Y[NC];
    sh_eval<DEG, float>(d0, d1, d2, Y);
    rgb[0] = rgb[1] = rgb[2] = 0.5f;
#pragma unroll
    for (int l = 0; l < NC; ++l)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float f = sh(l, c);
            ok = ok && isfinite(f);
            rgb[c] = fmaf(f, Y[l], rgb[c]);
        }
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
        if (k >= n_lobes) break;
        const float m0 = axis(k, 0), m1 = axis(k, 1), m2 = axis(k, 2);
        const float ls = lsh(k);
        const float a0 = amp(k, 0), a1 = amp(k, 1), a2 = amp(k, 2);
        ok = ok && isfinite(m0) && isfinite(m1) && isfinite(m2) && isfinite(ls) &&
             isfinite(a0) && isfinite(a1) && isfinite(a2);
        const float mn2 = m0 * m0 + m1 * m1 + m2 * m2;
        ok = ok && mn2 > 0.0f;
        const float t = (d0 * m0 + d1 * m1 + d2 * m2) * rsqrtf(mn2) - 1.0f;
        const float e = t == 0.0f ? 1.0f : fast_exp(fast_exp(ls) * t);
        rgb[0] = fmaf(a0, e, rgb[0]);
        rgb[1] = fmaf(a1, e, rgb[1]);
        rgb[2] = fmaf(a2, e, rgb[2]);
    }
    return ok;
}

// Colour record of a Gaussian: its colour coefficients in the row order
// SH coefficient (l, c) at 3 l + c, then per lobe k the axis at
// 3 NC + 3 k + j, the log-sharpness at 3 NC + 3 K + k and the amplitudes at
// 3 NC + 4 K + 3 k + c: 3 NC + 7 K floats.  The global arrays are
// Gaussian-major (block g of each at g times its stride p.cs_*), so a
// record is the concatenation of one contiguous block from each array (one
// run of memory when the four arrays interleave with a common stride).
__device__ __forceinline__ int colour_record_floats(int nc3, int K) { return nc3 + 7 * K; }

// Cooperative gather of colour records into LDS for the lanes of this wave
// that set `fetch`: the j-th of them (in lane order) gets record slot
// slot0 + j of `rec` (records of colour_record_floats() floats, back to back)
// and learns its slot in *slot.  Consecutive lanes of each direct
// global->LDS load fetch consecutive 16-byte pieces (4-byte pieces when a
// block is not a whole number of 16-byte pieces) of the same Gaussian's
// blocks, so one instruction covers several Gaussians' contiguous blocks
// rather than one float of each of 64 Gaussians.  s_g: 64 entries of the
// wave's LDS.  Returns how many lanes fetched (wave-uniform); the caller
// waits (s_waitcnt) before reading the records.
template <int NC3>
__device__ __forceinline__ int gather_colour(const Params& p, int64_t g, bool fetch, int slot0,
                                             float* rec, int64_t* s_g, int* slot) {
    const int lane = threadIdx.x & 63;
    const uint64_t b = __ballot(fetch);
    const int m = __popcll(b);
    if (m == 0) return 0;
    const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    const int rank = __popcll(b & lt);
    if (fetch) {
        s_g[rank] = g;   // read back below by other lanes of this wave (LDS order)
        *slot = slot0 + rank;
    }
    const int K = p.n_lobes;
    const bool v4 = (NC3 % 4 == 0) && (K % 4 == 0) &&
                    ((p.cs_sh | p.cs_ax | p.cs_ls | p.cs_am) & 3) == 0 &&
                    (((uintptr_t)p.sh | (uintptr_t)p.sg_axes | (uintptr_t)p.sg_log_sharpness |
                      (uintptr_t)p.sg_amplitudes) & 15u) == 0;
    const int wdt = v4 ? 4 : 1;   // floats per piece
    const int q_sh = NC3 / wdt, q_ax = 3 * K / wdt, q_ls = K / wdt;
    const int Q = q_sh + 2 * q_ax + q_ls;   // pieces per record
    const float invQ = 1.0f / (float)Q;
    const int total = m * Q;
    float* base = rec + slot0 * colour_record_floats(NC3, K);
    for (int P0 = 0; P0 < total; P0 += 64) {
        const int P = P0 + lane;
        const bool on = P < total;
        // P / Q through the reciprocal: (P + 0.5) / Q is at least 0.5 / Q
        // from an integer, far above its rounding error (P < 64 Q)
        const int j = on ? (int)(((float)P + 0.5f) * invQ) : 0;
        const int q = P - j * Q;
        const int64_t gj = s_g[j];
        const float* src;
        if (q < q_sh) src = p.sh + gj * p.cs_sh + q * wdt;
        else if (q < q_sh + q_ax) src = p.sg_axes + gj * p.cs_ax + (q - q_sh) * wdt;
        else if (q < q_sh + q_ax + q_ls) src = p.sg_log_sharpness + gj * p.cs_ls + (q - q_sh - q_ax) * wdt;
        else src = p.sg_amplitudes + gj * p.cs_am + (q - q_sh - q_ax - q_ls) * wdt;
        if (on) {
            if (v4)
                __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)src,
                                                 (__attribute__((address_space(3))) void*)(base + P0 * 4),
                                                 16, 0, 0);
            else
                __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)src,
                                                 (__attribute__((address_space(3))) void*)(base + P0),
                                                 4, 0, 0);
        }
    }
    return m;
}

// Unit view direction from the camera centre (-R^T t) to the mean X: the
// difference in float64 (no cancellation near the camera), the
// normalisation in float32.  *dist receives |X - centre|.
__device__ __forceinline__ void view_dir(const double X[3], const sgs_camera& cam, float d[3],
                                         float* dist) {
    const double c0 = -(((double)cam.R[0] * cam.t[0] + (double)cam.R[3] * cam.t[1]) + (double)cam.R[6] * cam.t[2]);
    const double c1 = -(((double)cam.R[1] * cam.t[0] + (double)cam.R[4] * cam.t[1]) + (double)cam.R[7] * cam.t[2]);
    const double c2 = -(((double)cam.R[2] * cam.t[0] + (double)cam.R[5] * cam.t[1]) + (double)cam.R[8] * cam.t[2]);
    const float e0 = (float)(X[0] - c0), e1 = (float)(X[1] - c1), e2 = (float)(X[2] - c2);
    const float n2 = e0 * e0 + e1 * e1 + e2 * e2;
    const float inv = rsqrtf(n2);
    d[0] = e0 * inv;
    d[1] = e1 * inv;
    d[2] = e2 * inv;
    *dist = n2 * inv;
}

// Backward of the colour.  grgb: dL/d(clamped rgb).  Adds the parameter
// gradients into the accumulators and returns dL/dd (the view direction,
// before the normalisation Jacobian).  Parameters are read through the same
// accessors as colour_eval.
template <int DEG, int KMAX, typename SH, typename AX, typename LS, typename AM>
__device__ __forceinline__ void colour_bwd_eval(SH sh, AX axis, LS lsh, AM amp, int n_lobes,
                                                float d0, float d1, float d2, const float grgb[3],
                                                float gsh[][3], float gamp[][3], float gax[][3],
                                                float glsh[], float gd[3]) {
    constexpr int NC = (DEG + 1) * (DEG + 1);
    float raw[3];
    colour_eval<DEG, KMAX>(sh, axis, lsh, amp, n_lobes, d0, d1, d2, raw);
    // max(0, .): derivative 1 where the raw colour is >= 0
    const float gc[3] = {raw[0] >= 0.0f ? grgb[0] : 0.0f, raw[1] >= 0.0f ? grgb[1] : 0.0f,
                         raw[2] >= 0.0f ? grgb[2] : 0.0f};
    float Y[NC], gx[NC], gy[NC], gz[NC];
    sh_eval<DEG, float>(d0, d1, d2, Y);
    sh_grad<DEG, float>(d0, d1, d2, gx, gy, gz);
    gd[0] = gd[1] = gd[2] = 0.0f;
#pragma unroll
    for (int l = 0; l < NC; ++l) {
        float cl = 0.0f;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            gsh[l][c] = fmaf(gc[c], Y[l], gsh[l][c]);
            cl = fmaf(gc[c], sh(l, c), cl);
        }
        gd[0] = fmaf(cl, gx[l], gd[0]);
        gd[1] = fmaf(cl, gy[l], gd[1]);
        gd[2] = fmaf(cl, gz[l], gd[2]);
    }
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
        if (k >= n_lobes) break;
        const float m0 = axis(k, 0), m1 = axis(k, 1), m2 = axis(k, 2);
        const float imn = rsqrtf(m0 * m0 + m1 * m1 + m2 * m2);
        const float mu0 = m0 * imn, mu1 = m1 * imn, mu2 = m2 * imn;
        const float lam = fast_exp(lsh(k));
        const float t = (d0 * m0 + d1 * m1 + d2 * m2) * imn - 1.0f;
        const float e = t == 0.0f ? 1.0f : fast_exp(lam * t);
        float sk = 0.0f;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            gamp[k][c] = fmaf(gc[c], e, gamp[k][c]);
            sk = fmaf(gc[c], amp(k, c), sk);
        }
        sk *= e;
        glsh[k] = fmaf(sk * t, lam, glsh[k]);
        // d/dmu_hat = sk lam d, then (I - mu mu^T) / |m|
        const float sl = sk * lam;
        const float dot = sl * (mu0 * d0 + mu1 * d1 + mu2 * d2);
        gax[k][0] += (sl * d0 - mu0 * dot) * imn;
        gax[k][1] += (sl * d1 - mu1 * dot) * imn;
        gax[k][2] += (sl * d2 - mu2 * dot) * imn;
        gd[0] = fmaf(sl, mu0, gd[0]);
        gd[1] = fmaf(sl, mu1, gd[1]);
        gd[2] = fmaf(sl, mu2, gd[2]);
    }
}

}  // namespace sgs
