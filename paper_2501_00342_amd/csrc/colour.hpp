// Colour of eq. 9 in float32 and its derivative, shared by the forward
// preprocess and the colour backward: rgb = 0.5 + SH(d) + sum_k a_k
// exp(lambda_k (d.mu_k - 1)) with lambda = exp(log-sharpness) and mu the
// normalised lobe axis (eqs. 4, 5, 9).
#pragma once

#include <type_traits>

#include "common.hpp"
#include "sh_basis.hpp"

namespace sgs {

__device__ __forceinline__ float fast_exp(float x) { return __builtin_amdgcn_exp2f(x * 1.44269504088896341f); }

// Unit lobe axes of the orthogonal modes.  FRAME: the columns of the
// rotation of the unit quaternion (1, w) / |(1, w)| built from the three
// frame parameters w (so the three axes are orthonormal by construction,
// eq. 8); *iq receives 1 / |(1, w)|.
__device__ __forceinline__ void frame_rotation(float w0, float w1, float w2, float r[3][3],
                                               float* iq) {
    const float n2 = 1.0f + w0 * w0 + w1 * w1 + w2 * w2;
    const float i = rsqrtf(n2);
    const float w = i, x = w0 * i, y = w1 * i, z = w2 * i;
    r[0][0] = 1.0f - 2.0f * (y * y + z * z);
    r[0][1] = 2.0f * (x * y - w * z);
    r[0][2] = 2.0f * (x * z + w * y);
    r[1][0] = 2.0f * (x * y + w * z);
    r[1][1] = 1.0f - 2.0f * (x * x + z * z);
    r[1][2] = 2.0f * (y * z - w * x);
    r[2][0] = 2.0f * (x * z - w * y);
    r[2][1] = 2.0f * (y * z + w * x);
    r[2][2] = 1.0f - 2.0f * (x * x + y * y);
    *iq = i;
}

// Number of axis 3-vectors per Gaussian in sg_axes for a lobe mode.
template <int LM, int KMAX>
struct AxisRows {
    static constexpr int value = LM == kLobesFree ? KMAX : (LM == kLobesFrame ? 1 : 0);
};

// SH coefficients used at projected radius r: (deg + 1)^2 with deg = 0 where
// r <= t0, at most 1 where r <= t1, else the stored degree (both thresholds
// 0: the stored degree everywhere).
template <int DEG>
__device__ __forceinline__ int sh_used(const Params& p, int radius) {
    constexpr int NC = (DEG + 1) * (DEG + 1);
    if ((p.sh_ad0 | p.sh_ad1) == 0) return NC;
    if (radius <= p.sh_ad0) return 1;
    if (radius <= p.sh_ad1) return DEG >= 1 ? 4 : 1;
    return NC;
}

// colour of eq. 9 in float32: 0.5 + SH(d) + sum_k a_k exp(lambda_k (d.mu_k - 1)),
// reading the parameters through accessors: sh(l, c), axis(k, j) (lobe k's
// free axis, or the frame parameters as axis(0, j)), lsh(k)
// (log-sharpness) and amp(k, c).  Only the first `ncu` SH coefficients are
// used (adaptive degree).  Returns false when a colour parameter is
// non-finite or a free lobe axis has zero length (the Gaussian is culled).
// KMAX >= n_lobes bounds the unrolled lobe loop; LM is the lobe mode.
template <int DEG, int KMAX, int LM, typename SH, typename AX, typename LS, typename AM>
__device__ __forceinline__ bool colour_eval(SH sh, AX axis, LS lsh, AM amp, int n_lobes, int ncu,
                                            float d0, float d1, float d2, float rgb[3]) {
    constexpr int NC = (DEG + 1) * (DEG + 1);
    bool ok = true;
    float Y[NC];
    sh_eval<DEG, float>(d0, d1, d2, Y);
    rgb[0] = rgb[1] = rgb[2] = 0.5f;
#pragma unroll
    for (int l = 0; l < NC; ++l) {
        const float y = l < ncu ? Y[l] : 0.0f;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float f = sh(l, c);
            ok = ok && isfinite(f);
            rgb[c] = fmaf(f, y, rgb[c]);
        }
    }
    float fr[3][3];
    if constexpr (LM == kLobesFrame) {
        const float w0 = axis(0, 0), w1 = axis(0, 1), w2 = axis(0, 2);
        ok = ok && isfinite(w0) && isfinite(w1) && isfinite(w2);
        float iq;
        frame_rotation(w0, w1, w2, fr, &iq);
    }
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
        if (k >= n_lobes) break;
        const float ls = lsh(k);
        const float a0 = amp(k, 0), a1 = amp(k, 1), a2 = amp(k, 2);
        ok = ok && isfinite(ls) && isfinite(a0) && isfinite(a1) && isfinite(a2);
        float t;
        if constexpr (LM == kLobesFree) {
            const float m0 = axis(k, 0), m1 = axis(k, 1), m2 = axis(k, 2);
            ok = ok && isfinite(m0) && isfinite(m1) && isfinite(m2);
            const float mn2 = m0 * m0 + m1 * m1 + m2 * m2;
            ok = ok && mn2 > 0.0f;
            t = (d0 * m0 + d1 * m1 + d2 * m2) * rsqrtf(mn2) - 1.0f;
        } else if constexpr (LM == kLobesWorld) {
            t = (k == 0 ? d0 : (k == 1 ? d1 : d2)) - 1.0f;
        } else {
            t = (d0 * fr[0][k] + d1 * fr[1][k] + d2 * fr[2][k]) - 1.0f;
        }
        const float e = t == 0.0f ? 1.0f : fast_exp(fast_exp(ls) * t);
        rgb[0] = fmaf(a0, e, rgb[0]);
        rgb[1] = fmaf(a1, e, rgb[1]);
        rgb[2] = fmaf(a2, e, rgb[2]);
    }
    return ok;
}

// Colour record of a Gaussian: its colour coefficients in the order SH
// coefficient (l, c) at 3 l + c, then the axis rows (A 3-vectors: one per
// free lobe, the three frame parameters, or none on the world axes) at
// 3 NC + 3 a + j, the log-sharpness at 3 NC + 3 A + k and the amplitudes
// at 3 NC + 3 A + K + 3 k + c: 3 NC + 3 A + 4 K floats (p.rec_floats, which
// rounds that up to whole 16-byte pieces when the four arrays interleave in
// one buffer whose stride leaves room).  The global arrays are
// Gaussian-major (block g of each at g times its stride p.cs_*), so a
// record is the concatenation of one contiguous block from each array (one
// run of memory when they interleave).
//
// Element types of the colour arrays (template parameter CT): float32,
// bfloat16 or float16 storage; the arithmetic is float32 either way (the
// conversions to float32 are exact).
enum ColourType : int { kColourF32 = 0, kColourBF16 = 1, kColourF16 = 2 };

template <int CT>
struct ColourElem {
    static constexpr int bytes = CT == kColourF32 ? 4 : 2;
};

// element i of a colour record in LDS, as float32
template <int CT>
__device__ __forceinline__ float colour_at(const void* r, int i) {
    if constexpr (CT == kColourF32) {
        return static_cast<const float*>(r)[i];
    } else if constexpr (CT == kColourBF16) {
        return __uint_as_float((uint32_t)static_cast<const uint16_t*>(r)[i] << 16);
    } else {
        return (float)static_cast<const _Float16*>(r)[i];
    }
}

// Cooperative gather of colour records into LDS for the lanes of this wave
// that set `fetch`: the j-th of them (in lane order) gets record slot
// slot0 + j of `rec` (records of p.rec_floats elements of the colour type,
// back to back) and learns its slot in *slot.  Consecutive lanes of each
// direct global->LDS load fetch consecutive 16-byte pieces (single-element
// pieces when a block is not a whole number of 16-byte pieces; 2-byte
// elements are then loaded to registers and stored) of the same
// Gaussian's blocks, so one instruction covers several Gaussians'
// contiguous blocks rather than one element of each of 64 Gaussians.
// s_g: 64 entries of the wave's LDS.  Returns how many lanes fetched
// (wave-uniform); the caller waits (s_waitcnt) before reading the records.
template <int NC3, int CT>
__device__ __forceinline__ int gather_colour(const Params& p, int64_t g, bool fetch, int slot0,
                                             void* rec, int64_t* s_g, int* slot) {
    // storage element: float32, or the 16 bits of a bfloat16 / float16
    using T = typename std::conditional<CT == kColourF32, float, uint16_t>::type;
    constexpr int E = (int)sizeof(T);           // bytes per element
    constexpr int W16 = 16 / E;                 // elements per 16-byte piece
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
    const int K = p.n_lobes, A = p.n_axes;
    const int RSF = p.rec_floats;
    T* base = static_cast<T*>(rec) + slot0 * RSF;
    const T* sh = reinterpret_cast<const T*>(p.sh);
    const T* ax = reinterpret_cast<const T*>(p.sg_axes);
    const T* ls = reinterpret_cast<const T*>(p.sg_log_sharpness);
    const T* am = reinterpret_cast<const T*>(p.sg_amplitudes);
    bool v16;
    int q_sh, q_ax, q_ls, Q;
    if (p.contig) {
        // one run of RSF elements per Gaussian
        v16 = (RSF % W16 == 0) && (p.cs_sh % W16 == 0) && (((uintptr_t)sh) & 15u) == 0;
        q_sh = RSF / (v16 ? W16 : 1);
        q_ax = q_ls = 0;
        Q = q_sh;
    } else {
        v16 = (NC3 % W16 == 0) && ((3 * A) % W16 == 0) && (K % W16 == 0) &&
              ((p.cs_sh | p.cs_ax | p.cs_ls | p.cs_am) & (W16 - 1)) == 0 &&
              (((uintptr_t)sh | (uintptr_t)ax | (uintptr_t)ls | (uintptr_t)am) & 15u) == 0;
        const int w = v16 ? W16 : 1;
        q_sh = NC3 / w;
        q_ax = 3 * A / w;
        q_ls = K / w;
        Q = q_sh + q_ax + q_ls + 3 * K / w;   // pieces per record
    }
    const int wdt = v16 ? W16 : 1;   // elements per piece
    const float invQ = 1.0f / (float)Q;
    const int total = m * Q;
    for (int P0 = 0; P0 < total; P0 += 64) {
        const int P = P0 + lane;
        const bool on = P < total;
        // P / Q through the reciprocal: (P + 0.5) / Q is at least 0.5 / Q
        // from an integer, far above its rounding error (P < 64 Q)
        const int j = on ? (int)(((float)P + 0.5f) * invQ) : 0;
        const int q = P - j * Q;
        const int64_t gj = s_g[j];
        const T* src;
        if (q < q_sh) src = sh + gj * p.cs_sh + q * wdt;
        else if (q < q_sh + q_ax) src = ax + gj * p.cs_ax + (q - q_sh) * wdt;
        else if (q < q_sh + q_ax + q_ls) src = ls + gj * p.cs_ls + (q - q_sh - q_ax) * wdt;
        else src = am + gj * p.cs_am + (q - q_sh - q_ax - q_ls) * wdt;
        if (on) {
            if (v16)
                __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)src,
                                                 (__attribute__((address_space(3))) void*)(base + P0 * W16),
                                                 16, 0, 0);
            else if constexpr (E == 4)
                __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)src,
                                                 (__attribute__((address_space(3))) void*)(base + P0),
                                                 4, 0, 0);
            else
                // direct loads of 1 or 2 bytes still place lane i at 4 i in
                // LDS: 2-byte elements go through a register instead
                base[P0 + lane] = *src;
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
// accessors as colour_eval.  gax: per free lobe, its axis gradient; in the
// frame mode gax[0] receives the gradient of the three frame parameters;
// untouched on the world axes.
template <int DEG, int KMAX, int LM, typename SH, typename AX, typename LS, typename AM>
__device__ __forceinline__ void colour_bwd_eval(SH sh, AX axis, LS lsh, AM amp, int n_lobes,
                                                int ncu, float d0, float d1, float d2,
                                                const float grgb[3], float gsh[][3],
                                                float gamp[][3], float gax[][3], float glsh[],
                                                float gd[3]) {
    constexpr int NC = (DEG + 1) * (DEG + 1);
    float raw[3];
    colour_eval<DEG, KMAX, LM>(sh, axis, lsh, amp, n_lobes, ncu, d0, d1, d2, raw);
    // max(0, .): derivative 1 where the raw colour is >= 0
    const float gc[3] = {raw[0] >= 0.0f ? grgb[0] : 0.0f, raw[1] >= 0.0f ? grgb[1] : 0.0f,
                         raw[2] >= 0.0f ? grgb[2] : 0.0f};
    float Y[NC], gx[NC], gy[NC], gz[NC];
    sh_eval<DEG, float>(d0, d1, d2, Y);
    sh_grad<DEG, float>(d0, d1, d2, gx, gy, gz);
    gd[0] = gd[1] = gd[2] = 0.0f;
#pragma unroll
    for (int l = 0; l < NC; ++l) {
        // unused coefficients (adaptive degree): zero gradient, no direction
        // term; a select rather than an exit keeps the loop fully unrolled
        // and gsh in registers
        const float y = l < ncu ? Y[l] : 0.0f;
        float cl = 0.0f;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            gsh[l][c] = fmaf(gc[c], y, gsh[l][c]);
            cl = fmaf(gc[c], sh(l, c), cl);
        }
        cl = l < ncu ? cl : 0.0f;
        gd[0] = fmaf(cl, gx[l], gd[0]);
        gd[1] = fmaf(cl, gy[l], gd[1]);
        gd[2] = fmaf(cl, gz[l], gd[2]);
    }
    float fr[3][3], iq = 1.0f;
    float gfr[3][3] = {{0.0f, 0.0f, 0.0f}, {0.0f, 0.0f, 0.0f}, {0.0f, 0.0f, 0.0f}};
    if constexpr (LM == kLobesFrame) frame_rotation(axis(0, 0), axis(0, 1), axis(0, 2), fr, &iq);
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
        if (k >= n_lobes) break;
        float mu0, mu1, mu2, t, imn = 1.0f;
        if constexpr (LM == kLobesFree) {
            const float m0 = axis(k, 0), m1 = axis(k, 1), m2 = axis(k, 2);
            imn = rsqrtf(m0 * m0 + m1 * m1 + m2 * m2);
            mu0 = m0 * imn;
            mu1 = m1 * imn;
            mu2 = m2 * imn;
            t = (d0 * m0 + d1 * m1 + d2 * m2) * imn - 1.0f;
        } else if constexpr (LM == kLobesWorld) {
            mu0 = k == 0 ? 1.0f : 0.0f;
            mu1 = k == 1 ? 1.0f : 0.0f;
            mu2 = k == 2 ? 1.0f : 0.0f;
            t = (k == 0 ? d0 : (k == 1 ? d1 : d2)) - 1.0f;
        } else {
            mu0 = fr[0][k];
            mu1 = fr[1][k];
            mu2 = fr[2][k];
            t = (d0 * mu0 + d1 * mu1 + d2 * mu2) - 1.0f;
        }
        const float lam = fast_exp(lsh(k));
        const float e = t == 0.0f ? 1.0f : fast_exp(lam * t);
        float sk = 0.0f;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            gamp[k][c] = fmaf(gc[c], e, gamp[k][c]);
            sk = fmaf(gc[c], amp(k, c), sk);
        }
        sk *= e;
        glsh[k] = fmaf(sk * t, lam, glsh[k]);
        // d/dmu_hat = sk lam d
        const float sl = sk * lam;
        if constexpr (LM == kLobesFree) {
            // then (I - mu mu^T) / |m|
            const float dot = sl * (mu0 * d0 + mu1 * d1 + mu2 * d2);
            gax[k][0] += (sl * d0 - mu0 * dot) * imn;
            gax[k][1] += (sl * d1 - mu1 * dot) * imn;
            gax[k][2] += (sl * d2 - mu2 * dot) * imn;
        } else if constexpr (LM == kLobesFrame) {
            // mu_k is column k of the frame rotation
            gfr[0][k] += sl * d0;
            gfr[1][k] += sl * d1;
            gfr[2][k] += sl * d2;
        }
        gd[0] = fmaf(sl, mu0, gd[0]);
        gd[1] = fmaf(sl, mu1, gd[1]);
        gd[2] = fmaf(sl, mu2, gd[2]);
    }
    if constexpr (LM == kLobesFrame) {
        // rotation entries -> unit quaternion (w, x, y, z) -> q = (1, w0, w1, w2)
        // through the normalisation (I - q_hat q_hat^T) / |q|; keep x, y, z
        const float w = iq, x = axis(0, 0) * iq, y = axis(0, 1) * iq, z = axis(0, 2) * iq;
        const float (*g)[3] = gfr;
        const float gw = 2.0f * (-z * g[0][1] + y * g[0][2] + z * g[1][0] - x * g[1][2] -
                                 y * g[2][0] + x * g[2][1]);
        const float gx_ = 2.0f * (y * g[0][1] + z * g[0][2] + y * g[1][0] - 2.0f * x * g[1][1] -
                                  w * g[1][2] + z * g[2][0] + w * g[2][1] - 2.0f * x * g[2][2]);
        const float gy_ = 2.0f * (-2.0f * y * g[0][0] + x * g[0][1] + w * g[0][2] + x * g[1][0] +
                                  z * g[1][2] - w * g[2][0] + z * g[2][1] - 2.0f * y * g[2][2]);
        const float gz_ = 2.0f * (-2.0f * z * g[0][0] - w * g[0][1] + x * g[0][2] + w * g[1][0] -
                                  2.0f * z * g[1][1] + y * g[1][2] + x * g[2][0] + y * g[2][1]);
        const float dq = w * gw + x * gx_ + y * gy_ + z * gz_;
        gax[0][0] += (gx_ - x * dq) * iq;
        gax[0][1] += (gy_ - y * dq) * iq;
        gax[0][2] += (gz_ - z * dq) * iq;
    }
}

}  // namespace sgs
