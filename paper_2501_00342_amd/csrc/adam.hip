// Fused Adam update of every Gaussian parameter array in one launch, with
// the staged introduction of the SG lobes (Experiments, Implementation: the
// lobes join training after the first 2,000 iterations, with learning rate
// 0.0025; the other learning rates are the 3D-GS ones).
//
// Adam (Kingma and Ba), per element, in float32:
//   m = b1 m + (1 - b1) g,   v = b2 v + (1 - b2) g^2,
//   p -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
// The lobe arrays (axes or frame parameters, log-sharpness, amplitudes) are
// left untouched, moments included, before iteration sg_start; from there
// their step count t starts at 1.
//
// Memory: pure streaming (4 floats read, 3 written per element).  Geometry
// rows and packed colour arrays are flat runs read and written with 16-byte
// accesses; a colour array inside an interleaved record (colour_stride) is
// addressed per Gaussian on the parameter side only (gradients and moments
// are always packed).
#include "common.hpp"

namespace sgs {

__global__ void __launch_bounds__(256)
k_adam(AdamArrays a) {
    const int k = blockIdx.y;
    if (!a.on[k]) return;
    const int64_t count = a.count[k];
    float* __restrict__ p = a.p[k];
    const float* __restrict__ g = a.g[k];
    float* __restrict__ m = a.m[k];
    float* __restrict__ v = a.v[k];
    const float lr = a.lr[k], c1 = a.c1[k], c2 = a.c2[k];
    const float b1 = a.b1, b2 = a.b2, ob1 = a.ob1, ob2 = a.ob2, eps = a.eps;
    const int64_t w = a.width[k], ps = a.pstride[k];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    auto step = [&](float& pp, float gg, float& mm, float& vv) {
        mm = b1 * mm + ob1 * gg;
        vv = b2 * vv + ob2 * (gg * gg);
        pp -= lr * (mm * c1) / (sqrtf(vv * c2) + eps);
    };
    if (ps == w) {
        // flat: the parameter side is packed like the moments
        const bool v4 = ((((uintptr_t)p) | ((uintptr_t)g) | ((uintptr_t)m) | ((uintptr_t)v)) & 15u) == 0;
        int64_t head = 0;
        if (v4) {
            const int64_t n4 = count / 4;
            for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride) {
                float4 P = reinterpret_cast<float4*>(p)[i];
                const float4 G = reinterpret_cast<const float4*>(g)[i];
                float4 M = reinterpret_cast<float4*>(m)[i];
                float4 V = reinterpret_cast<float4*>(v)[i];
                step(P.x, G.x, M.x, V.x);
                step(P.y, G.y, M.y, V.y);
                step(P.z, G.z, M.z, V.z);
                step(P.w, G.w, M.w, V.w);
                reinterpret_cast<float4*>(p)[i] = P;
                reinterpret_cast<float4*>(m)[i] = M;
                reinterpret_cast<float4*>(v)[i] = V;
            }
            head = n4 * 4;
        }
        for (int64_t i = head + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) {
            float P = p[i], M = m[i], V = v[i];
            step(P, g[i], M, V);
            p[i] = P;
            m[i] = M;
            v[i] = V;
        }
    } else {
        // colour array inside an interleaved record: element i of the packed
        // side is float j of Gaussian gi, at gi * ps + j on the parameter side
        for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) {
            const int64_t gi = i / w, j = i - gi * w;
            float P = p[gi * ps + j], M = m[i], V = v[i];
            step(P, g[i], M, V);
            p[gi * ps + j] = P;
            m[i] = M;
            v[i] = V;
        }
    }
}

void launch_adam(const AdamArrays& a, hipStream_t s) {
    int64_t most = 0;
    for (int k = 0; k < kAdamArrays; ++k)
        if (a.on[k] && a.count[k] > most) most = a.count[k];
    if (most == 0) return;
    int64_t blocks = (most / 4 + 255) / 256;
    blocks = blocks < 1 ? 1 : (blocks > 2048 ? 2048 : blocks);
    hipLaunchKernelGGL(k_adam, dim3((unsigned)blocks, kAdamArrays), dim3(256), 0, s, a);
}

}  // namespace sgs
