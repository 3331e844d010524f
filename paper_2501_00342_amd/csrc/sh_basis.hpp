// Real spherical harmonics up to degree 3 (Condon-Shortley phase), as
// polynomials of a unit direction (x, y, z), and their partial derivatives.
// Colour model eq. 4 of SG-Splatting; normalisation
// K_l^m = sqrt((2l+1)/(4 pi) (l-|m|)!/(l+|m|)!), times sqrt(2) for m != 0.
// Order: l-major, m = -l..l.
#pragma once

#include <hip/hip_runtime.h>

namespace sgs {

#define SGS_PI 3.14159265358979323846

template <int DEG, typename T>
__device__ __forceinline__ void sh_eval(T x, T y, T z, T* Y) {
    Y[0] = T(0.5 * sqrt(1.0 / SGS_PI));
    if (DEG >= 1) {
        const T c1 = T(sqrt(3.0 / (4.0 * SGS_PI)));
        Y[1] = -c1 * y;
        Y[2] = c1 * z;
        Y[3] = -c1 * x;
    }
    if (DEG >= 2) {
        const T a = T(0.5 * sqrt(15.0 / SGS_PI));
        const T b = T(0.25 * sqrt(5.0 / SGS_PI));
        const T c = T(0.25 * sqrt(15.0 / SGS_PI));
        Y[4] = a * x * y;
        Y[5] = -a * y * z;
        Y[6] = b * (T(3) * z * z - T(1));
        Y[7] = -a * x * z;
        Y[8] = c * (x * x - y * y);
    }
    if (DEG >= 3) {
        const T a = T(0.25 * sqrt(35.0 / (2.0 * SGS_PI)));
        const T b = T(0.5 * sqrt(105.0 / SGS_PI));
        const T c = T(0.25 * sqrt(21.0 / (2.0 * SGS_PI)));
        const T d = T(0.25 * sqrt(7.0 / SGS_PI));
        const T e = T(0.25 * sqrt(105.0 / SGS_PI));
        const T z5 = T(5) * z * z - T(1);
        Y[9] = -a * y * (T(3) * x * x - y * y);
        Y[10] = b * x * y * z;
        Y[11] = -c * y * z5;
        Y[12] = d * z * (T(5) * z * z - T(3));
        Y[13] = -c * x * z5;
        Y[14] = e * z * (x * x - y * y);
        Y[15] = -a * x * (x * x - T(3) * y * y);
    }
}

// dY/dx, dY/dy, dY/dz of the polynomials above (x, y, z independent).
template <int DEG, typename T>
__device__ __forceinline__ void sh_grad(T x, T y, T z, T* gx, T* gy, T* gz) {
    gx[0] = gy[0] = gz[0] = T(0);
    if (DEG >= 1) {
        const T c1 = T(sqrt(3.0 / (4.0 * SGS_PI)));
        gx[1] = T(0); gy[1] = -c1; gz[1] = T(0);
        gx[2] = T(0); gy[2] = T(0); gz[2] = c1;
        gx[3] = -c1; gy[3] = T(0); gz[3] = T(0);
    }
    if (DEG >= 2) {
        const T a = T(0.5 * sqrt(15.0 / SGS_PI));
        const T b = T(0.25 * sqrt(5.0 / SGS_PI));
        const T c = T(0.25 * sqrt(15.0 / SGS_PI));
        gx[4] = a * y;       gy[4] = a * x;        gz[4] = T(0);
        gx[5] = T(0);        gy[5] = -a * z;       gz[5] = -a * y;
        gx[6] = T(0);        gy[6] = T(0);         gz[6] = T(6) * b * z;
        gx[7] = -a * z;      gy[7] = T(0);         gz[7] = -a * x;
        gx[8] = T(2) * c * x; gy[8] = T(-2) * c * y; gz[8] = T(0);
    }
    if (DEG >= 3) {
        const T a = T(0.25 * sqrt(35.0 / (2.0 * SGS_PI)));
        const T b = T(0.5 * sqrt(105.0 / SGS_PI));
        const T c = T(0.25 * sqrt(21.0 / (2.0 * SGS_PI)));
        const T d = T(0.25 * sqrt(7.0 / SGS_PI));
        const T e = T(0.25 * sqrt(105.0 / SGS_PI));
        const T z5 = T(5) * z * z - T(1);
        gx[9] = -a * T(6) * x * y;           gy[9] = -a * (T(3) * x * x - T(3) * y * y); gz[9] = T(0);
        gx[10] = b * y * z;                  gy[10] = b * x * z;                          gz[10] = b * x * y;
        gx[11] = T(0);                       gy[11] = -c * z5;                            gz[11] = -c * y * T(10) * z;
        gx[12] = T(0);                       gy[12] = T(0);                               gz[12] = d * (T(15) * z * z - T(3));
        gx[13] = -c * z5;                    gy[13] = T(0);                               gz[13] = -c * x * T(10) * z;
        gx[14] = T(2) * e * x * z;           gy[14] = T(-2) * e * y * z;                  gz[14] = e * (x * x - y * y);
        gx[15] = -a * (T(3) * x * x - T(3) * y * y); gy[15] = a * T(6) * x * y;          gz[15] = T(0);
    }
}

}  // namespace sgs
