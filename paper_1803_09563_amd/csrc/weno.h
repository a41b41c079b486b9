// Device helpers shared by the stencil kernels: a full-precision reciprocal, the fifth-order WENO
// derivative of Sec. 3.1 (Jiang-Peng form with the Jiang-Shu smoothness indicators) and the
// regularised Heaviside of the two-phase mixture.
#pragma once

#include <hip/hip_runtime.h>

namespace evp {

// reciprocal to full precision: hardware estimate refined by Newton steps (x <- x (2 - a x))
__device__ __forceinline__ double fast_rcp(double a)
{
    double x = __builtin_amdgcn_rcp(a);
    x = fma(x, fma(-a, x, 1.0), x);
    x = fma(x, fma(-a, x, 1.0), x);
    return x;
}
__device__ __forceinline__ float fast_rcp(float a)
{
    float x = __builtin_amdgcn_rcpf(a);
    return fmaf(x, fmaf(-a, x, 1.0f), x);
}

// Fifth-order WENO from the five undivided one-sided differences e1..e5 (spacing folded out):
// returns h * dB/dx.  eps2 = eps h^2 keeps the weights equal to those of the divided form.
template <typename T>
__device__ __forceinline__ T weno5u(T v1, T v2, T v3, T v4, T v5, T eps2)
{
    const T c13 = (T)(13.0 / 12.0), q = (T)0.25;
    const T p1 = v1 * (T)(1.0 / 3.0) - v2 * (T)(7.0 / 6.0) + v3 * (T)(11.0 / 6.0);
    const T p2 = -v2 * (T)(1.0 / 6.0) + v3 * (T)(5.0 / 6.0) + v4 * (T)(1.0 / 3.0);
    const T p3 = v3 * (T)(1.0 / 3.0) + v4 * (T)(5.0 / 6.0) - v5 * (T)(1.0 / 6.0);
    T a = v1 - (T)2 * v2 + v3, b = v1 - (T)4 * v2 + (T)3 * v3;
    T e1 = eps2 + c13 * a * a + q * b * b;
    a = v2 - (T)2 * v3 + v4; b = v2 - v4;
    T e2 = eps2 + c13 * a * a + q * b * b;
    a = v3 - (T)2 * v4 + v5; b = (T)3 * v3 - (T)4 * v4 + v5;
    T e3 = eps2 + c13 * a * a + q * b * b;
    if constexpr (sizeof(T) == 4) {
        // FP32: eps h^2 squared twice in the common denominator underflows on fine grids; the
        // weights are invariant under a common scale, so normalise by the largest indicator
        const T im = fast_rcp(fmaxf(fmaxf(e1, e2), e3));
        e1 *= im; e2 *= im; e3 *= im;
    }
    e1 *= e1; e2 *= e2; e3 *= e3;
    const T w1 = (T)0.1 * e2 * e3, w2 = (T)0.6 * e1 * e3, w3 = (T)0.3 * e1 * e2;
    return (w1 * p1 + w2 * p2 + w3 * p3) * fast_rcp(w1 + w2 + w3);
}

// regularised Heaviside of the two-phase mixture (Sec. 3.2.1): 0 below -e, 1 above e, smooth
// between
__device__ __forceinline__ double heaviside(double phi, double e)
{
    if (phi < -e) return 0.0;
    if (phi > e) return 1.0;
    return 0.5 * (1.0 + phi / e + sin(M_PI * phi / e) / M_PI);
}

}  // namespace evp
