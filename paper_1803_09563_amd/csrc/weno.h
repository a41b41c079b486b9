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

// Fifth-order WENO from the five undivided one-sided differences v1..v5 (spacing folded out):
// returns h * dB/dx.  eps2 = eps h^2 keeps the weights equal to those of the divided form.
// Written on the differences s_k = v_{k+1} - v_k: the three candidate stencils are v3 plus
// q1 = -s1/3 + 5 s2/6, q2 = s2/6 + s3/3, q3 = 2 s3/3 - s4/6, and the Jiang-Shu indicators are
// 13/12 a_k^2 + 1/4 b_k^2 with a_k = s_{k+1} - s_k and b = 3 s2 - s1, s2 + s3, s4 - 3 s3 (the
// same numbers as the usual form in v, up to the sign of b, with fewer operations).
template <typename T>
__device__ __forceinline__ T weno5u(T v1, T v2, T v3, T v4, T v5, T eps2)
{
    const T c13 = (T)(13.0 / 12.0), q = (T)0.25;
    const T s1 = v2 - v1, s2 = v3 - v2, s3 = v4 - v3, s4 = v5 - v4;
    const T a1 = s2 - s1, a2 = s3 - s2, a3 = s4 - s3;
    const T b1 = (T)3 * s2 - s1, b2 = s2 + s3, b3 = s4 - (T)3 * s3;
    T e1 = eps2 + c13 * a1 * a1 + q * b1 * b1;
    T e2 = eps2 + c13 * a2 * a2 + q * b2 * b2;
    T e3 = eps2 + c13 * a3 * a3 + q * b3 * b3;
    if constexpr (sizeof(T) == 4) {
        // FP32: eps h^2 squared twice in the common denominator underflows on fine grids; the
        // weights are invariant under a common scale, so normalise by (about) the largest
        // indicator; any scale serves, so the hardware reciprocal needs no refinement here
        const T im = __builtin_amdgcn_rcpf(fmaxf(fmaxf(e1, e2), e3));
        e1 *= im; e2 *= im; e3 *= im;
    }
    e1 *= e1; e2 *= e2; e3 *= e3;
    const T w1 = (T)0.1 * e2 * e3, w2 = (T)0.6 * e1 * e3, w3 = (T)0.3 * e1 * e2;
    const T q1 = (T)(5.0 / 6.0) * s2 - (T)(1.0 / 3.0) * s1;
    const T q2 = (T)(1.0 / 6.0) * s2 + (T)(1.0 / 3.0) * s3;
    const T q3 = (T)(2.0 / 3.0) * s3 - (T)(1.0 / 6.0) * s4;
    // FP32: the hardware reciprocal (about one ulp) is already at the precision of the FP32 sum;
    // FP64 refines it to full precision
    const T iw = sizeof(T) == 4 ? (T)__builtin_amdgcn_rcpf((float)(w1 + w2 + w3)) : fast_rcp(w1 + w2 + w3);
    return v3 + (w1 * q1 + w2 * q2 + w3 * q3) * iw;
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
