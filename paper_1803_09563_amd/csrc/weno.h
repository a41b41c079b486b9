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
// same numbers as the usual form in v, up to the sign of b).  The weights d_k / (eps + IS_k)^2,
// normalised, are invariant under a common scale of the indicators, so they are formed from
// 4 (eps + IS_k) = 4 eps + 13/3 a_k^2 + b_k^2, and over the common denominator
// e1^2 e2^2 e3^2: w_k = d_k prod_{m != k} e_m^2, with the linear weights d_k = 0.1, 0.6, 0.3
// folded into the candidate coefficients of the numerator.
template <typename T>
__device__ __forceinline__ T weno5u(T v1, T v2, T v3, T v4, T v5, T eps2)
{
    const T s1 = v2 - v1, s2 = v3 - v2, s3 = v4 - v3, s4 = v5 - v4;
    const T a1 = s2 - s1, a2 = s3 - s2, a3 = s4 - s3;
    const T b1 = (T)3 * s2 - s1, b2 = s2 + s3, b3 = s4 - (T)3 * s3;
    const T c = (T)(13.0 / 3.0), e4 = (T)4 * eps2;
    T e1 = b1 * b1 + (c * a1 * a1 + e4);
    T e2 = b2 * b2 + (c * a2 * a2 + e4);
    T e3 = b3 * b3 + (c * a3 * a3 + e4);
    if constexpr (sizeof(T) == 4) {
        // FP32: eps h^2 squared twice in the common denominator underflows on fine grids; any
        // common scale serves, so normalise by (about) the largest indicator with the unrefined
        // hardware reciprocal
        const T im = __builtin_amdgcn_rcpf(fmaxf(fmaxf(e1, e2), e3));
        e1 *= im; e2 *= im; e3 *= im;
    }
    e1 *= e1; e2 *= e2; e3 *= e3;
    const T p1 = e2 * e3, p2 = e1 * e3, p3 = e1 * e2;
    // 0.1 q1, 0.6 q2, 0.3 q3
    const T r1 = (T)(1.0 / 12.0) * s2 - (T)(1.0 / 30.0) * s1;
    const T r2 = (T)0.1 * s2 + (T)0.2 * s3;
    const T r3 = (T)0.2 * s3 - (T)0.05 * s4;
    const T num = p1 * r1 + p2 * r2 + p3 * r3;
    const T den = (T)0.1 * p1 + (T)0.6 * p2 + (T)0.3 * p3;
    // FP32: the hardware reciprocal (about one ulp) is already at the precision of the FP32 sum;
    // FP64 refines it to full precision
    const T iw = sizeof(T) == 4 ? (T)__builtin_amdgcn_rcpf((float)den) : fast_rcp(den);
    return v3 + num * iw;
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
