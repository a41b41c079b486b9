// Mixed-radix (8, 4, 3, 2, 5) FP64 complex FFT of one line held in LDS, computed cooperatively by a
// group of threads: Stockham autosort stages, each thread reads its butterflies' inputs into
// registers, the group synchronises, then writes the outputs back in place.  Forward transform
// X_k = sum_n x_n exp(-2 pi i n k / N), unnormalised; the inverse is taken by conjugating data
// on the way in and out.  Twiddles W_N^n come from a table in LDS (host-computed in FP64).
#pragma once

#include <hip/hip_runtime.h>

namespace evp {

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
// multiply by -i
__device__ __forceinline__ double2 cmi(double2 a) { return make_double2(a.y, -a.x); }

// Complex values in global memory, accessed through address-space-1 pointers as native two-lane
// vectors (the HIP vector class has no assignment for address-space-qualified objects).
typedef double dvec2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ double2 gload2(gptr<const double2> p)
{
    const dvec2 t = *(gptr<const dvec2>)p;
    return make_double2(t.x, t.y);
}
__device__ __forceinline__ void gstore2(gptr<double2> p, double2 v)
{
    dvec2 t;
    t.x = v.x;
    t.y = v.y;
    *(gptr<dvec2>)p = t;
}

struct FftPlan {
    int n, nst;
    int r[10];
};

// Greedy factorisation into radices 8, 4, 3, 2, 5 (nst = -1 if another prime divides n).
__host__ __device__ constexpr FftPlan make_plan(int n)
{
    FftPlan p{n, 0, {0, 0, 0, 0, 0, 0, 0, 0, 0, 0}};
    int m = n;
    while (m > 1) {
        int R = (m % 8 == 0) ? 8 : (m % 4 == 0) ? 4 : (m % 3 == 0) ? 3 : (m % 2 == 0) ? 2 : (m % 5 == 0) ? 5 : 0;
        if (R == 0) { p.nst = -1; return p; }
        p.r[p.nst++] = R;
        m /= R;
    }
    return p;
}

template <int R> __device__ __forceinline__ void dft(double2* v);

template <> __device__ __forceinline__ void dft<2>(double2* v)
{
    double2 a = cadd(v[0], v[1]), b = csub(v[0], v[1]);
    v[0] = a; v[1] = b;
}

template <> __device__ __forceinline__ void dft<3>(double2* v)
{
    const double h3 = 0.86602540378443864676;   // sin(pi/3)
    double2 s = cadd(v[1], v[2]), d = csub(v[1], v[2]);
    double2 m = make_double2(v[0].x - 0.5 * s.x, v[0].y - 0.5 * s.y);
    double2 t = make_double2(h3 * d.y, -h3 * d.x);   // -i sin(pi/3) d
    v[0] = cadd(v[0], s);
    v[1] = cadd(m, t);
    v[2] = csub(m, t);
}

template <> __device__ __forceinline__ void dft<4>(double2* v)
{
    double2 a = cadd(v[0], v[2]), b = csub(v[0], v[2]);
    double2 c = cadd(v[1], v[3]), d = cmi(csub(v[1], v[3]));
    v[0] = cadd(a, c); v[2] = csub(a, c);
    v[1] = cadd(b, d); v[3] = csub(b, d);
}

// X_k = sum_n x_n W_5^{nk}: with a_1 = x1 + x4, b_1 = x1 - x4, a_2 = x2 + x3, b_2 = x2 - x3,
// X_{1,4} = x0 + c1 a1 + c2 a2 -/+ i (s1 b1 + s2 b2), X_{2,3} = x0 + c2 a1 + c1 a2 -/+ i (s2 b1 - s1 b2),
// c_k = cos(2 pi k / 5), s_k = sin(2 pi k / 5)
template <> __device__ __forceinline__ void dft<5>(double2* v)
{
    const double c1 = 0.30901699437494742410, c2 = -0.80901699437494742410;
    const double s1 = 0.95105651629515357212, s2 = 0.58778525229247312917;
    const double2 a1 = cadd(v[1], v[4]), b1 = csub(v[1], v[4]);
    const double2 a2 = cadd(v[2], v[3]), b2 = csub(v[2], v[3]);
    const double2 p1 = make_double2(v[0].x + c1 * a1.x + c2 * a2.x, v[0].y + c1 * a1.y + c2 * a2.y);
    const double2 p2 = make_double2(v[0].x + c2 * a1.x + c1 * a2.x, v[0].y + c2 * a1.y + c1 * a2.y);
    const double2 q1 = cmi(make_double2(s1 * b1.x + s2 * b2.x, s1 * b1.y + s2 * b2.y));   // -i (s1 b1 + s2 b2)
    const double2 q2 = cmi(make_double2(s2 * b1.x - s1 * b2.x, s2 * b1.y - s1 * b2.y));   // -i (s2 b1 - s1 b2)
    v[0] = cadd(v[0], cadd(a1, a2));
    v[1] = cadd(p1, q1);
    v[4] = csub(p1, q1);
    v[2] = cadd(p2, q2);
    v[3] = csub(p2, q2);
}

template <> __device__ __forceinline__ void dft<8>(double2* v)
{
    const double r2 = 0.70710678118654752440;   // 1/sqrt(2)
    double2 a[4], b[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) { a[k] = cadd(v[k], v[k + 4]); b[k] = csub(v[k], v[k + 4]); }
    // b_k *= W_8^k
    b[1] = make_double2(r2 * (b[1].x + b[1].y), r2 * (b[1].y - b[1].x));
    b[2] = cmi(b[2]);
    b[3] = make_double2(r2 * (b[3].y - b[3].x), -r2 * (b[3].x + b[3].y));
    dft<4>(a);
    dft<4>(b);
#pragma unroll
    for (int k = 0; k < 4; ++k) { v[2 * k] = a[k]; v[2 * k + 1] = b[k]; }
}

// Stage S of the N-point transform; NS = product of the radices of the earlier stages.
// buf: the line's element 0 in LDS, es: element stride, t in [0, T): this thread's slot.
template <int N, int T, int S, int NS>
__device__ __forceinline__ void fft_stages(double2* buf, int es, int t, bool active,
                                           const double2* tw)
{
    constexpr FftPlan P = make_plan(N);
    if constexpr (S < P.nst) {
        constexpr int R = P.r[S];
        constexpr int NB = N / R;
        constexpr int MB = (NB + T - 1) / T;
        constexpr int TWS = N / (NS * R);
        double2 v[MB][R];
#pragma unroll
        for (int m = 0; m < MB; ++m) {
            const int j = t + m * T;
            if (active && (NB % T == 0 || j < NB)) {
                const int k = j % NS;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    double2 x = buf[(j + r * NB) * es];
                    if (NS > 1 && r > 0) x = cmul(x, tw[r * k * TWS]);
                    v[m][r] = x;
                }
                dft<R>(v[m]);
            }
        }
        __syncthreads();
#pragma unroll
        for (int m = 0; m < MB; ++m) {
            const int j = t + m * T;
            if (active && (NB % T == 0 || j < NB)) {
                const int base = (j / NS) * NS * R + (j % NS);
#pragma unroll
                for (int r = 0; r < R; ++r) buf[(base + r * NS) * es] = v[m][r];
            }
        }
        __syncthreads();
        fft_stages<N, T, S + 1, NS * R>(buf, es, t, active, tw);
    }
}

// Threads per line used by the transform kernels for length N.
template <int N> constexpr int fft_threads() { return N >= 8 ? N / 8 : 1; }

}  // namespace evp
