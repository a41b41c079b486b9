// Field I/O (FP64 user arrays <-> internal storage, where B is kept as B - I) and the health
// reduction: the trigger conditions of the paper's local artificial diffusion (Sec. 3.1: loss of
// positive definiteness det B < 0, and tr B >= 0.95 L^2 for FENE-P), non-finite cells, the
// largest discrete divergence and the kinetic energy.
#include "evp_internal.h"

namespace evp {

namespace {

constexpr int HB = 256;            // threads per health block
constexpr int HBLOCKS = 1024;      // health blocks (grid-stride); partials stay small

template <typename T>
__global__ __launch_bounds__(256) void k_write(const Desc* Dp, int parity, int walls, int ny,
                                               int nx, const double* u, const double* v,
                                               const double* w, const double* B6,
                                               const double* hist)
{
    const Desc& D = *Dp;
    const long long n = D.ncell, ps = D.ps;
    const long long q = (long long)blockIdx.x * 256 + threadIdx.x;
    if (q >= n) return;
    D.u[q] = u[q];
    D.w[q] = w[q];
    const int j = (int)((q / nx) % ny);
    D.v[q] = (walls && j == ny - 1) ? 0.0 : v[q];
    T* Bt = (T*)D.Bt[parity];
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        const double d = (c == 0 || c == 3 || c == 5) ? 1.0 : 0.0;
        Bt[c * ps + q] = (T)(B6[c * n + q] - d);
    }
    T* RT = (T*)D.RT;
    T* RU = (T*)D.RU;
#pragma unroll
    for (int c = 0; c < 6; ++c) RT[c * ps + q] = hist ? (T)hist[c * n + q] : (T)0;
#pragma unroll
    for (int c = 0; c < 3; ++c) RU[c * ps + q] = hist ? (T)hist[(6 + c) * n + q] : (T)0;
    D.p[q] = 0.0;
}

template <typename T>
__global__ __launch_bounds__(256) void k_read(const Desc* Dp, int parity, unsigned mask, double* u,
                                              double* v, double* w, double* p, double* B6,
                                              double* hist)
{
    const Desc& D = *Dp;
    const long long n = D.ncell, ps = D.ps;
    const long long q = (long long)blockIdx.x * 256 + threadIdx.x;
    if (q >= n) return;
    if (mask & EVP_READ_U) u[q] = D.u[q];
    if (mask & EVP_READ_V) v[q] = D.v[q];
    if (mask & EVP_READ_W) w[q] = D.w[q];
    if (mask & EVP_READ_P) p[q] = D.p[q];
    if (mask & EVP_READ_B) {
        const T* Bt = (const T*)D.Bt[parity];
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            const double d = (c == 0 || c == 3 || c == 5) ? 1.0 : 0.0;
            B6[c * n + q] = (double)Bt[c * ps + q] + d;
        }
    }
    if (mask & EVP_READ_HIST) {
        const T* RT = (const T*)D.RT;
        const T* RU = (const T*)D.RU;
#pragma unroll
        for (int c = 0; c < 6; ++c) hist[c * n + q] = (double)RT[c * ps + q];
#pragma unroll
        for (int c = 0; c < 3; ++c) hist[(6 + c) * n + q] = (double)RU[c * ps + q];
    }
}

// per-block partials: [nonfinite, det_le0, trace_ge95, max_div, energy]
template <typename T>
__global__ __launch_bounds__(HB) void k_health(const Desc* Dp, int parity)
{
    const Desc& D = *Dp;
    const int nx = D.nx, ny = D.ny, nz = D.nz;
    const long long n = D.ncell, ps = D.ps, sxy = (long long)nx * ny;
    const T* Bt = (const T*)D.Bt[parity];
    double cnt0 = 0, cnt1 = 0, cnt2 = 0, mdiv = 0, en = 0;
    const double thr = 0.95 * D.L2;
    for (long long q = (long long)blockIdx.x * HB + threadIdx.x; q < n; q += (long long)gridDim.x * HB) {
        const int i = (int)(q % nx);
        const long long r = q / nx;
        const int j = (int)(r % ny), k = (int)(r / ny);
        double b[6];
#pragma unroll
        for (int c = 0; c < 6; ++c) b[c] = (double)Bt[c * ps + q];
        b[0] += 1.0; b[3] += 1.0; b[5] += 1.0;
        const double u = D.u[q], v = D.v[q], w = D.w[q];
        bool fin = isfinite(u) && isfinite(v) && isfinite(w);
#pragma unroll
        for (int c = 0; c < 6; ++c) fin = fin && isfinite(b[c]);
        cnt0 += fin ? 0.0 : 1.0;
        const double det = b[0] * (b[3] * b[5] - b[4] * b[4]) - b[1] * (b[1] * b[5] - b[4] * b[2])
                         + b[2] * (b[1] * b[4] - b[3] * b[2]);
        cnt1 += (det <= 0.0) ? 1.0 : 0.0;
        if (D.model == EVP_FENE_P) cnt2 += (b[0] + b[3] + b[5] >= thr) ? 1.0 : 0.0;
        const double um = D.u[q - i + (i == 0 ? nx - 1 : i - 1)];
        const double wm = D.w[k == 0 ? q + (long long)(nz - 1) * sxy : q - sxy];
        double vm;
        if (j > 0) vm = D.v[q - nx];
        else vm = D.walls ? 0.0 : D.v[q + (long long)(ny - 1) * nx];
        const double dv = fabs((u - um) * D.idx + (v - vm) * D.idy + (w - wm) * D.idz);
        mdiv = fmax(mdiv, dv);
        en += u * u + v * v + w * w;
    }
    __shared__ double sh[5][HB];
    sh[0][threadIdx.x] = cnt0; sh[1][threadIdx.x] = cnt1; sh[2][threadIdx.x] = cnt2;
    sh[3][threadIdx.x] = mdiv; sh[4][threadIdx.x] = en;
    __syncthreads();
    for (int s = HB / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            sh[0][threadIdx.x] += sh[0][threadIdx.x + s];
            sh[1][threadIdx.x] += sh[1][threadIdx.x + s];
            sh[2][threadIdx.x] += sh[2][threadIdx.x + s];
            sh[3][threadIdx.x] = fmax(sh[3][threadIdx.x], sh[3][threadIdx.x + s]);
            sh[4][threadIdx.x] += sh[4][threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x < 5) D.red[blockIdx.x * 5 + threadIdx.x] = sh[threadIdx.x][0];
}

// Fixed-order reduction of the HBLOCKS partials -> red[HBLOCKS*5 .. +5) and, if out5 is not null,
// out5[0..5): thread t folds the partials of blocks t, t + HB, t + 2 HB, ... in that order, then a
// fixed pairwise tree over the threads, so every call sums in the same order (bitwise
// reproducible).
__global__ __launch_bounds__(HB) void k_health_final(const Desc* Dp, int nblocks, double* out5)
{
    const Desc& D = *Dp;
    const int t = threadIdx.x;
    double a0 = 0, a1 = 0, a2 = 0, a3 = 0, a4 = 0;
    for (int b = t; b < nblocks; b += HB) {
        a0 += D.red[b * 5 + 0]; a1 += D.red[b * 5 + 1]; a2 += D.red[b * 5 + 2];
        a3 = fmax(a3, D.red[b * 5 + 3]); a4 += D.red[b * 5 + 4];
    }
    __shared__ double sh[5][HB];
    sh[0][t] = a0; sh[1][t] = a1; sh[2][t] = a2; sh[3][t] = a3; sh[4][t] = a4;
    __syncthreads();
    for (int s = HB / 2; s > 0; s >>= 1) {
        if (t < s) {
            sh[0][t] += sh[0][t + s];
            sh[1][t] += sh[1][t + s];
            sh[2][t] += sh[2][t + s];
            sh[3][t] = fmax(sh[3][t], sh[3][t + s]);
            sh[4][t] += sh[4][t + s];
        }
        __syncthreads();
    }
    if (t < 5) {
        const double v = t == 4 ? 0.5 * sh[4][0] * D.dx * D.dy * D.dz : sh[t][0];
        D.red[HBLOCKS * 5 + t] = v;
        if (out5) out5[t] = v;
    }
}

// one block per guard region: every word gets the pattern
__global__ __launch_bounds__(256) void k_guard_fill(gptr<unsigned long long> ws, gptr<const long long> table, int n)
{
    const int gi = blockIdx.x;
    if (gi >= n) return;
    const long long off = table[2 * gi] / 8, words = table[2 * gi + 1];
    for (long long t = threadIdx.x; t < words; t += 256) ws[off + t] = kGuardWord;
}

// one block: count the words of every region that differ from the pattern, summed in a fixed
// order
__global__ __launch_bounds__(256) void k_guard_check(gptr<const unsigned long long> ws, gptr<const long long> table,
                                                     int n, gptr<double> out)
{
    double bad = 0.0;
    for (int gi = 0; gi < n; ++gi) {
        const long long off = table[2 * gi] / 8, words = table[2 * gi + 1];
        for (long long t = threadIdx.x; t < words; t += 256) bad += ws[off + t] != kGuardWord ? 1.0 : 0.0;
    }
    __shared__ double sh[256];
    sh[threadIdx.x] = bad;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = sh[0];
}

}  // namespace

hipError_t launch_guard_fill(char* ws, const long long* table, int n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_guard_fill, dim3(n), dim3(256), 0, s, (gptr<unsigned long long>)ws,
                       (gptr<const long long>)table, n);
    return hipGetLastError();
}

hipError_t launch_guard_check(const char* ws, const long long* table, int n, double* out, hipStream_t s)
{
    hipLaunchKernelGGL(k_guard_check, dim3(1), dim3(256), 0, s, (gptr<const unsigned long long>)ws,
                       (gptr<const long long>)table, n, (gptr<double>)out);
    return hipGetLastError();
}

hipError_t launch_write_fields(const Desc* d, int precision, long long ncell, int ny, int nx,
                               int walls, int parity, const double* u, const double* v,
                               const double* w, const double* B6, const double* hist,
                               hipStream_t s)
{
    dim3 grid((unsigned)((ncell + 255) / 256));
    if (precision == EVP_MIXED)
        hipLaunchKernelGGL(k_write<float>, grid, dim3(256), 0, s, d, parity, walls, ny, nx, u, v, w, B6, hist);
    else
        hipLaunchKernelGGL(k_write<double>, grid, dim3(256), 0, s, d, parity, walls, ny, nx, u, v, w, B6, hist);
    return hipGetLastError();
}

hipError_t launch_read_fields(const Desc* d, int precision, long long ncell, int parity,
                              unsigned mask, double* u, double* v, double* w, double* p,
                              double* B6, double* hist, hipStream_t s)
{
    dim3 grid((unsigned)((ncell + 255) / 256));
    if (precision == EVP_MIXED)
        hipLaunchKernelGGL(k_read<float>, grid, dim3(256), 0, s, d, parity, mask, u, v, w, p, B6, hist);
    else
        hipLaunchKernelGGL(k_read<double>, grid, dim3(256), 0, s, d, parity, mask, u, v, w, p, B6, hist);
    return hipGetLastError();
}

// Enqueues the reduction; the five results land at d->red + HBLOCKS*5 and, if out5 is not null,
// in out5 (device memory or host memory the device can write); the caller synchronises.
hipError_t launch_health(const Desc* d, int precision, int parity, double* out5, hipStream_t s)
{
    if (precision == EVP_MIXED)
        hipLaunchKernelGGL(k_health<float>, dim3(HBLOCKS), dim3(HB), 0, s, d, parity);
    else
        hipLaunchKernelGGL(k_health<double>, dim3(HBLOCKS), dim3(HB), 0, s, d, parity);
    hipLaunchKernelGGL(k_health_final, dim3(1), dim3(HB), 0, s, d, HBLOCKS, out5);
    return hipGetLastError();
}

}  // namespace evp
