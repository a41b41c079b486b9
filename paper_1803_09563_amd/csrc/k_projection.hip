// Pressure projection, Sec. 3.2.2 Eqs. (var poisson) and (projection) with constant rho:
//   r = rho (D_h u*) / dt;  L_h p = r (zero-mean p);  u^{n+1} = u* - (dt/rho) G_h p.
// The 7-point Laplacian L_h = D_h G_h is diagonalised by discrete Fourier transforms in periodic
// directions (eigenvalues -(4/h^2) sin^2(pi k/N)); across walls (homogeneous Neumann rows) each
// (kx, kz) mode is a tridiagonal system in y solved by a Thomas sweep.
//
// Passes over the half spectrum S[kz][j][kx] (kx < nx/2+1, FP64 complex; rows padded to a
// multiple of 8 values, 128 bytes):
//   periodic: div+fft(x) | fft(y) | fft(z), divide, ifft(z) | ifft(y) | ifft(x) -> p | correct
//   walls:    div+fft(x) | fft(z) | Thomas(y)                | ifft(z) | ifft(x) -> p | correct
// Real x-lines are transformed two at a time as one complex line (a + i b).  Periodic batches of
// nx == ny <= 128 with enough z planes to fill the chip fuse the first two and the last two
// periodic passes into one block per z plane, whose half-spectrum plane stays in LDS.
#include "evp_internal.h"
#include "fft_lds.h"

namespace evp {

namespace {

constexpr int NT = 256;    // threads per block of the line-transform kernels
constexpr int TK = 16;     // consecutive kx per block in the strided passes

__device__ __forceinline__ int wrapi(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// Strided tile <-> LDS: element e = tid + m NT of the N x TK tile is (row n = e / TK, column
// c = e % TK).  The column is the same for every m of a thread, so its bounds check is hoisted;
// loads are issued in groups of up to 16 before their LDS stores.
template <int N, bool CONJ>
__device__ __forceinline__ void tile_in(double2* buf, gptr<const double2> __restrict__ src, long long es,
                                        bool colok, int tid)
{
    constexpr int TOT = N * TK, M = (TOT + NT - 1) / NT, G = M < 16 ? M : 16;
    const int c = tid % TK, n0 = tid / TK;
#pragma unroll
    for (int g0 = 0; g0 < M; g0 += G) {
        double2 v[G];
#pragma unroll
        for (int m = 0; m < G; ++m) {
            const int n = n0 + (g0 + m) * (NT / TK);
            v[m] = make_double2(0.0, 0.0);
            if (colok && n < N) v[m] = gload2(src + n * es + c);
        }
#pragma unroll
        for (int m = 0; m < G; ++m) {
            const int n = n0 + (g0 + m) * (NT / TK);
            if (n < N) buf[n * TK + c] = CONJ ? cconj(v[m]) : v[m];
        }
    }
}

template <int N, bool CONJ>
__device__ __forceinline__ void tile_out(const double2* buf, gptr<double2> __restrict__ dst, long long es,
                                         bool colok, int tid)
{
    constexpr int TOT = N * TK, M = (TOT + NT - 1) / NT;
    const int c = tid % TK, n0 = tid / TK;
    if (!colok) return;
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const int n = n0 + m * (NT / TK);
        if (n < N) {
            const double2 x = buf[n * TK + c];
            gstore2(dst + n * es + c, CONJ ? cconj(x) : x);
        }
    }
}

// ---------------------------------------------------------------------------------------------
// div + forward x transform
// ---------------------------------------------------------------------------------------------
template <int N>
__global__ __launch_bounds__(NT) void k_div_fftx(Batch B)
{
    constexpr int T = fft_threads<N>();
    constexpr int LP = NT / T;                 // complex lines (= real line pairs) per block
    constexpr int NHF = N / 2 + 1;
    __shared__ double2 buf[LP * N];
    __shared__ double2 tw[N];
    const Desc& D = *B.d[blockIdx.y];
    const double sc = D.rho / B.dt[blockIdx.y];
    const int tid = threadIdx.x;
    for (int n = tid; n < N; n += NT) tw[n] = gload2((gptr<const double2>)D.twx + n);
    const gptr<const double> us = (gptr<const double>)D.us;
    const gptr<const double> vs = (gptr<const double>)D.vs;
    const gptr<const double> ws = (gptr<const double>)D.ws;
    const gptr<double2> spec = (gptr<double2>)D.spec;
    const int ny = D.ny, nz = D.nz;
    const int nlines = ny * nz;
    const int npairs = (nlines + 1) >> 1;
    const int pair0 = blockIdx.x * LP;
    const double idx = D.idx, idy = D.idy, idz = D.idz;
    const long long sxy = (long long)N * ny;
    // divergence of u* on the block's lines; loads of four elements (24 values) are issued
    // before their arithmetic and LDS stores
    constexpr int M = (LP * N + NT - 1) / NT, G = M < 4 ? M : 4;
    const bool walls = D.walls != 0;
#pragma unroll
    for (int g0 = 0; g0 < M; g0 += G) {
        double ld[G][2][7];
        int slot[G];
#pragma unroll
        for (int m = 0; m < G; ++m) {
            const int e = tid + (g0 + m) * NT;
            const int ee = e < LP * N ? e : 0;
            const int lp = ee / N, i = ee - lp * N;
            const int pair = pair0 + lp;
            slot[m] = (e < LP * N) ? ee : -1;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                int l = 2 * pair + h;
                const bool ok = pair < npairs && l < nlines;
                l = ok ? l : 0;
                const int k = l / ny, j = l - k * ny;
                const long long q = (long long)l * N + i;
                ld[m][h][0] = us[q];
                ld[m][h][1] = us[q - i + wrapi(i - 1, N)];
                ld[m][h][2] = vs[q];
                ld[m][h][3] = (j > 0) ? vs[q - N] : vs[q + (long long)(ny - 1) * N];
                ld[m][h][4] = ws[q];
                ld[m][h][5] = (k > 0) ? ws[q - sxy] : ws[q + (long long)(nz - 1) * sxy];
                ld[m][h][6] = (ok ? 1.0 : 0.0) * ((j == 0 && walls) ? 0.0 : 1.0);   // flags
                if (!ok) ld[m][h][6] = -1.0;
            }
        }
#pragma unroll
        for (int m = 0; m < G; ++m) {
            if (slot[m] < 0) continue;
            double r2[2];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const double* a = ld[m][h];
                const double vm = (a[6] > 0.0) ? a[3] : 0.0;        // wall: v = 0 below row 0
                const double rr = sc * ((a[0] - a[1]) * idx + (a[2] - vm) * idy + (a[4] - a[5]) * idz);
                r2[h] = (a[6] < 0.0) ? 0.0 : rr;
            }
            buf[slot[m]] = make_double2(r2[0], r2[1]);
        }
    }
    __syncthreads();
    const int lp = tid / T, t = tid - (tid / T) * T;
    fft_stages<N, T, 0, 1>(buf + lp * N, 1, t, lp < LP, tw);
    const int sh = D.sh;
    for (int e = tid; e < LP * NHF; e += NT) {
        const int l2 = e / NHF, k = e - l2 * NHF;
        const int pair = pair0 + l2;
        if (pair >= npairs) continue;
        const double2 Z = buf[l2 * N + k];
        const double2 Zc = cconj(buf[l2 * N + (k == 0 ? 0 : N - k)]);
        const double2 s = cadd(Z, Zc), d = csub(Z, Zc);
        const int la = 2 * pair;
        gstore2(spec + (long long)la * sh + k, make_double2(0.5 * s.x, 0.5 * s.y));
        if (la + 1 < nlines)
            gstore2(spec + (long long)(la + 1) * sh + k, make_double2(0.5 * d.y, -0.5 * d.x));
    }
}

// ---------------------------------------------------------------------------------------------
// periodic grids whose x-y half-spectrum plane fits in LDS: one block per z plane does the
// divergence and the forward x and y transforms in one pass, and the inverse y and x transforms
// in another (the same line transforms, twiddles and two-for-one formulas as the separate
// passes, so the same numbers, with two spectrum round trips and two launches fewer)
// ---------------------------------------------------------------------------------------------
constexpr int NTP = 1024;   // threads of the plane kernels

// threads per y column: the largest of N/8, N/16, N/32 (at least 1) that lets all N/2 + 1 columns
// of the plane be transformed at once
template <int N>
constexpr int plane_y_threads()
{
    int t = fft_threads<N>();
    while (t > 1 && (N / 2 + 1) * t > NTP) t /= 2;
    return t;
}

// y transforms of all nh columns of the plane in LDS (stride nh)
template <int N>
__device__ __forceinline__ void plane_y_fft(double2* buf, const double2* tw, int tid)
{
    constexpr int NH = N / 2 + 1, TY = plane_y_threads<N>();
    static_assert(NH * TY <= NTP, "one pass of y transforms");
    const int col = tid / TY, t = tid - (tid / TY) * TY;
    fft_stages<N, TY, 0, 1>(buf + (col < NH ? col : 0), NH, t, col < NH, tw);
}

template <int N>
__global__ __launch_bounds__(NTP) void k_div_fftxy(Batch B)
{
    constexpr int NH = N / 2 + 1, L = N / 2, TX = fft_threads<N>();
    static_assert(L * TX <= NTP, "one pass of x transforms");
    __shared__ double2 buf[N * NH];
    __shared__ double2 twx[N], twy[N];
    const Desc& D = *B.d[blockIdx.y];
    const int tid = threadIdx.x, k = blockIdx.x;
    for (int n = tid; n < N; n += NTP) {
        twx[n] = gload2((gptr<const double2>)D.twx + n);
        twy[n] = gload2((gptr<const double2>)D.twy + n);
    }
    const double sc = D.rho / B.dt[blockIdx.y];
    const gptr<const double> us = (gptr<const double>)D.us;
    const gptr<const double> vs = (gptr<const double>)D.vs;
    const gptr<const double> ws = (gptr<const double>)D.ws;
    const int nz = D.nz;
    const long long sxy = (long long)N * N;
    const double idx = D.idx, idy = D.idy, idz = D.idz;
    // divergence of u* on the plane; complex line p holds rows 2p (real) and 2p + 1 (imaginary).
    // Loads of four elements (48 values) are issued before their arithmetic and LDS stores.
    constexpr int MD = (L * N + NTP - 1) / NTP, GD = MD < 4 ? MD : 4;
#pragma unroll
    for (int g0 = 0; g0 < MD; g0 += GD) {
        double ld[GD][2][6];
#pragma unroll
        for (int m = 0; m < GD; ++m) {
            const int e = tid + (g0 + m) * NTP;
            const int ee = (g0 + m < MD && e < L * N) ? e : 0;
            const int p = ee / N, i = ee - (ee / N) * N;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int j = 2 * p + h;
                const long long q = ((long long)k * N + j) * N + i;
                ld[m][h][0] = us[q];
                ld[m][h][1] = us[q - i + wrapi(i - 1, N)];
                ld[m][h][2] = vs[q];
                ld[m][h][3] = (j > 0) ? vs[q - N] : vs[q + (long long)(N - 1) * N];
                ld[m][h][4] = ws[q];
                ld[m][h][5] = (k > 0) ? ws[q - sxy] : ws[q + (long long)(nz - 1) * sxy];
            }
        }
#pragma unroll
        for (int m = 0; m < GD; ++m) {
            const int e = tid + (g0 + m) * NTP;
            if (g0 + m >= MD || e >= L * N) continue;
            double r2[2];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const double* a = ld[m][h];
                r2[h] = sc * ((a[0] - a[1]) * idx + (a[2] - a[3]) * idy + (a[4] - a[5]) * idz);
            }
            buf[e] = make_double2(r2[0], r2[1]);
        }
    }
    __syncthreads();
    {
        const int lp = tid / TX, t = tid - (tid / TX) * TX;
        fft_stages<N, TX, 0, 1>(buf + (lp < L ? lp : 0) * N, 1, t, lp < L, twx);
    }
    // two real spectra from each complex line, into rows j of the plane's half spectrum [j][kx]
    constexpr int MS = (L * NH + NTP - 1) / NTP;
    double2 za[MS], zb[MS];
#pragma unroll
    for (int m = 0; m < MS; ++m) {
        const int e = tid + m * NTP;
        if (e < L * NH) {
            const int p = e / NH, kx = e - (e / NH) * NH;
            const double2 Z = buf[p * N + kx];
            const double2 Zc = cconj(buf[p * N + (kx == 0 ? 0 : N - kx)]);
            const double2 sm = cadd(Z, Zc), d = csub(Z, Zc);
            za[m] = make_double2(0.5 * sm.x, 0.5 * sm.y);
            zb[m] = make_double2(0.5 * d.y, -0.5 * d.x);
        }
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < MS; ++m) {
        const int e = tid + m * NTP;
        if (e < L * NH) {
            const int p = e / NH, kx = e - (e / NH) * NH;
            buf[(2 * p) * NH + kx] = za[m];
            buf[(2 * p + 1) * NH + kx] = zb[m];
        }
    }
    __syncthreads();
    plane_y_fft<N>(buf, twy, tid);
    const int sh = D.sh;
    const gptr<double2> spec = (gptr<double2>)D.spec + (long long)k * N * sh;
    for (int e = tid; e < N * NH; e += NTP) {
        const int row = e / NH, kx = e - row * NH;
        gstore2(spec + row * sh + kx, buf[e]);
    }
}

template <int N>
__global__ __launch_bounds__(NTP) void k_ifftxy(Batch B)
{
    constexpr int NH = N / 2 + 1, L = N / 2, TX = fft_threads<N>();
    static_assert(L * TX <= NTP, "one pass of x transforms");
    __shared__ double2 buf[N * NH];
    __shared__ double2 twx[N], twy[N];
    const Desc& D = *B.d[blockIdx.y];
    const int tid = threadIdx.x, k = blockIdx.x;
    for (int n = tid; n < N; n += NTP) {
        twx[n] = gload2((gptr<const double2>)D.twx + n);
        twy[n] = gload2((gptr<const double2>)D.twy + n);
    }
    // inverse y transform by conjugation on the way in and out
    const int sh = D.sh;
    const gptr<const double2> spec = (gptr<const double2>)D.spec + (long long)k * N * sh;
    {
        constexpr int MS = (N * NH + NTP - 1) / NTP;
        double2 v[MS];
#pragma unroll
        for (int m = 0; m < MS; ++m) {
            const int e0 = tid + m * NTP, e = e0 < N * NH ? e0 : 0;
            const int row = e / NH, kx = e - row * NH;
            v[m] = gload2(spec + row * sh + kx);
        }
#pragma unroll
        for (int m = 0; m < MS; ++m) {
            const int e = tid + m * NTP;
            if (e < N * NH) buf[e] = cconj(v[m]);
        }
    }
    __syncthreads();
    plane_y_fft<N>(buf, twy, tid);
    // Hermitian extension of rows 2p and 2p + 1 into complex line p (a + i b)
    constexpr int ME = (L * N + NTP - 1) / NTP;
    double2 ze[ME];
#pragma unroll
    for (int m = 0; m < ME; ++m) {
        const int e = tid + m * NTP;
        if (e < L * N) {
            const int p = e / N, n = e - (e / N) * N;
            const int kx = n <= N / 2 ? n : N - n;
            double2 a = cconj(buf[(2 * p) * NH + kx]), b = cconj(buf[(2 * p + 1) * NH + kx]);
            if (n > N / 2) { a = cconj(a); b = cconj(b); }
            ze[m] = cconj(make_double2(a.x - b.y, a.y + b.x));
        }
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < ME; ++m) {
        const int e = tid + m * NTP;
        if (e < L * N) buf[e] = ze[m];
    }
    __syncthreads();
    {
        const int lp = tid / TX, t = tid - (tid / TX) * TX;
        fft_stages<N, TX, 0, 1>(buf + (lp < L ? lp : 0) * N, 1, t, lp < L, twx);
    }
    const gptr<double> p = (gptr<double>)D.p + (long long)k * N * N;
    for (int e = tid; e < L * N; e += NTP) {
        const int pr = e / N, n = e - (e / N) * N;
        const double2 z = cconj(buf[e]);
        p[(long long)(2 * pr) * N + n] = z.x;
        p[(long long)(2 * pr + 1) * N + n] = z.y;
    }
}

// ---------------------------------------------------------------------------------------------
// strided forward / inverse transform along y (axis 1) or z (axis 2), in place
// ---------------------------------------------------------------------------------------------
template <int N>
constexpr int strided_threads() { return fft_threads<N>() < NT / TK ? fft_threads<N>() : NT / TK; }

template <int N, bool INV>
__global__ __launch_bounds__(NT) void k_fft_strided(Batch B, int axis)
{
    constexpr int T = strided_threads<N>();
    __shared__ double2 buf[N * TK];
    __shared__ double2 tw[N];
    const Desc& D = *B.d[blockIdx.y];
    const int tid = threadIdx.x;
    const gptr<const double2> twg = (gptr<const double2>)(axis == 1 ? D.twy : D.twz);
    const gptr<double2> spec = (gptr<double2>)D.spec;
    for (int n = tid; n < N; n += NT) tw[n] = gload2(twg + n);
    const int nh = D.nh, sh = D.sh, ny = D.ny;
    const int ntk = (nh + TK - 1) / TK;
    const int tile = blockIdx.x % ntk, other = blockIdx.x / ntk;
    const int kx0 = tile * TK;
    long long base, es;
    if (axis == 1) { base = (long long)other * ny * sh + kx0; es = sh; }
    else { base = (long long)other * sh + kx0; es = (long long)sh * ny; }
    const bool colok = kx0 + tid % TK < nh;
    tile_in<N, INV>(buf, spec + base, es, colok, tid);
    __syncthreads();
    const int c = tid % TK, t = tid / TK;
    fft_stages<N, T, 0, 1>(buf + c, TK, t, t < T, tw);
    tile_out<N, INV>(buf, spec + base, es, colok, tid);
}

// ---------------------------------------------------------------------------------------------
// periodic: transform along z, divide by the Laplacian eigenvalue, transform back (in place)
// ---------------------------------------------------------------------------------------------
template <int N>
__global__ __launch_bounds__(NT) void k_solve_periodic(Batch B)
{
    constexpr int T = strided_threads<N>();
    __shared__ double2 buf[N * TK];
    __shared__ double2 tw[N];
    __shared__ double ez[N];        // Laplacian eigenvalues along z and of the block's kx columns
    __shared__ double ex[TK];
    const Desc& D = *B.d[blockIdx.y];
    const int tid = threadIdx.x;
    const gptr<const double> eigx = (gptr<const double>)D.eigx;
    const gptr<const double> eigz = (gptr<const double>)D.eigz;
    for (int n = tid; n < N; n += NT) {
        tw[n] = gload2((gptr<const double2>)D.twz + n);
        ez[n] = eigz[n];
    }
    const gptr<double2> spec = (gptr<double2>)D.spec;
    const int nh = D.nh, sh = D.sh, ny = D.ny;
    const int ntk = (nh + TK - 1) / TK;
    const int tile = blockIdx.x % ntk, ky = blockIdx.x / ntk;
    const int kx0 = tile * TK;
    if (tid < TK) ex[tid] = kx0 + tid < nh ? eigx[kx0 + tid] : 0.0;
    const long long base = (long long)ky * sh + kx0, es = (long long)sh * ny;
    const bool colok = kx0 + tid % TK < nh;
    tile_in<N, false>(buf, spec + base, es, colok, tid);
    __syncthreads();
    const int c = tid % TK, t = tid / TK;
    fft_stages<N, T, 0, 1>(buf + c, TK, t, t < T, tw);
    const double scale = 1.0 / ((double)D.nx * ny * N);
    const double ey = ((gptr<const double>)D.eigy)[ky];
    for (int e = tid; e < N * TK; e += NT) {
        const int kz = e / TK, cc = e - kz * TK;
        const int kx = kx0 + cc;
        double2 x = buf[e];
        if (kx < nh) {
            const double den = ex[cc] + ey + ez[kz];
            const double f = (kx == 0 && ky == 0 && kz == 0) ? 0.0 : scale / den;
            x = cscale(x, f);
        }
        buf[e] = cconj(x);        // inverse transform by conjugation
    }
    __syncthreads();
    fft_stages<N, T, 0, 1>(buf + c, TK, t, t < T, tw);
    tile_out<N, true>(buf, spec + base, es, colok, tid);
}

// ---------------------------------------------------------------------------------------------
// walls: tridiagonal solve in y for every (kx, kz), pivots precomputed per (kx, |kz|)
// ---------------------------------------------------------------------------------------------
constexpr int TH_NT = 64;   // one wave per block: modes are few, spread them over all CUs
// TH_P: rows loaded ahead of the dependent recurrence
template <int TH_P>
__global__ __launch_bounds__(TH_NT) void k_thomas(Batch B)
{
    const Desc& D = *B.d[blockIdx.y];
    const int nh = D.nh, sh = D.sh, ny = D.ny, nz = D.nz;
    // lanes run over the padded rows, so each wave's modes start on a 128-byte line
    const int col = blockIdx.x * TH_NT + threadIdx.x;
    const int kz = col / sh, kx = col - kz * sh;
    if (kz >= nz || kx >= nh) return;
    const int kzs = kz <= nz - kz ? kz : nz - kz;
    const gptr<const double> __restrict__ piv = (gptr<const double>)D.piv + (long long)kzs * ny * sh + kx;
    const gptr<double2> __restrict__ s = (gptr<double2>)D.spec + (long long)kz * ny * sh + kx;
    const double a = D.idy * D.idy;                  // sub- and super-diagonal 1/dy^2
    const double scale = 1.0 / ((double)D.nx * nz);  // inverse x and z transforms
    // From row jc on (up to row ny-2) the pivot recurrence of every mode of this wave has reached
    // its fixed point in floating point: those rows use the mode's pivot of row ny-2, loaded once,
    // instead of a load per row (the same numbers)
    const int jc = ((gptr<const int>)D.pvj)[blockIdx.x];
    const double pinf = ny >= 2 ? piv[(long long)(ny - 2) * sh] : 0.0;
    auto pivot = [&](int jj) {
        double pv = pinf;
        if (jj < jc || jj == ny - 1) pv = piv[(long long)jj * sh];
        return pv;
    };
    // forward sweep d'_j = (r_j - a d'_{j-1}) / (b_j - a c'_{j-1}); the loads of the next block
    // of TH_P rows are issued before the dependent updates of the current one
    double2 dp = make_double2(0.0, 0.0);
    double2 r[TH_P], rn[TH_P];
    double iv[TH_P], ivn[TH_P];
    auto fload = [&](int j0, double2* rr, double* ii) {
#pragma unroll
        for (int m = 0; m < TH_P; ++m) {
            const int jj = min(j0 + m, ny - 1);
            rr[m] = gload2(s + (long long)jj * sh);
            ii[m] = pivot(jj);
        }
    };
    fload(0, r, iv);
    for (int j0 = 0; j0 < ny; j0 += TH_P) {
        if (j0 + TH_P < ny) fload(j0 + TH_P, rn, ivn);
#pragma unroll
        for (int m = 0; m < TH_P; ++m) {
            if (j0 + m < ny) {
                dp = make_double2((scale * r[m].x - a * dp.x) * iv[m], (scale * r[m].y - a * dp.y) * iv[m]);
                gstore2(s + (long long)(j0 + m) * sh, dp);
            }
        }
#pragma unroll
        for (int m = 0; m < TH_P; ++m) { r[m] = rn[m]; iv[m] = ivn[m]; }
    }
    // backward sweep x_j = d'_j - c'_j x_{j+1}, c'_j = a / (b_j - a c'_{j-1}); the (0, 0) mode
    // also sums its profile for the zero-mean gauge
    double2 x = dp;
    double sum = dp.x;
    auto bload = [&](int j1, double2* dd, double* cc) {
#pragma unroll
        for (int m = 0; m < TH_P; ++m) {
            const int jj = max(j1 - m, 0);
            dd[m] = gload2(s + (long long)jj * sh);
            cc[m] = a * pivot(jj);
        }
    };
    if (ny >= 2) bload(ny - 2, r, iv);
    for (int j1 = ny - 2; j1 >= 0; j1 -= TH_P) {
        if (j1 - TH_P >= 0) bload(j1 - TH_P, rn, ivn);
#pragma unroll
        for (int m = 0; m < TH_P; ++m) {
            if (j1 - m >= 0) {
                x = make_double2(r[m].x - iv[m] * x.x, r[m].y - iv[m] * x.y);
                gstore2(s + (long long)(j1 - m) * sh, x);
                sum += x.x;
            }
        }
#pragma unroll
        for (int m = 0; m < TH_P; ++m) { r[m] = rn[m]; iv[m] = ivn[m]; }
    }
    // gauge: the volume mean of p is the mean over y of the (0, 0) mode (every other mode has zero
    // mean over x and z); the inverse x transform subtracts it from p
    if (kx == 0 && kz == 0) ((gptr<double>)D.gauge)[0] = sum / ny;
}

// Segmented form of the same solve for ny <= TS_L * TS_SEG: a block holds TS_M modes, and each
// group of TS_M lanes holds TS_L rows of them in registers (segment w of a block: rows
// [TS_L w, TS_L w + TS_L)), so the spectrum is read once and written once.  Both sweeps are
// first-order linear recurrences,
//   forward   d'_j = s r_j iv_j + g_j d'_{j-1},
//   backward  x_j  = d'_j + g_j x_{j+1}  (j <= ny-2; x_{ny-1} = d'_{ny-1}),  g_j = -a iv_j,
// with |g_j| <= 1 (diagonally dominant rows).  Each segment runs its rows with a zero
// value coming in and keeps the product of its coefficients; the segments' (product, last value)
// pairs go through LDS, each segment composes those of the segments before it (after it,
// backward) into its incoming value, and adds that value times the running product of its
// coefficients to its rows.  Mathematically the sequential sweep; the sums are associated
// differently.  At 512x256x256 this takes the solve from 208 to 96 us.  Blocks of 256 threads
// (16 modes) let three of them share a CU at the kernel's 166 registers; 32 modes (two per CU)
// took 114 us, 8 modes 99 us.
constexpr int TS_L = 16;     // rows per lane
constexpr int TS_M = 16;     // modes per block: 256 contiguous bytes of a row per segment
constexpr int TS_SEG = 16;   // segments per block at most: 256 threads, ny <= 256
constexpr int kRawWord3 = 0x00020000;   // raw-buffer format word of CDNA: 32-bit data, no swizzle
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(TS_M * TS_SEG) void k_thomas_seg(Batch B)
{
    __shared__ double fwd[3][TS_SEG][TS_M];    // forward: product, last d'.x, last d'.y
    __shared__ double bwd[3][TS_SEG][TS_M];    // backward: product, first x.x, first x.y
    __shared__ double gsum[TS_SEG];
    const Desc& D = *B.d[blockIdx.y];
    const int nh = D.nh, sh = D.sh, ny = D.ny, nz = D.nz;
    const int lane = threadIdx.x % TS_M, seg = threadIdx.x / TS_M, nseg = blockDim.x / TS_M;
    // modes run over the padded rows (a block's modes start on a 128-byte line); lanes past the
    // last mode take part in the barriers and load only in-bounds lines they discard
    const int col = blockIdx.x * TS_M + lane;
    const int kz = col / sh, kx = col - kz * sh;
    const bool live = kz < nz && kx < nh;
    const int kzc = live ? kz : 0;
    const int kzs = kzc <= nz - kzc ? kzc : nz - kzc;
    const double a = D.idy * D.idy;
    const double scale = 1.0 / ((double)D.nx * nz);
    // converged pivots from row jc on (up to row ny-2), as in k_thomas; jc is kept per 64 modes
    const int jc = ((gptr<const int>)D.pvj)[blockIdx.x * TS_M / 64];
    const int j0 = seg * TS_L;
    // raw buffer accesses: the lane's byte offset of its first row in one register, the row step
    // m sh as the wave-uniform offset (no per-row 64-bit addresses held for the stores)
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc((EVP_GLOBAL void*)D.spec, (short)0, 0x7fffffff, kRawWord3);
    const __amdgpu_buffer_rsrc_t rp = __builtin_amdgcn_make_buffer_rsrc((EVP_GLOBAL void*)D.piv, (short)0, 0x7fffffff, kRawWord3);
    const unsigned vs = (unsigned)((((long long)kzc * ny + j0) * sh + kx) * 16);
    const unsigned vp = (unsigned)((((long long)kzs * ny + j0) * sh + kx) * 8);
    // v: the right-hand side scaled by the row's pivot, then d', then x; g: -a iv_j.  All loads
    // are issued before any is used: a row past ny, a lane past the last mode and a converged
    // pivot read row m of the first mode instead (in bounds, the same few lines for the whole
    // grid) and discard it, so that no load sits behind a branch.
    double2 v[TS_L];
    double g[TS_L];
    {
        const unsigned plast = (unsigned)((((long long)kzs * ny + ny - 2) * sh + kx) * 8);
        const double pinf = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rp, live ? plast : 0u, 0, 0));
        dvec2 t[TS_L];
        double pl[TS_L];
#pragma unroll
        for (int m = 0; m < TS_L; ++m) {
            const int j = j0 + m;
            const bool in = live && j < ny;
            const bool need = in && (j < jc || j == ny - 1);
            t[m] = __builtin_bit_cast(dvec2, __builtin_amdgcn_raw_buffer_load_b128(rs, in ? vs : 0u, (unsigned)(m * sh * 16), 0));
            pl[m] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rp, need ? vp : 0u, (unsigned)(m * sh * 8), 0));
        }
#pragma unroll
        for (int m = 0; m < TS_L; ++m) {
            const int j = j0 + m;
            const bool in = live && j < ny;
            const double iv = in ? ((j < jc || j == ny - 1) ? pl[m] : pinf) : 0.0;
            v[m] = make_double2(scale * iv * t[m].x, scale * iv * t[m].y);
            g[m] = -a * iv;
        }
    }
    // forward sweep of the segment from a zero incoming value (rows past ny have iv = 0 and stay 0)
    {
        double2 dp = make_double2(0.0, 0.0);
        double pr = 1.0;
#pragma unroll
        for (int m = 0; m < TS_L; ++m) {
            dp = make_double2(v[m].x + g[m] * dp.x, v[m].y + g[m] * dp.y);
            v[m] = dp;
            pr *= g[m];
        }
        fwd[0][seg][lane] = pr;
        fwd[1][seg][lane] = dp.x;
        fwd[2][seg][lane] = dp.y;
    }
    __syncthreads();
    if (seg > 0) {
        double2 in = make_double2(0.0, 0.0);
#pragma unroll 2
        for (int q = 0; q < seg; ++q) {
            const double p = fwd[0][q][lane];
            in = make_double2(fwd[1][q][lane] + p * in.x, fwd[2][q][lane] + p * in.y);
        }
        double pr = 1.0;
#pragma unroll
        for (int m = 0; m < TS_L; ++m) {
            pr *= g[m];
            v[m] = make_double2(v[m].x + pr * in.x, v[m].y + pr * in.y);
        }
    }
    // backward sweep of the segment from a zero incoming value x_{j0 + TS_L}
    {
        double2 x = make_double2(0.0, 0.0);
        double pr = 1.0;
#pragma unroll
        for (int m = TS_L - 1; m >= 0; --m) {
            const double gb = j0 + m <= ny - 2 ? g[m] : 0.0;
            x = make_double2(v[m].x + gb * x.x, v[m].y + gb * x.y);
            v[m] = x;
            pr *= gb;
        }
        bwd[0][seg][lane] = pr;
        bwd[1][seg][lane] = x.x;
        bwd[2][seg][lane] = x.y;
    }
    __syncthreads();
    if (seg < nseg - 1) {
        double2 in = make_double2(0.0, 0.0);
#pragma unroll 2
        for (int q = nseg - 1; q > seg; --q) {
            const double p = bwd[0][q][lane];
            in = make_double2(bwd[1][q][lane] + p * in.x, bwd[2][q][lane] + p * in.y);
        }
        double pr = 1.0;
#pragma unroll
        for (int m = TS_L - 1; m >= 0; --m) {
            pr *= j0 + m <= ny - 2 ? g[m] : 0.0;
            v[m] = make_double2(v[m].x + pr * in.x, v[m].y + pr * in.y);
        }
    }
    double sum = 0.0;
#pragma unroll
    for (int m = 0; m < TS_L; ++m) {
        const int j = j0 + m;
        if (live && j < ny) {
            dvec2 t;
            t.x = v[m].x;
            t.y = v[m].y;
            __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, t), rs, vs, (unsigned)(m * sh * 16), 0);
            sum += v[m].x;
        }
    }
    // gauge from the (0, 0) mode (lane 0 of block 0): segment sums added in segment order
    if (blockIdx.x == 0) {
        if (lane == 0) gsum[seg] = sum;
        __syncthreads();
        if (threadIdx.x == 0) {
            double t = 0.0;
            for (int q = 0; q < nseg; ++q) t += gsum[q];
            ((gptr<double>)D.gauge)[0] = t / ny;
        }
    }
}

// ---------------------------------------------------------------------------------------------
// inverse x transform of two half spectra -> two real lines of p
// ---------------------------------------------------------------------------------------------
template <int N>
__global__ __launch_bounds__(NT) void k_ifftx(Batch B)
{
    constexpr int T = fft_threads<N>();
    constexpr int LP = NT / T;
    __shared__ double2 buf[LP * N];
    __shared__ double2 tw[N];
    const Desc& D = *B.d[blockIdx.y];
    const int tid = threadIdx.x;
    for (int n = tid; n < N; n += NT) tw[n] = gload2((gptr<const double2>)D.twx + n);
    const gptr<const double2> spec = (gptr<const double2>)D.spec;
    const gptr<double> p = (gptr<double>)D.p;
    const int nlines = D.ny * D.nz;
    const int npairs = (nlines + 1) >> 1;
    const int pair0 = blockIdx.x * LP;
    const int sh = D.sh;
    // Hermitian extension of two half spectra into one complex line; loads of eight elements are
    // issued before their LDS stores
    constexpr int M = (LP * N + NT - 1) / NT, G = M < 8 ? M : 8;
#pragma unroll
    for (int g0 = 0; g0 < M; g0 += G) {
        double2 av[G], bv[G];
#pragma unroll
        for (int m = 0; m < G; ++m) {
            const int e = tid + (g0 + m) * NT;
            const int ee = e < LP * N ? e : 0;
            const int lp = ee / N, n = ee - lp * N;
            const int pair = pair0 + lp;
            const int la = pair < npairs ? 2 * pair : 0;
            const int lb = (pair < npairs && la + 1 < nlines) ? la + 1 : la;
            const int k = n <= N / 2 ? n : N - n;
            av[m] = gload2(spec + (long long)la * sh + k);
            bv[m] = gload2(spec + (long long)lb * sh + k);
        }
#pragma unroll
        for (int m = 0; m < G; ++m) {
            const int e = tid + (g0 + m) * NT;
            if (e >= LP * N) continue;
            const int lp = e / N, n = e - lp * N;
            const int pair = pair0 + lp;
            double2 Z = make_double2(0.0, 0.0);
            if (pair < npairs) {
                double2 a = av[m];
                double2 b = (2 * pair + 1 < nlines) ? bv[m] : make_double2(0.0, 0.0);
                if (n > N / 2) { a = cconj(a); b = cconj(b); }
                Z = make_double2(a.x - b.y, a.y + b.x);   // a + i b
            }
            buf[e] = cconj(Z);
        }
    }
    __syncthreads();
    const int lp = tid / T, t = tid - (tid / T) * T;
    fft_stages<N, T, 0, 1>(buf + lp * N, 1, t, lp < LP, tw);
    // walls: zero-mean gauge (the mean of the Neumann solution, from the tridiagonal solve)
    const double pm = D.walls ? ((gptr<const double>)D.gauge)[0] : 0.0;
    for (int e = tid; e < LP * N; e += NT) {
        const int l2 = e / N, n = e - l2 * N;
        const int pair = pair0 + l2;
        if (pair >= npairs) continue;
        const double2 z = cconj(buf[e]);
        const int la = 2 * pair;
        p[(long long)la * N + n] = z.x - pm;
        if (la + 1 < nlines) p[(long long)(la + 1) * N + n] = z.y - pm;
    }
}

// ---------------------------------------------------------------------------------------------
// velocity correction u = u* - (dt/rho) G_h p; copies between u and u*
// ---------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_correct(Batch B)
{
    const Desc& D = *B.d[blockIdx.y];
    const int nx = D.nx, ny = D.ny, nz = D.nz;
    // consecutive blocks on one XCD (the hardware deals blocks round-robin over the eight XCDs),
    // so the rows j + 1 and the plane k + 1 whose p this block reads are read by blocks of the
    // same XCD's L2
    const int nb = gridDim.x;
    int bid = blockIdx.x;
    if ((nb & 7) == 0) bid = (bid & 7) * (nb >> 3) + (bid >> 3);
    const long long q = (long long)bid * 256 + threadIdx.x;
    if (q >= D.ncell) return;
    const int i = (int)(q % nx);
    const long long r = q / nx;
    const int j = (int)(r % ny), k = (int)(r / ny);
    const double c = B.dt[blockIdx.y] * D.inv_rho;
    const gptr<const double> p = (gptr<const double>)D.p;
    const gptr<const double> us = (gptr<const double>)D.us, vs = (gptr<const double>)D.vs,
                             ws = (gptr<const double>)D.ws;
    const gptr<double> u = (gptr<double>)D.u, v = (gptr<double>)D.v, w = (gptr<double>)D.w;
    const double p0 = p[q];
    const double px = p[q - i + (i + 1 == nx ? 0 : i + 1)];
    const long long sxy = (long long)nx * ny;
    const double pz = p[k + 1 == nz ? q - (long long)(nz - 1) * sxy : q + sxy];
    u[q] = us[q] - c * (px - p0) * D.idx;
    w[q] = ws[q] - c * (pz - p0) * D.idz;
    if (j + 1 == ny) {
        v[q] = D.walls ? 0.0 : vs[q] - c * (p[q - (long long)(ny - 1) * nx] - p0) * D.idy;
    } else {
        v[q] = vs[q] - c * (p[q + nx] - p0) * D.idy;
    }
}

__global__ __launch_bounds__(256) void k_copy_ustar(Batch B, int to_u)
{
    const Desc& D = *B.d[blockIdx.y];
    const long long ncell = D.ncell;
    const gptr<double> u = (gptr<double>)D.u, v = (gptr<double>)D.v, w = (gptr<double>)D.w;
    const gptr<double> us = (gptr<double>)D.us, vs = (gptr<double>)D.vs, ws = (gptr<double>)D.ws;
    const long long q = (long long)blockIdx.x * 256 + threadIdx.x;
    if (q >= ncell) return;
    if (to_u) {
        const double a = us[q], b = vs[q], c = ws[q];
        u[q] = a; v[q] = b; w[q] = c;
    } else {
        const double a = u[q], b = v[q], c = w[q];
        us[q] = a; vs[q] = b; ws[q] = c;
    }
}

}  // namespace

bool fft_size_supported(int n)
{
    switch (n) {
    case 8: case 12: case 16: case 24: case 32: case 48: case 64: case 96: case 128: case 192:
    case 256: case 384: case 512:
    case 10: case 20: case 30: case 40: case 60: case 80: case 120: case 160: case 240: case 320:
    case 480:
        return true;
    default:
        return false;
    }
}

#define EVP_FFT_SWITCH(n, CALL)                                                                  \
    switch (n) {                                                                                 \
    case 8: CALL(8); break;                                                                      \
    case 12: CALL(12); break;                                                                    \
    case 16: CALL(16); break;                                                                    \
    case 24: CALL(24); break;                                                                    \
    case 32: CALL(32); break;                                                                    \
    case 48: CALL(48); break;                                                                    \
    case 64: CALL(64); break;                                                                    \
    case 96: CALL(96); break;                                                                    \
    case 128: CALL(128); break;                                                                  \
    case 192: CALL(192); break;                                                                  \
    case 256: CALL(256); break;                                                                  \
    case 384: CALL(384); break;                                                                  \
    case 512: CALL(512); break;                                                                  \
    case 10: CALL(10); break;                                                                    \
    case 20: CALL(20); break;                                                                    \
    case 30: CALL(30); break;                                                                    \
    case 40: CALL(40); break;                                                                    \
    case 60: CALL(60); break;                                                                    \
    case 80: CALL(80); break;                                                                    \
    case 120: CALL(120); break;                                                                  \
    case 160: CALL(160); break;                                                                  \
    case 240: CALL(240); break;                                                                  \
    case 320: CALL(320); break;                                                                  \
    case 480: CALL(480); break;                                                                  \
    default: return hipErrorInvalidValue;                                                        \
    }

hipError_t launch_div_fftx(const Batch& b, int nx, int ny, int nz, hipStream_t s)
{
    const int npairs = (ny * nz + 1) / 2;
#define CALL(N)                                                                                  \
    {                                                                                            \
        constexpr int LP = NT / fft_threads<N>();                                                \
        dim3 grid((npairs + LP - 1) / LP, b.count);                                              \
        hipLaunchKernelGGL(k_div_fftx<N>, grid, dim3(NT), 0, s, b);                              \
    }
    EVP_FFT_SWITCH(nx, CALL)
#undef CALL
    return hipGetLastError();
}

hipError_t launch_ifftx(const Batch& b, int nx, int ny, int nz, hipStream_t s)
{
    const int npairs = (ny * nz + 1) / 2;
#define CALL(N)                                                                                  \
    {                                                                                            \
        constexpr int LP = NT / fft_threads<N>();                                                \
        dim3 grid((npairs + LP - 1) / LP, b.count);                                              \
        hipLaunchKernelGGL(k_ifftx<N>, grid, dim3(NT), 0, s, b);                                 \
    }
    EVP_FFT_SWITCH(nx, CALL)
#undef CALL
    return hipGetLastError();
}

bool plane_transforms(int nx, int ny, int nz, int count)
{
    // one block per z plane and at most one per CU at 128^2: with fewer planes than the chip's 256
    // CUs the separate line-transform passes are as fast (measured on one 128^3 grid); with at
    // least that many, the fused passes save 2-11 % of the step (batches of 32^3 to 128^3 grids)
    const bool size = nx == ny && (nx == 16 || nx == 24 || nx == 32 || nx == 48 || nx == 64 ||
                                   nx == 96 || nx == 128);
    return size && (long long)nz * count >= 256;
}

hipError_t launch_div_fftxy(const Batch& b, int n, int nz, hipStream_t s)
{
    dim3 grid(nz, b.count);
    switch (n) {
#define CALL(N) case N: hipLaunchKernelGGL(k_div_fftxy<N>, grid, dim3(NTP), 0, s, b); break;
    CALL(16) CALL(24) CALL(32) CALL(48) CALL(64) CALL(96) CALL(128)
#undef CALL
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_ifftxy(const Batch& b, int n, int nz, hipStream_t s)
{
    dim3 grid(nz, b.count);
    switch (n) {
#define CALL(N) case N: hipLaunchKernelGGL(k_ifftxy<N>, grid, dim3(NTP), 0, s, b); break;
    CALL(16) CALL(24) CALL(32) CALL(48) CALL(64) CALL(96) CALL(128)
#undef CALL
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_fft_strided(const Batch& b, int nx, int ny, int nz, int axis, bool inverse,
                              hipStream_t s)
{
    const int nh = nx / 2 + 1;
    const int ntk = (nh + TK - 1) / TK;
    const int n = axis == 1 ? ny : nz;
    const int other = axis == 1 ? nz : ny;
    dim3 grid(ntk * other, b.count);
#define CALL(N)                                                                                  \
    {                                                                                            \
        if (inverse) hipLaunchKernelGGL((k_fft_strided<N, true>), grid, dim3(NT), 0, s, b, axis); \
        else hipLaunchKernelGGL((k_fft_strided<N, false>), grid, dim3(NT), 0, s, b, axis);       \
    }
    EVP_FFT_SWITCH(n, CALL)
#undef CALL
    return hipGetLastError();
}

hipError_t launch_solve_periodic(const Batch& b, int nx, int ny, int nz, hipStream_t s)
{
    const int nh = nx / 2 + 1;
    const int ntk = (nh + TK - 1) / TK;
    dim3 grid(ntk * ny, b.count);
#define CALL(N) hipLaunchKernelGGL(k_solve_periodic<N>, grid, dim3(NT), 0, s, b);
    EVP_FFT_SWITCH(nz, CALL)
#undef CALL
    return hipGetLastError();
}

hipError_t launch_thomas(const Batch& b, int nx, int ny, int nz, hipStream_t s)
{
    const int cols = (int)((nx / 2 + 1 + 7) / 8 * 8) * nz;   // padded rows (Desc::sh)
    if (ny <= TS_L * TS_SEG) {
        // TS_M lanes per TS_L rows of TS_M modes
        const int nseg = (ny + TS_L - 1) / TS_L;
        dim3 grid((cols + TS_M - 1) / TS_M, b.count);
        hipLaunchKernelGGL(k_thomas_seg, grid, dim3(TS_M * nseg), 0, s, b);
    } else {
        dim3 grid((cols + TH_NT - 1) / TH_NT, b.count);
        // 16 rows ahead (248 VGPRs, two waves per SIMD): measured best against 8 and 32
        hipLaunchKernelGGL(k_thomas<16>, grid, dim3(TH_NT), 0, s, b);
    }
    return hipGetLastError();
}

hipError_t launch_correct(const Batch& b, int nx, int ny, int nz, hipStream_t s)
{
    const long long n = (long long)nx * ny * nz;
    dim3 grid((unsigned)((n + 255) / 256), b.count);
    hipLaunchKernelGGL(k_correct, grid, dim3(256), 0, s, b);
    return hipGetLastError();
}

hipError_t launch_copy_ustar(const Batch& b, int nx, int ny, int nz, bool to_u, hipStream_t s)
{
    const long long n = (long long)nx * ny * nz;
    dim3 grid((unsigned)((n + 255) / 256), b.count);
    hipLaunchKernelGGL(k_copy_ustar, grid, dim3(256), 0, s, b, to_u ? 1 : 0);
    return hipGetLastError();
}

}  // namespace evp
