// Stress divergence at the new Runge-Kutta level (Sec. 3.3.1, Eq. NS-num1): once the substep's
// stress update has produced B^k everywhere, u* += dt (alpha / rho) div tau(B^k) on every face.
// Same face stencils as the momentum part of the predictor: tau_aa differenced across the face,
// the off-diagonal components averaged over the four cells around the face and differenced
// across it; wall ghost rows of B extrapolated linearly, no update on the top wall v-face.  With
// a solid (Sec. 3.3.2), the completed prediction is then penalised: u** = (1 - alpha) u*.
//
// Layout: a block of 32 x 8 threads owns a 32 x 8 column of cells and marches along z over a
// chunk of planes.  tau (six components, from B - I and the closure) of planes k-1, k, k+1 on the
// tile plus a 1-cell ring sits in a three-slot LDS ring, so each B value is read and converted
// once per block; block ids are remapped so consecutive tiles share an XCD.
#include <cstdlib>

#include "evp_internal.h"

namespace evp {

namespace {

constexpr int SX = 32, SY = 8, SN = SX * SY;
constexpr int HW = SX + 2, HH = SY + 2, HB = HW * HH;
constexpr int NHALO = 2 * HW + 2 * SY;      // ring cells of the 34 x 10 box

__device__ __forceinline__ int wrap(int i, int n)
{
    int r = i % n;
    return r < 0 ? r + n : r;
}

template <typename T, bool WALLS>
__global__ __launch_bounds__(SN) void k_stress_div(Batch B, int kc)
{
    __shared__ T S[3][6][HB];
    const int b = blockIdx.y;
    const Desc& D = *B.d[b];
    const int nx = D.nx, ny = D.ny, nz = D.nz;
    const long long sxy = (long long)nx * ny, ps = D.ps;
    const int ntx = (nx + SX - 1) / SX, nty = (ny + SY - 1) / SY, nch = (nz + kc - 1) / kc;
    const int nblk = ntx * nty * nch;
    int bid = blockIdx.x;
    if ((nblk & 7) == 0) bid = (bid & 7) * (nblk >> 3) + (bid >> 3);     // XCD-contiguous tiles
    const int tile_x = bid % ntx, tile_y = (bid / ntx) % nty, ch = bid / (ntx * nty);
    const int i0 = tile_x * SX, j0 = tile_y * SY, k0 = ch * kc, k1 = min(k0 + kc, nz);
    const int t = threadIdx.x, tx = t % SX, ty = t / SX;
    const int i = i0 + tx, j = j0 + ty;
    const bool valid = i < nx && j < ny;

    const gptr<const T> __restrict__ Bk = (gptr<const T>)D.Bt[(B.state[b] & 1) ^ 1];
    const gptr<double> __restrict__ us = (gptr<double>)D.us;
    const gptr<double> __restrict__ vs = (gptr<double>)D.vs;
    const gptr<double> __restrict__ ws = (gptr<double>)D.ws;
    const bool fene = D.model == EVP_FENE_P;
    const T G = (T)D.G, L2 = (T)D.L2, afene = (T)D.a_fene;
    const T idx = (T)D.idx, idy = (T)D.idy, idz = (T)D.idz, qt = (T)0.25;
    const T c = (T)(B.dt[b] * B.rk[2] * D.inv_rho);
    const bool solid = D.alpha[0] != nullptr;

    // source of a box cell (ii, jj): value = wa B[oa] + wb B[ob] (plane-relative offsets)
    struct Src { long long oa, ob; T wa, wb; };
    auto src = [&](int ii, int jj) {
        Src q;
        ii = wrap(ii, nx);
        q.wa = (T)1; q.wb = (T)0;
        if (!WALLS) { q.oa = (long long)wrap(jj, ny) * nx + ii; q.ob = q.oa; return q; }
        if (jj < 0) { const T g = (T)(-jj); q.oa = ii; q.ob = nx + ii; q.wa = (T)1 + g; q.wb = -g; return q; }
        if (jj >= ny) {
            const T g = (T)(jj - ny + 1);
            q.oa = (long long)(ny - 1) * nx + ii; q.ob = q.oa - nx; q.wa = (T)1 + g; q.wb = -g; return q;
        }
        q.oa = (long long)jj * nx + ii; q.ob = q.oa; return q;
    };
    // this thread's box slots: its own cell, and one ring cell for t < NHALO
    const int own = (ty + 1) * HW + (tx + 1);
    const Src os = src(i, j);
    int hl = -1;
    Src hs{0, 0, (T)1, (T)0};
    if (t < NHALO) {
        int r, cc;
        if (t < 2 * HW) { r = t < HW ? 0 : SY + 1; cc = t % HW; }
        else { const int u = t - 2 * HW; r = 1 + u / 2; cc = (u & 1) ? SX + 1 : 0; }
        hl = r * HW + cc;
        hs = src(i0 + cc - 1, j0 + r - 1);
    }

    // tau of plane kk (own cell and ring cell) into ring slot sl
    auto tau6 = [&](gptr<const T> pl, const Src& q, T (&o)[6]) {
        T x[6];
#pragma unroll
        for (int cc = 0; cc < 6; ++cc) {
            x[cc] = pl[cc * ps + q.oa];
            if (WALLS) x[cc] = q.wa * x[cc] + q.wb * pl[cc * ps + q.ob];
        }
        if (fene) {
            const T F = L2 / (L2 - (x[0] + x[3] + x[5] + (T)3));
            const T gf = G * F, ga = G * (F - afene);
#pragma unroll
            for (int cc = 0; cc < 6; ++cc) o[cc] = gf * x[cc] + ((cc == 0 || cc == 3 || cc == 5) ? ga : (T)0);
        } else {
#pragma unroll
            for (int cc = 0; cc < 6; ++cc) o[cc] = G * x[cc];
        }
    };
    auto load = [&](int kk, int sl) {
        const gptr<const T> pl = Bk + (long long)wrap(kk, nz) * sxy;
        T a[6], h[6];
        tau6(pl, os, a);
        if (hl >= 0) tau6(pl, hs, h);
#pragma unroll
        for (int cc = 0; cc < 6; ++cc) {
            S[sl][cc][own] = a[cc];
            if (hl >= 0) S[sl][cc][hl] = h[cc];
        }
    };

    load(k0 - 1, (k0 + 2) % 3);
    load(k0, k0 % 3);
    const bool vwall = WALLS && j == ny - 1;
    for (int k = k0; k < k1; ++k) {
        const long long q = (long long)k * sxy + (long long)j * nx + i;
        double uo = 0.0, vo = 0.0, wo = 0.0;
        double pen[3] = {1.0, 1.0, 1.0};         // 1 - alpha of the solid fractions, if any
        if (valid) {
            // u* is read and written once, by this cell: non-temporal, so L2 keeps the B halos
            uo = __builtin_nontemporal_load(us + q); vo = __builtin_nontemporal_load(vs + q);
            wo = __builtin_nontemporal_load(ws + q);
            if (solid)
                for (int m = 0; m < 3; ++m) pen[m] = 1.0 - ((gptr<const double>)D.alpha[m])[q];
        }
        load(k + 1, (k + 1) % 3);
        __syncthreads();
        if (valid) {
            const T* P0 = &S[k % 3][0][0];
            const T* Pm = &S[(k + 2) % 3][0][0];
            const T* Pp = &S[(k + 1) % 3][0][0];
#define TA(P, cc, di, dj) (P)[(cc) * HB + own + (dj) * HW + (di)]
            // x-face (i+1/2, j, k)
            const T dx_ = (TA(P0, 0, 1, 0) - TA(P0, 0, 0, 0)) * idx
                        + qt * (TA(P0, 1, 0, 1) + TA(P0, 1, 1, 1) - TA(P0, 1, 0, -1) - TA(P0, 1, 1, -1)) * idy
                        + qt * (TA(Pp, 2, 0, 0) + TA(Pp, 2, 1, 0) - TA(Pm, 2, 0, 0) - TA(Pm, 2, 1, 0)) * idz;
            __builtin_nontemporal_store((uo + (double)(c * dx_)) * pen[0], us + q);
            // y-face (i, j+1/2, k); the top wall face stays 0
            if (!vwall) {
                const T dy_ = qt * (TA(P0, 1, 1, 0) + TA(P0, 1, 1, 1) - TA(P0, 1, -1, 0) - TA(P0, 1, -1, 1)) * idx
                            + (TA(P0, 3, 0, 1) - TA(P0, 3, 0, 0)) * idy
                            + qt * (TA(Pp, 4, 0, 0) + TA(Pp, 4, 0, 1) - TA(Pm, 4, 0, 0) - TA(Pm, 4, 0, 1)) * idz;
                __builtin_nontemporal_store((vo + (double)(c * dy_)) * pen[1], vs + q);
            }
            // z-face (i, j, k+1/2)
            const T dz_ = qt * (TA(P0, 2, 1, 0) + TA(Pp, 2, 1, 0) - TA(P0, 2, -1, 0) - TA(Pp, 2, -1, 0)) * idx
                        + qt * (TA(P0, 4, 0, 1) + TA(Pp, 4, 0, 1) - TA(P0, 4, 0, -1) - TA(Pp, 4, 0, -1)) * idy
                        + (TA(Pp, 5, 0, 0) - TA(P0, 5, 0, 0)) * idz;
            __builtin_nontemporal_store((wo + (double)(c * dz_)) * pen[2], ws + q);
#undef TA
        }
        __syncthreads();
    }
}

// Volume-penalisation immersed boundary for the AB2 step (Sec. 3.3.2, Eq. forceAdded):
// u** = (1 - alpha) u* on every face of the grids in the batch that have a solid.  (Under RK3 the
// same product is fused into k_stress_div.)  A pass of its own so that the predictor's register
// allocation is not shared with it.
__global__ __launch_bounds__(256) void k_penalise(Batch B)
{
    const Desc& D = *B.d[blockIdx.y];
    if (D.alpha[0] == nullptr) return;
    const long long q = (long long)blockIdx.x * 256 + threadIdx.x;
    if (q >= D.ncell) return;
    const gptr<double> us = (gptr<double>)D.us, vs = (gptr<double>)D.vs, ws = (gptr<double>)D.ws;
    const gptr<const double> au = (gptr<const double>)D.alpha[0], av = (gptr<const double>)D.alpha[1],
                             aw = (gptr<const double>)D.alpha[2];
    const double x = us[q], y = vs[q], z = ws[q], a = au[q], b = av[q], c = aw[q];
    us[q] = x * (1.0 - a);
    vs[q] = y * (1.0 - b);
    ws[q] = z * (1.0 - c);
}

}  // namespace

hipError_t launch_penalise(const Batch& b, int nx, int ny, int nz, hipStream_t s)
{
    const long long ncell = (long long)nx * ny * nz;
    dim3 grid((unsigned)((ncell + 255) / 256), b.count);
    hipLaunchKernelGGL(k_penalise, grid, dim3(256), 0, s, b);
    return hipGetLastError();
}

hipError_t launch_stress_div(const Batch& b, int precision, int nx, int ny, int nz, bool walls,
                             hipStream_t s)
{
    // z chunks: about 512 blocks in all (two per CU), at least two planes per block
    static const int target = [] {
        const char* e = std::getenv("EVP_SD_BLOCKS");
        const int v = e ? std::atoi(e) : 0;
        return v > 0 ? v : 512;
    }();
    const int tiles = ((nx + SX - 1) / SX) * ((ny + SY - 1) / SY);
    int nch = (target + tiles - 1) / tiles;
    nch = max(1, min(nch, nz / 2));
    const int kc = (nz + nch - 1) / nch;
    const int nblk = ((nx + SX - 1) / SX) * ((ny + SY - 1) / SY) * ((nz + kc - 1) / kc);
    dim3 grid(nblk, b.count);
    if (precision == EVP_MIXED) {
        if (walls) hipLaunchKernelGGL((k_stress_div<float, true>), grid, dim3(SN), 0, s, b, kc);
        else hipLaunchKernelGGL((k_stress_div<float, false>), grid, dim3(SN), 0, s, b, kc);
    } else {
        if (walls) hipLaunchKernelGGL((k_stress_div<double, true>), grid, dim3(SN), 0, s, b, kc);
        else hipLaunchKernelGGL((k_stress_div<double, false>), grid, dim3(SN), 0, s, b, kc);
    }
    return hipGetLastError();
}

}  // namespace evp
