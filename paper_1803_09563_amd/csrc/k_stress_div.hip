// Stress divergence at the new Runge-Kutta level (Sec. 3.3.1, Eq. NS-num1): once the substep's
// stress update has produced B^k everywhere, u* += dt (alpha / rho) div tau(B^k) on every face.
// Same face stencils as the momentum part of the predictor: tau_aa differenced across the face,
// the off-diagonal components averaged over the four cells around the face and differenced
// across it; wall ghost rows of B extrapolated linearly, no update on the top wall v-face.
#include "evp_internal.h"

namespace evp {

namespace {

constexpr int SD_NT = 256;

template <typename T, bool WALLS>
__global__ __launch_bounds__(SD_NT) void k_stress_div(Batch B)
{
    const int b = blockIdx.y;
    const Desc& D = *B.d[b];
    const int nx = D.nx, ny = D.ny, nz = D.nz;
    const long long ncell = D.ncell;
    const long long cell = (long long)blockIdx.x * SD_NT + threadIdx.x;
    if (cell >= ncell) return;
    const int i = (int)(cell % nx), j = (int)((cell / nx) % ny), k = (int)(cell / ((long long)nx * ny));
    const long long ps = D.ps, sxy = (long long)nx * ny;
    const T* __restrict__ Bk = (const T*)D.Bt[(B.state[b] & 1) ^ 1];
    const bool fene = D.model == EVP_FENE_P;
    const T G = (T)D.G, L2 = (T)D.L2, afene = (T)D.a_fene;
    const T idx = (T)D.idx, idy = (T)D.idy, idz = (T)D.idz, qt = (T)0.25;

    const int ip = i + 1 == nx ? 0 : i + 1, im = i == 0 ? nx - 1 : i - 1;
    const int kp = k + 1 == nz ? 0 : k + 1, km = k == 0 ? nz - 1 : k - 1;

    // tau_cc of cell (ii, jj, kk); jj in -1..ny (walls: ghost rows) or wrapped (periodic)
    auto tau = [&](int cc, int ii, int jj, int kk) -> T {
        long long oa, ob = 0;
        T wa = (T)1, wb = (T)0;
        const long long base = kk * sxy + ii;
        if (WALLS && jj < 0) { oa = base; ob = base + nx; wa = (T)2; wb = (T)-1; }
        else if (WALLS && jj >= ny) { oa = base + (long long)(ny - 1) * nx; ob = oa - nx; wa = (T)2; wb = (T)-1; }
        else {
            const int jw = WALLS ? jj : (jj < 0 ? jj + ny : (jj >= ny ? jj - ny : jj));
            oa = base + (long long)jw * nx;
        }
        auto bv = [&](int c) {
            T x = Bk[c * ps + oa];
            if (WALLS && wb != (T)0) x = wa * x + wb * Bk[c * ps + ob];
            return x;
        };
        const T x = bv(cc);
        if (!fene) return G * x;
        const T F = L2 / (L2 - (bv(0) + bv(3) + bv(5) + (T)3));
        return G * F * x + ((cc == 0 || cc == 3 || cc == 5) ? G * (F - afene) : (T)0);
    };

    const T c = (T)(B.dt[b] * B.rk[2] * D.inv_rho);
    const long long q = cell;
    // x-face (i+1/2, j, k)
    {
        const T d = (tau(0, ip, j, k) - tau(0, i, j, k)) * idx
                  + qt * (tau(1, i, j + 1, k) + tau(1, ip, j + 1, k) - tau(1, i, j - 1, k) - tau(1, ip, j - 1, k)) * idy
                  + qt * (tau(2, i, j, kp) + tau(2, ip, j, kp) - tau(2, i, j, km) - tau(2, ip, j, km)) * idz;
        D.us[q] += (double)(c * d);
    }
    // y-face (i, j+1/2, k); the top wall face stays 0
    if (!(WALLS && j == ny - 1)) {
        const T d = qt * (tau(1, ip, j, k) + tau(1, ip, j + 1, k) - tau(1, im, j, k) - tau(1, im, j + 1, k)) * idx
                  + (tau(3, i, j + 1, k) - tau(3, i, j, k)) * idy
                  + qt * (tau(4, i, j, kp) + tau(4, i, j + 1, kp) - tau(4, i, j, km) - tau(4, i, j + 1, km)) * idz;
        D.vs[q] += (double)(c * d);
    }
    // z-face (i, j, k+1/2)
    {
        const T d = qt * (tau(2, ip, j, k) + tau(2, ip, j, kp) - tau(2, im, j, k) - tau(2, im, j, kp)) * idx
                  + qt * (tau(4, i, j + 1, k) + tau(4, i, j + 1, kp) - tau(4, i, j - 1, k) - tau(4, i, j - 1, kp)) * idy
                  + (tau(5, i, j, kp) - tau(5, i, j, k)) * idz;
        D.ws[q] += (double)(c * d);
    }
}

}  // namespace

hipError_t launch_stress_div(const Batch& b, int precision, int nx, int ny, int nz, bool walls,
                             hipStream_t s)
{
    const long long ncell = (long long)nx * ny * nz;
    dim3 grid((unsigned)((ncell + SD_NT - 1) / SD_NT), b.count);
    if (precision == EVP_MIXED) {
        if (walls) hipLaunchKernelGGL((k_stress_div<float, true>), grid, dim3(SD_NT), 0, s, b);
        else hipLaunchKernelGGL((k_stress_div<float, false>), grid, dim3(SD_NT), 0, s, b);
    } else {
        if (walls) hipLaunchKernelGGL((k_stress_div<double, true>), grid, dim3(SD_NT), 0, s, b);
        else hipLaunchKernelGGL((k_stress_div<double, false>), grid, dim3(SD_NT), 0, s, b);
    }
    return hipGetLastError();
}

}  // namespace evp
