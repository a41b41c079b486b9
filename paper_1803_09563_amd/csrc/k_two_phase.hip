// Two-phase (bubbly-flow) path of Sec. 3.2, FP64, one thread per cell:
//   * level-set transport, Eq. (ls adv): one stage of the three-stage TVD Runge-Kutta scheme per
//     launch, fifth-order WENO upwinded on the cell-centre velocity;
//   * reinitialisation, Eq. (reinit): the same stages with the Godunov form of |grad phi| on the
//     one-sided WENO derivatives and the mollified sign of phi before reinitialisation;
//   * curvature kappa = -div(grad phi / |grad phi|) at cell centres (central differences);
//   * momentum, Eq. (ru), with the mixture properties of Eq. (mat prop) taken from phi^{n+1}:
//     div(mu_s (grad u + grad u^T)), div tau with a per-cell modulus G = mu_p / lambda, the
//     surface-tension force sigma kappa delta(phi) n of Eq. (fLS) formed as sigma kappa grad H,
//     1/rho on the faces, AB2 in time;
//   * the pressure splitting of Eq. (poisson LS): 2 p^n - p^{n-1} and the split velocity update
//     u* -= dt (1/rho - 1/rho_0) grad(2 p^n - p^{n-1}), after which the constant-coefficient
//     projection with rho_0 yields p^{n+1} and u^{n+1} exactly as the split Poisson equation.
// Level-set ghost rows beyond a wall are linear extrapolations of the two nearest rows (as for
// B); material properties of ghost rows copy the adjacent interior row.
#include "evp_internal.h"
#include "weno.h"

namespace evp {

namespace {

constexpr int NT2 = 256;

__device__ __forceinline__ int wrap2(int i, int n)
{
    int r = i % n;
    return r < 0 ? r + n : r;
}

// cell index helpers bound to one grid
struct Cells {
    int nx, ny, nz;
    bool walls;
    __device__ long long at(int i, int j, int k) const { return ((long long)k * ny + j) * nx + i; }
    // level-set / B style access: periodic x, z; y periodic or linear extrapolation past walls
    __device__ double ext(gptr<const double> f, int i, int j, int k) const
    {
        i = wrap2(i, nx); k = wrap2(k, nz);
        if (!walls) return f[at(i, wrap2(j, ny), k)];
        if (j < 0) { const double g = -j; return (1.0 + g) * f[at(i, 0, k)] - g * f[at(i, 1, k)]; }
        if (j >= ny) { const double g = j - ny + 1; return (1.0 + g) * f[at(i, ny - 1, k)] - g * f[at(i, ny - 2, k)]; }
        return f[at(i, j, k)];
    }
    // property access: ghost rows copy the nearest interior row
    __device__ double clamp(gptr<const double> f, int i, int j, int k) const
    {
        i = wrap2(i, nx); k = wrap2(k, nz);
        j = walls ? (j < 0 ? 0 : (j >= ny ? ny - 1 : j)) : wrap2(j, ny);
        return f[at(i, j, k)];
    }
};

// ---------------------------------------------------------------------------------------------
// level-set transport / reinitialisation stage
// ---------------------------------------------------------------------------------------------
template <bool WALLS>
__global__ __launch_bounds__(NT2) void k_level_set_stage(Batch B, int reinit, int stage)
{
    const int b = blockIdx.y;
    const Desc& D = *B.d[b];
    if (reinit && !(B.state[b] & ST_REINIT)) return;
    const Cells C{D.nx, D.ny, D.nz, WALLS};
    const long long q = (long long)blockIdx.x * NT2 + threadIdx.x;
    if (q >= D.ncell) return;
    const int i = (int)(q % C.nx), j = (int)((q / C.nx) % C.ny), k = (int)(q / ((long long)C.nx * C.ny));
    // stages of the TVD scheme: out = a base + c (src + dt L(src)), base = phi
    const gptr<const double> base = (gptr<const double>)D.phi;
    gptr<const double> src;
    gptr<double> out;
    double a, c;
    if (stage == 0) { src = (gptr<const double>)D.phi; out = (gptr<double>)D.phi1; a = 0.0; c = 1.0; }
    else if (stage == 1) { src = (gptr<const double>)D.phi1; out = (gptr<double>)D.phi2; a = 0.75; c = 0.25; }
    else { src = (gptr<const double>)D.phi2; out = (gptr<double>)D.phi; a = 1.0 / 3.0; c = 2.0 / 3.0; }
    const double hs[3] = {D.dx, D.dy, D.dz};
    double dm[3], dp[3];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        double f[7];
#pragma unroll
        for (int m = 0; m < 7; ++m)
            f[m] = C.ext(src, i + (ax == 0 ? m - 3 : 0), j + (ax == 1 ? m - 3 : 0), k + (ax == 2 ? m - 3 : 0));
        const double e2 = 1e-6 * hs[ax] * hs[ax], ih = 1.0 / hs[ax];
        dm[ax] = weno5u<double>(f[1] - f[0], f[2] - f[1], f[3] - f[2], f[4] - f[3], f[5] - f[4], e2) * ih;
        dp[ax] = weno5u<double>(f[6] - f[5], f[5] - f[4], f[4] - f[3], f[3] - f[2], f[2] - f[1], e2) * ih;
    }
    double L, dt;
    if (!reinit) {
        const gptr<const double> u = (gptr<const double>)D.u, v = (gptr<const double>)D.v,
                                 w = (gptr<const double>)D.w;
        const double uc = 0.5 * (u[q] + u[C.at(wrap2(i - 1, C.nx), j, k)]);
        const double vm = (WALLS && j == 0) ? 0.0 : v[C.at(i, wrap2(j - 1, C.ny), k)];
        const double vc = 0.5 * (v[q] + vm);
        const double wc = 0.5 * (w[q] + w[C.at(i, j, wrap2(k - 1, C.nz))]);
        const double vel[3] = {uc, vc, wc};
        L = 0.0;
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) L -= vel[ax] * (vel[ax] >= 0.0 ? dm[ax] : dp[ax]);
        dt = B.dt[b];
    } else {
        const double S = ((gptr<const double>)D.sgn)[q];
        double g2 = 0.0;
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            const double am = dm[ax], bp = dp[ax];
            const double pos = fmax(fmax(am, 0.0) * fmax(am, 0.0), fmin(bp, 0.0) * fmin(bp, 0.0));
            const double neg = fmax(fmin(am, 0.0) * fmin(am, 0.0), fmax(bp, 0.0) * fmax(bp, 0.0));
            g2 += S >= 0.0 ? pos : neg;
        }
        L = -S * (sqrt(g2) - 1.0);
        dt = 0.5 * fmin(fmin(D.dx, D.dy), D.dz);
    }
    const double r = src[q] + dt * L;
    out[q] = a == 0.0 ? c * r : a * base[q] + c * r;
}

// mollified sign of the level set before reinitialisation: phi / sqrt(phi^2 + h^2)
__global__ __launch_bounds__(NT2) void k_reinit_sign(Batch B)
{
    const int b = blockIdx.y;
    const Desc& D = *B.d[b];
    if (!(B.state[b] & ST_REINIT)) return;
    const long long q = (long long)blockIdx.x * NT2 + threadIdx.x;
    if (q >= D.ncell) return;
    const double h = fmin(fmin(D.dx, D.dy), D.dz);
    const double p = ((gptr<const double>)D.phi)[q];
    ((gptr<double>)D.sgn)[q] = p / sqrt(p * p + h * h);
}

// ---------------------------------------------------------------------------------------------
// curvature at cell centres
// ---------------------------------------------------------------------------------------------
template <bool WALLS>
__global__ __launch_bounds__(NT2) void k_curvature(Batch B)
{
    const Desc& D = *B.d[blockIdx.y];
    const Cells C{D.nx, D.ny, D.nz, WALLS};
    const long long q = (long long)blockIdx.x * NT2 + threadIdx.x;
    if (q >= D.ncell) return;
    const int i = (int)(q % C.nx), j = (int)((q / C.nx) % C.ny), k = (int)(q / ((long long)C.nx * C.ny));
    const gptr<const double> phi = (gptr<const double>)D.phi;
    const double ix2 = 0.5 / D.dx, iy2 = 0.5 / D.dy, iz2 = 0.5 / D.dz;
    // unit normal component `ax` at cell (ii, jj, kk) from central differences
    auto normal = [&](int ii, int jj, int kk, int ax) {
        const double gx = (C.ext(phi, ii + 1, jj, kk) - C.ext(phi, ii - 1, jj, kk)) * ix2;
        const double gy = (C.ext(phi, ii, jj + 1, kk) - C.ext(phi, ii, jj - 1, kk)) * iy2;
        const double gz = (C.ext(phi, ii, jj, kk + 1) - C.ext(phi, ii, jj, kk - 1)) * iz2;
        const double mag = fmax(sqrt(gx * gx + gy * gy + gz * gz), 1e-12);
        return (ax == 0 ? gx : (ax == 1 ? gy : gz)) / mag;
    };
    const double div = (normal(i + 1, j, k, 0) - normal(i - 1, j, k, 0)) * ix2
                     + (normal(i, j + 1, k, 1) - normal(i, j - 1, k, 1)) * iy2
                     + (normal(i, j, k + 1, 2) - normal(i, j, k - 1, 2)) * iz2;
    ((gptr<double>)D.kap)[q] = -div;
}

// ---------------------------------------------------------------------------------------------
// momentum with mixture properties and surface tension
// ---------------------------------------------------------------------------------------------
template <bool WALLS, int MODEL>
__global__ __launch_bounds__(NT2) void k_momentum_two_phase(Batch B)
{
    const int b = blockIdx.y;
    const Desc& D = *B.d[b];
    const Cells C{D.nx, D.ny, D.nz, WALLS};
    const long long q = (long long)blockIdx.x * NT2 + threadIdx.x;
    if (q >= D.ncell) return;
    const int nx = C.nx, ny = C.ny;
    const int i = (int)(q % nx), j = (int)((q / nx) % ny), k = (int)(q / ((long long)nx * ny));
    const int st = B.state[b];
    const bool euler = (st & ST_EULER) != 0;
    const double dt = B.dt[b];
    const double c1 = euler ? 1.0 : 1.5, c2 = euler ? 0.0 : -0.5;
    const long long ps = D.ps, n = D.ncell;
    const gptr<const double> gu = (gptr<const double>)D.u, gv = (gptr<const double>)D.v,
                             gw = (gptr<const double>)D.w;
    const gptr<const double> Bn = (gptr<const double>)D.Bt[st & 1];
    const gptr<const double> phi = (gptr<const double>)D.phi, kap = (gptr<const double>)D.kap;
    const gptr<double> RU = (gptr<double>)D.RU;
    const double dx = D.dx, dy = D.dy, dz = D.dz, e = D.eps_if;
    const double L2 = D.L2, afene = D.a_fene;

    // velocities with the ghost rules of the walls
    auto U = [&](int ii, int jj, int kk) {
        ii = wrap2(ii, nx); kk = wrap2(kk, C.nz);
        if (!WALLS) return gu[C.at(ii, wrap2(jj, ny), kk)];
        if (jj < 0) return 2.0 * D.u_bot - gu[C.at(ii, -1 - jj, kk)];
        if (jj >= ny) return 2.0 * D.u_top - gu[C.at(ii, 2 * ny - 1 - jj, kk)];
        return gu[C.at(ii, jj, kk)];
    };
    auto W = [&](int ii, int jj, int kk) {
        ii = wrap2(ii, nx); kk = wrap2(kk, C.nz);
        if (!WALLS) return gw[C.at(ii, wrap2(jj, ny), kk)];
        if (jj < 0) return 2.0 * D.w_bot - gw[C.at(ii, -1 - jj, kk)];
        if (jj >= ny) return 2.0 * D.w_top - gw[C.at(ii, 2 * ny - 1 - jj, kk)];
        return gw[C.at(ii, jj, kk)];
    };
    auto V = [&](int ii, int jj, int kk) {
        ii = wrap2(ii, nx); kk = wrap2(kk, C.nz);
        if (!WALLS) return gv[C.at(ii, wrap2(jj, ny), kk)];
        if (jj == -1 || jj == ny - 1) return 0.0;
        if (jj < -1) return -gv[C.at(ii, -2 - jj, kk)];
        if (jj > ny - 1) return -gv[C.at(ii, 2 * ny - 2 - jj, kk)];
        return gv[C.at(ii, jj, kk)];
    };
    // mixture properties of a cell (ghost rows copy the interior row)
    auto Hc = [&](int ii, int jj, int kk) { return heaviside(C.clamp(phi, ii, jj, kk), e); };
    auto mus = [&](int ii, int jj, int kk) { const double h = Hc(ii, jj, kk); return D.mus1 * h + D.mus2 * (1.0 - h); };
    auto rho = [&](int ii, int jj, int kk) { const double h = Hc(ii, jj, kk); return D.rho1 * h + D.rho2 * (1.0 - h); };
    auto Gc = [&](int ii, int jj, int kk) {
        const double h = Hc(ii, jj, kk);
        return (D.mup1 * h + D.mup2 * (1.0 - h)) / (D.lam1 * h + D.lam2 * (1.0 - h));
    };
    // extra stress component c of a cell (B - I extrapolated past walls, per-cell modulus)
    auto tau = [&](int c, int ii, int jj, int kk) {
        const double G = Gc(ii, jj, kk);
        const double x = C.ext(Bn + c * ps, ii, jj, kk);
        if constexpr (MODEL == EVP_FENE_P) {
            const double tr = C.ext(Bn, ii, jj, kk) + C.ext(Bn + 3 * ps, ii, jj, kk) + C.ext(Bn + 5 * ps, ii, jj, kk) + 3.0;
            const double F = L2 / (L2 - tr);
            return G * F * x + ((c == 0 || c == 3 || c == 5) ? G * (F - afene) : 0.0);
        } else {
            return G * x;
        }
    };
    // surface tension on a face between cells a and b along an axis: sigma kappa_face grad H
    auto csf = [&](int ia, int ja, int ka, int ib, int jb, int kb, double h) {
        if (D.sigma == 0.0) return 0.0;
        const long long qa = C.at(wrap2(ia, nx), ja, wrap2(ka, C.nz)), qb = C.at(wrap2(ib, nx), jb, wrap2(kb, C.nz));
        return D.sigma * 0.5 * (kap[qa] + kap[qb]) * (heaviside(phi[qb], e) - heaviside(phi[qa], e)) / h;
    };
    const double fx = D.force_kind == EVP_FORCE_CONST_X ? D.force_amp
                    : (D.force_kind == EVP_FORCE_SIN_X_OF_Y ? D.force_amp * sin(D.force_ky * (D.y0 + (j + 0.5) * dy)) : 0.0);
    // loads of this cell's history and velocity before any store
    const double ox = euler ? 0.0 : RU[q], oy = euler ? 0.0 : RU[ps + q], oz = euler ? 0.0 : RU[2 * ps + q];
    const double u0 = gu[q], v0 = gv[q], w0 = gw[q];
    double ru[3];
    // ---- x-face (i+1/2, j, k)
    {
        const double cR = 0.5 * (U(i, j, k) + U(i + 1, j, k)), cL = 0.5 * (U(i - 1, j, k) + U(i, j, k));
        const double vT = 0.5 * (V(i, j, k) + V(i + 1, j, k)), vB = 0.5 * (V(i, j - 1, k) + V(i + 1, j - 1, k));
        const double uT = 0.5 * (U(i, j, k) + U(i, j + 1, k)), uB = 0.5 * (U(i, j - 1, k) + U(i, j, k));
        const double wF = 0.5 * (W(i, j, k) + W(i + 1, j, k)), wK = 0.5 * (W(i, j, k - 1) + W(i + 1, j, k - 1));
        const double uF = 0.5 * (U(i, j, k) + U(i, j, k + 1)), uK = 0.5 * (U(i, j, k - 1) + U(i, j, k));
        const double adv = (cR * cR - cL * cL) / dx + (vT * uT - vB * uB) / dy + (wF * uF - wK * uK) / dz;
        const double t1 = 2.0 * mus(i + 1, j, k) * (U(i + 1, j, k) - U(i, j, k)) / dx;
        const double t0 = 2.0 * mus(i, j, k) * (U(i, j, k) - U(i - 1, j, k)) / dx;
        const double mT = 0.25 * (mus(i, j, k) + mus(i + 1, j, k) + mus(i, j + 1, k) + mus(i + 1, j + 1, k));
        const double mB = 0.25 * (mus(i, j, k) + mus(i + 1, j, k) + mus(i, j - 1, k) + mus(i + 1, j - 1, k));
        const double mF = 0.25 * (mus(i, j, k) + mus(i + 1, j, k) + mus(i, j, k + 1) + mus(i + 1, j, k + 1));
        const double mK = 0.25 * (mus(i, j, k) + mus(i + 1, j, k) + mus(i, j, k - 1) + mus(i + 1, j, k - 1));
        const double sT = mT * ((U(i, j + 1, k) - U(i, j, k)) / dy + (V(i + 1, j, k) - V(i, j, k)) / dx);
        const double sB = mB * ((U(i, j, k) - U(i, j - 1, k)) / dy + (V(i + 1, j - 1, k) - V(i, j - 1, k)) / dx);
        const double sF = mF * ((U(i, j, k + 1) - U(i, j, k)) / dz + (W(i + 1, j, k) - W(i, j, k)) / dx);
        const double sK = mK * ((U(i, j, k) - U(i, j, k - 1)) / dz + (W(i + 1, j, k - 1) - W(i, j, k - 1)) / dx);
        const double vis = (t1 - t0) / dx + (sT - sB) / dy + (sF - sK) / dz;
        const double dtau = (tau(0, i + 1, j, k) - tau(0, i, j, k)) / dx
            + 0.25 * (tau(1, i, j + 1, k) + tau(1, i + 1, j + 1, k) - tau(1, i, j - 1, k) - tau(1, i + 1, j - 1, k)) / dy
            + 0.25 * (tau(2, i, j, k + 1) + tau(2, i + 1, j, k + 1) - tau(2, i, j, k - 1) - tau(2, i + 1, j, k - 1)) / dz;
        const double rf = 0.5 * (rho(i, j, k) + rho(i + 1, j, k));
        ru[0] = -adv + (vis + dtau + fx + csf(i, j, k, i + 1, j, k, dx)) / rf;
    }
    // ---- y-face (i, j+1/2, k); the top wall face stays 0
    if (WALLS && j == ny - 1) {
        ru[1] = 0.0;
    } else {
        const double cT = 0.5 * (V(i, j, k) + V(i, j + 1, k)), cB = 0.5 * (V(i, j - 1, k) + V(i, j, k));
        const double uR = 0.5 * (U(i, j, k) + U(i, j + 1, k)), uL = 0.5 * (U(i - 1, j, k) + U(i - 1, j + 1, k));
        const double vR = 0.5 * (V(i, j, k) + V(i + 1, j, k)), vL = 0.5 * (V(i - 1, j, k) + V(i, j, k));
        const double wF = 0.5 * (W(i, j, k) + W(i, j + 1, k)), wK = 0.5 * (W(i, j, k - 1) + W(i, j + 1, k - 1));
        const double vF = 0.5 * (V(i, j, k) + V(i, j, k + 1)), vK = 0.5 * (V(i, j, k - 1) + V(i, j, k));
        const double adv = (uR * vR - uL * vL) / dx + (cT * cT - cB * cB) / dy + (wF * vF - wK * vK) / dz;
        const double t1 = 2.0 * mus(i, j + 1, k) * (V(i, j + 1, k) - V(i, j, k)) / dy;
        const double t0 = 2.0 * mus(i, j, k) * (V(i, j, k) - V(i, j - 1, k)) / dy;
        const double mR = 0.25 * (mus(i, j, k) + mus(i + 1, j, k) + mus(i, j + 1, k) + mus(i + 1, j + 1, k));
        const double mL = 0.25 * (mus(i, j, k) + mus(i - 1, j, k) + mus(i, j + 1, k) + mus(i - 1, j + 1, k));
        const double mF = 0.25 * (mus(i, j, k) + mus(i, j + 1, k) + mus(i, j, k + 1) + mus(i, j + 1, k + 1));
        const double mK = 0.25 * (mus(i, j, k) + mus(i, j + 1, k) + mus(i, j, k - 1) + mus(i, j + 1, k - 1));
        const double sR = mR * ((U(i, j + 1, k) - U(i, j, k)) / dy + (V(i + 1, j, k) - V(i, j, k)) / dx);
        const double sL = mL * ((U(i - 1, j + 1, k) - U(i - 1, j, k)) / dy + (V(i, j, k) - V(i - 1, j, k)) / dx);
        const double sF = mF * ((V(i, j, k + 1) - V(i, j, k)) / dz + (W(i, j + 1, k) - W(i, j, k)) / dy);
        const double sK = mK * ((V(i, j, k) - V(i, j, k - 1)) / dz + (W(i, j + 1, k - 1) - W(i, j, k - 1)) / dy);
        const double vis = (t1 - t0) / dy + (sR - sL) / dx + (sF - sK) / dz;
        const double dtau = 0.25 * (tau(1, i + 1, j, k) + tau(1, i + 1, j + 1, k) - tau(1, i - 1, j, k) - tau(1, i - 1, j + 1, k)) / dx
            + (tau(3, i, j + 1, k) - tau(3, i, j, k)) / dy
            + 0.25 * (tau(4, i, j, k + 1) + tau(4, i, j + 1, k + 1) - tau(4, i, j, k - 1) - tau(4, i, j + 1, k - 1)) / dz;
        const int jn = WALLS ? j + 1 : wrap2(j + 1, ny);
        const double rf = 0.5 * (rho(i, j, k) + rho(i, j + 1, k));
        ru[1] = -adv + (vis + dtau + csf(i, j, k, i, jn, k, dy)) / rf;
    }
    // ---- z-face (i, j, k+1/2)
    {
        const double cF = 0.5 * (W(i, j, k) + W(i, j, k + 1)), cK = 0.5 * (W(i, j, k - 1) + W(i, j, k));
        const double uR = 0.5 * (U(i, j, k) + U(i, j, k + 1)), uL = 0.5 * (U(i - 1, j, k) + U(i - 1, j, k + 1));
        const double wR = 0.5 * (W(i, j, k) + W(i + 1, j, k)), wL = 0.5 * (W(i - 1, j, k) + W(i, j, k));
        const double vT = 0.5 * (V(i, j, k) + V(i, j, k + 1)), vB = 0.5 * (V(i, j - 1, k) + V(i, j - 1, k + 1));
        const double wT = 0.5 * (W(i, j, k) + W(i, j + 1, k)), wB = 0.5 * (W(i, j - 1, k) + W(i, j, k));
        const double adv = (uR * wR - uL * wL) / dx + (vT * wT - vB * wB) / dy + (cF * cF - cK * cK) / dz;
        const double t1 = 2.0 * mus(i, j, k + 1) * (W(i, j, k + 1) - W(i, j, k)) / dz;
        const double t0 = 2.0 * mus(i, j, k) * (W(i, j, k) - W(i, j, k - 1)) / dz;
        const double mR = 0.25 * (mus(i, j, k) + mus(i + 1, j, k) + mus(i, j, k + 1) + mus(i + 1, j, k + 1));
        const double mL = 0.25 * (mus(i, j, k) + mus(i - 1, j, k) + mus(i, j, k + 1) + mus(i - 1, j, k + 1));
        const double mT = 0.25 * (mus(i, j, k) + mus(i, j + 1, k) + mus(i, j, k + 1) + mus(i, j + 1, k + 1));
        const double mB = 0.25 * (mus(i, j, k) + mus(i, j - 1, k) + mus(i, j, k + 1) + mus(i, j - 1, k + 1));
        const double sR = mR * ((U(i, j, k + 1) - U(i, j, k)) / dz + (W(i + 1, j, k) - W(i, j, k)) / dx);
        const double sL = mL * ((U(i - 1, j, k + 1) - U(i - 1, j, k)) / dz + (W(i, j, k) - W(i - 1, j, k)) / dx);
        const double sT = mT * ((V(i, j, k + 1) - V(i, j, k)) / dz + (W(i, j + 1, k) - W(i, j, k)) / dy);
        const double sB = mB * ((V(i, j - 1, k + 1) - V(i, j - 1, k)) / dz + (W(i, j, k) - W(i, j - 1, k)) / dy);
        const double vis = (t1 - t0) / dz + (sR - sL) / dx + (sT - sB) / dy;
        const double dtau = 0.25 * (tau(2, i + 1, j, k) + tau(2, i + 1, j, k + 1) - tau(2, i - 1, j, k) - tau(2, i - 1, j, k + 1)) / dx
            + 0.25 * (tau(4, i, j + 1, k) + tau(4, i, j + 1, k + 1) - tau(4, i, j - 1, k) - tau(4, i, j - 1, k + 1)) / dy
            + (tau(5, i, j, k + 1) - tau(5, i, j, k)) / dz;
        const double rf = 0.5 * (rho(i, j, k) + rho(i, j, k + 1));
        ru[2] = -adv + (vis + dtau + csf(i, j, k, i, j, k + 1, dz)) / rf;
    }
    const gptr<double> us = (gptr<double>)D.us, vs = (gptr<double>)D.vs, ws = (gptr<double>)D.ws;
    us[q] = u0 + dt * (c1 * ru[0] + c2 * ox);
    vs[q] = (WALLS && j == ny - 1) ? 0.0 : v0 + dt * (c1 * ru[1] + c2 * oy);
    ws[q] = w0 + dt * (c1 * ru[2] + c2 * oz);
    RU[q] = ru[0];
    RU[ps + q] = ru[1];
    RU[2 * ps + q] = ru[2];
    (void)n;
}

// freeze: u* = u, RU = 0 (the stress alone advances)
__global__ __launch_bounds__(NT2) void k_momentum_freeze(Batch B)
{
    const Desc& D = *B.d[blockIdx.y];
    const long long q = (long long)blockIdx.x * NT2 + threadIdx.x;
    if (q >= D.ncell) return;
    const double a = ((gptr<const double>)D.u)[q], b = ((gptr<const double>)D.v)[q],
                 c = ((gptr<const double>)D.w)[q];
    ((gptr<double>)D.us)[q] = a;
    ((gptr<double>)D.vs)[q] = b;
    ((gptr<double>)D.ws)[q] = c;
    const gptr<double> RU = (gptr<double>)D.RU;
    RU[q] = 0.0;
    RU[D.ps + q] = 0.0;
    RU[2 * D.ps + q] = 0.0;
}

// ---------------------------------------------------------------------------------------------
// pressure splitting: p_hat = 2 p^n - p^{n-1} (0 without history), p_old <- p^n
// ---------------------------------------------------------------------------------------------
__global__ __launch_bounds__(NT2) void k_split_history(Batch B)
{
    const int b = blockIdx.y;
    const Desc& D = *B.d[b];
    const long long q = (long long)blockIdx.x * NT2 + threadIdx.x;
    if (q >= D.ncell) return;
    const gptr<double> ph = (gptr<double>)D.p_hat, po = (gptr<double>)D.p_old;
    if (B.state[b] & ST_PZERO) {
        ph[q] = 0.0;
        po[q] = 0.0;
    } else {
        const double p = ((gptr<const double>)D.p)[q], o = po[q];
        ph[q] = 2.0 * p - o;
        po[q] = p;
    }
}

// u* -= dt (1/rho_face - 1/rho_0) grad p_hat (no change on the top wall face)
template <bool WALLS>
__global__ __launch_bounds__(NT2) void k_split_velocity(Batch B)
{
    const int b = blockIdx.y;
    const Desc& D = *B.d[b];
    if (B.state[b] & ST_PZERO) return;            // p_hat = 0
    const Cells C{D.nx, D.ny, D.nz, WALLS};
    const long long q = (long long)blockIdx.x * NT2 + threadIdx.x;
    if (q >= D.ncell) return;
    const int nx = C.nx, ny = C.ny;
    const int i = (int)(q % nx), j = (int)((q / nx) % ny), k = (int)(q / ((long long)nx * ny));
    const gptr<const double> ph = (gptr<const double>)D.p_hat, phi = (gptr<const double>)D.phi;
    const double e = D.eps_if, dt = B.dt[b], ir0 = 1.0 / D.rho0;
    auto rho = [&](long long c) { const double h = heaviside(phi[c], e); return D.rho1 * h + D.rho2 * (1.0 - h); };
    const double r0 = rho(q), p0 = ph[q];
    const long long qx = C.at(wrap2(i + 1, nx), j, k), qz = C.at(i, j, wrap2(k + 1, C.nz));
    const double ux = ((gptr<const double>)D.us)[q], wz = ((gptr<const double>)D.ws)[q];
    const double vy = ((gptr<const double>)D.vs)[q];
    const double px = ph[qx], pz = ph[qz], rx = rho(qx), rz = rho(qz);
    double py = 0.0, ry = 1.0;
    const bool top = WALLS && j == ny - 1;
    if (!top) {
        const long long qy = C.at(i, wrap2(j + 1, ny), k);
        py = ph[qy];
        ry = rho(qy);
    }
    ((gptr<double>)D.us)[q] = ux - dt * (1.0 / (0.5 * (r0 + rx)) - ir0) * ((px - p0) / D.dx);
    ((gptr<double>)D.ws)[q] = wz - dt * (1.0 / (0.5 * (r0 + rz)) - ir0) * ((pz - p0) / D.dz);
    if (!top) ((gptr<double>)D.vs)[q] = vy - dt * (1.0 / (0.5 * (r0 + ry)) - ir0) * ((py - p0) / D.dy);
}

__global__ __launch_bounds__(NT2) void k_fill(gptr<double> p, long long n, double value)
{
    const long long q = (long long)blockIdx.x * NT2 + threadIdx.x;
    if (q < n) p[q] = value;
}

}  // namespace

hipError_t launch_fill(double* p, long long n, double value, hipStream_t s)
{
    hipLaunchKernelGGL(k_fill, dim3((unsigned)((n + NT2 - 1) / NT2)), dim3(NT2), 0, s, (gptr<double>)p, n, value);
    return hipGetLastError();
}

static dim3 cells_grid(const Batch& b, int nx, int ny, int nz)
{
    const long long n = (long long)nx * ny * nz;
    return dim3((unsigned)((n + NT2 - 1) / NT2), b.count);
}

hipError_t launch_level_set_stage(const Batch& b, int nx, int ny, int nz, bool walls, bool reinit,
                                  int stage, hipStream_t s)
{
    const dim3 g = cells_grid(b, nx, ny, nz);
    if (walls) hipLaunchKernelGGL(k_level_set_stage<true>, g, dim3(NT2), 0, s, b, reinit ? 1 : 0, stage);
    else hipLaunchKernelGGL(k_level_set_stage<false>, g, dim3(NT2), 0, s, b, reinit ? 1 : 0, stage);
    return hipGetLastError();
}

hipError_t launch_reinit_sign(const Batch& b, int nx, int ny, int nz, hipStream_t s)
{
    hipLaunchKernelGGL(k_reinit_sign, cells_grid(b, nx, ny, nz), dim3(NT2), 0, s, b);
    return hipGetLastError();
}

hipError_t launch_curvature(const Batch& b, int nx, int ny, int nz, bool walls, hipStream_t s)
{
    const dim3 g = cells_grid(b, nx, ny, nz);
    if (walls) hipLaunchKernelGGL(k_curvature<true>, g, dim3(NT2), 0, s, b);
    else hipLaunchKernelGGL(k_curvature<false>, g, dim3(NT2), 0, s, b);
    return hipGetLastError();
}

hipError_t launch_momentum_two_phase(const Batch& b, int nx, int ny, int nz, bool walls, int model,
                                     bool freeze, hipStream_t s)
{
    const dim3 g = cells_grid(b, nx, ny, nz);
    if (freeze) {
        hipLaunchKernelGGL(k_momentum_freeze, g, dim3(NT2), 0, s, b);
        return hipGetLastError();
    }
#define EVP_MOM2(WW, MM) hipLaunchKernelGGL((k_momentum_two_phase<WW, MM>), g, dim3(NT2), 0, s, b)
    if (walls) {
        if (model == EVP_FENE_P) EVP_MOM2(true, EVP_FENE_P); else EVP_MOM2(true, EVP_OLDROYD_B);
    } else {
        if (model == EVP_FENE_P) EVP_MOM2(false, EVP_FENE_P); else EVP_MOM2(false, EVP_OLDROYD_B);
    }
#undef EVP_MOM2
    return hipGetLastError();
}

hipError_t launch_split_pressure(const Batch& b, int nx, int ny, int nz, bool walls, hipStream_t s)
{
    const dim3 g = cells_grid(b, nx, ny, nz);
    hipLaunchKernelGGL(k_split_history, g, dim3(NT2), 0, s, b);
    if (walls) hipLaunchKernelGGL(k_split_velocity<true>, g, dim3(NT2), 0, s, b);
    else hipLaunchKernelGGL(k_split_velocity<false>, g, dim3(NT2), 0, s, b);
    return hipGetLastError();
}

}  // namespace evp
