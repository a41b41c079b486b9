// Predictor of the Adams-Bashforth step, Sec. 3.2.2: for every cell, the stress right-hand side
// RT of Eq. (rt) -- relaxation / yield of Table 1, fifth-order WENO advection (Sec. 3.1) and the
// upper-convected terms of Eq. (SRM2) -- with the AB2 update of Eq. (ab2tau); and on the three
// faces the cell owns, the momentum right-hand side RU of Eq. (ru) (divergence-form advection,
// mu_s times the 7-point Laplacian, div(tau) from centre and edge-averaged stresses, body force)
// with the AB2 predictor u* of Eq. (ab2).
//
// Storage: B is kept as Bt = B - I (exact algebra; keeps the small stresses near equilibrium
// representable in FP32).  T is the compute and storage type of Bt, RT and RU (double for
// EVP_FP64, float for EVP_MIXED); velocities are FP64 in memory, and the FP32 momentum increment
// is added to the FP64 u^n.
//
// Conventions: L_ab = du_a/dx_b at cell centres, upper-convected terms L.B + B.L^T; WENO5 in
// the Hamilton-Jacobi form (Jiang-Peng) with Jiang-Shu weights, eps = 1e-6, upwinded on the
// cell-centre velocity (>= 0: left-biased); walls: u, w reflected about the wall velocity, v = 0
// on wall faces, Bt extrapolated linearly into ghost rows.
#include "evp_internal.h"

namespace evp {

namespace {

constexpr int BX = 64, BY = 4;

__device__ __forceinline__ int wrapi(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

template <typename T> struct Cell {
    const Desc& D;
    int nx, ny, nz;
    bool walls;
    long long sxy;
    // x and z neighbour coordinates, offsets -3..+3 (index o+3)
    int xi[7], zk[7];
    int j;

    __device__ Cell(const Desc& d, int i, int jj, int k)
        : D(d), nx(d.nx), ny(d.ny), nz(d.nz), walls(d.walls != 0), sxy((long long)d.nx * d.ny), j(jj)
    {
#pragma unroll
        for (int o = 0; o < 7; ++o) { xi[o] = wrapi(i + o - 3, nx); zk[o] = wrapi(k + o - 3, nz); }
    }

    __device__ __forceinline__ long long at(int ox, int jj, int oz) const
    {
        return (long long)zk[oz + 3] * sxy + (long long)jj * nx + xi[ox + 3];
    }

    // u (or w, with its wall velocities) on a face row jj = j + oy
    __device__ __forceinline__ double vel_uw(const double* f, double bot, double top, int ox,
                                             int oy, int oz) const
    {
        int jj = j + oy;
        if (!walls) return f[at(ox, wrapi(jj, ny), oz)];
        if (jj < 0) return 2.0 * bot - f[at(ox, -1 - jj, oz)];
        if (jj >= ny) return 2.0 * top - f[at(ox, 2 * ny - 1 - jj, oz)];
        return f[at(ox, jj, oz)];
    }
    __device__ __forceinline__ double U(int ox, int oy, int oz) const { return vel_uw(D.u, D.u_bot, D.u_top, ox, oy, oz); }
    __device__ __forceinline__ double W(int ox, int oy, int oz) const { return vel_uw(D.w, D.w_bot, D.w_top, ox, oy, oz); }
    __device__ __forceinline__ double V(int ox, int oy, int oz) const
    {
        int jj = j + oy;
        if (!walls) return D.v[at(ox, wrapi(jj, ny), oz)];
        if (jj <= -1 || jj >= ny - 1) return 0.0;   // wall faces (only j-1..j+1 are used)
        return D.v[at(ox, jj, oz)];
    }
    // component of Bt = B - I at a neighbouring centre; linear extrapolation beyond a wall
    __device__ __forceinline__ T Bt(const T* b, int ox, int oy, int oz) const
    {
        int jj = j + oy;
        if (!walls) return b[at(ox, wrapi(jj, ny), oz)];
        if (jj < 0) {
            T g = (T)(-jj);
            return ((T)1 + g) * b[at(ox, 0, oz)] - g * b[at(ox, 1, oz)];
        }
        if (jj >= ny) {
            T g = (T)(jj - (ny - 1));
            return ((T)1 + g) * b[at(ox, ny - 1, oz)] - g * b[at(ox, ny - 2, oz)];
        }
        return b[at(ox, jj, oz)];
    }
};

// Fifth-order WENO derivative from the one-sided difference quotients v1..v5; the three weights
// share one division.
template <typename T>
__device__ __forceinline__ T weno5(T v1, T v2, T v3, T v4, T v5)
{
    const T eps = (T)1e-6;
    const T c13 = (T)(13.0 / 12.0), q = (T)0.25;
    T p1 = v1 * (T)(1.0 / 3.0) - v2 * (T)(7.0 / 6.0) + v3 * (T)(11.0 / 6.0);
    T p2 = -v2 * (T)(1.0 / 6.0) + v3 * (T)(5.0 / 6.0) + v4 * (T)(1.0 / 3.0);
    T p3 = v3 * (T)(1.0 / 3.0) + v4 * (T)(5.0 / 6.0) - v5 * (T)(1.0 / 6.0);
    T a = v1 - (T)2 * v2 + v3, b = v1 - (T)4 * v2 + (T)3 * v3;
    T s1 = c13 * a * a + q * b * b;
    a = v2 - (T)2 * v3 + v4; b = v2 - v4;
    T s2 = c13 * a * a + q * b * b;
    a = v3 - (T)2 * v4 + v5; b = (T)3 * v3 - (T)4 * v4 + v5;
    T s3 = c13 * a * a + q * b * b;
    T e1 = eps + s1, e2 = eps + s2, e3 = eps + s3;
    e1 *= e1; e2 *= e2; e3 *= e3;
    // alpha_k = d_k / e_k; omega_k = alpha_k / sum -> common denominator e1 e2 e3
    T w1 = (T)0.1 * e2 * e3, w2 = (T)0.6 * e1 * e3, w3 = (T)0.3 * e1 * e2;
    return (w1 * p1 + w2 * p2 + w3 * p3) / (w1 + w2 + w3);
}

// Upwind WENO5 derivative at the centre of f[0..6] (offsets -3..+3), inverse spacing ih.
template <typename T>
__device__ __forceinline__ T weno_upwind(const T* f, T ih, T vel)
{
    T d0 = (f[1] - f[0]) * ih, d1 = (f[2] - f[1]) * ih, d2 = (f[3] - f[2]) * ih;
    T d3 = (f[4] - f[3]) * ih, d4 = (f[5] - f[4]) * ih, d5 = (f[6] - f[5]) * ih;
    if (vel >= (T)0) return weno5<T>(d0, d1, d2, d3, d4);
    return weno5<T>(d5, d4, d3, d2, d1);
}

// Extra stress (Table 1 solved for tau) from the six Bt values at one centre.
template <typename T>
__device__ __forceinline__ void stress(const Desc& D, const T* bt, T* tau)
{
    const T G = (T)D.G;
    if (D.model == EVP_FENE_P) {
        const T L2 = (T)D.L2;
        const T F = L2 / (L2 - (bt[0] + bt[3] + bt[5] + (T)3));
        const T fa = F - (T)D.a_fene;
#pragma unroll
        for (int c = 0; c < 6; ++c) tau[c] = G * F * bt[c];
        tau[0] += G * fa; tau[3] += G * fa; tau[5] += G * fa;
    } else {
#pragma unroll
        for (int c = 0; c < 6; ++c) tau[c] = G * bt[c];
    }
}

template <typename T>
__device__ __forceinline__ T tau_at(const Cell<T>& C, const T* Bin, long long ps, int c, int ox,
                                    int oy, int oz)
{
    const Desc& D = C.D;
    const T G = (T)D.G;
    const T b = C.Bt(Bin + c * ps, ox, oy, oz);
    if (D.model != EVP_FENE_P) return G * b;
    const T L2 = (T)D.L2;
    const T tr = C.Bt(Bin, ox, oy, oz) + C.Bt(Bin + 3 * ps, ox, oy, oz) + C.Bt(Bin + 5 * ps, ox, oy, oz);
    const T F = L2 / (L2 - (tr + (T)3));
    T t = G * F * b;
    if (c == 0 || c == 3 || c == 5) t += G * (F - (T)D.a_fene);
    return t;
}

// edge average of a stress component over the four centres (0,0), (a), (b), (a+b) where a and b
// are unit offsets given as (ax, ay, az) and (bx, by, bz)
template <typename T>
__device__ __forceinline__ T tau_edge(const Cell<T>& C, const T* Bin, long long ps, int c,
                                      int ax, int ay, int az, int bx, int by, int bz)
{
    return (T)0.25 * (tau_at(C, Bin, ps, c, 0, 0, 0) + tau_at(C, Bin, ps, c, ax, ay, az)
                      + tau_at(C, Bin, ps, c, bx, by, bz)
                      + tau_at(C, Bin, ps, c, ax + bx, ay + by, az + bz));
}

template <typename T>
__global__ __launch_bounds__(BX * BY) void k_predictor(Batch B, int freeze)
{
    const Desc& D = *B.d[blockIdx.z];
    const int nx = D.nx, ny = D.ny;
    const int tilesy = (ny + BY - 1) / BY;
    const int k = blockIdx.y / tilesy;
    const int j = (blockIdx.y - k * tilesy) * BY + threadIdx.y;
    const int i = blockIdx.x * BX + threadIdx.x;
    if (i >= nx || j >= ny) return;                // no barrier in this kernel
    const int st = B.state[blockIdx.z];
    const T* Bin = (const T*)D.Bt[st & 1];
    T* Bout = (T*)D.Bt[(st & 1) ^ 1];
    T* RT = (T*)D.RT;
    T* RU = (T*)D.RU;
    const bool euler = (st & ST_EULER) != 0;
    const double dtd = B.dt[blockIdx.z];
    const T dt = (T)dtd;
    const T c1 = euler ? (T)1 : (T)1.5, c2 = euler ? (T)0 : (T)-0.5;
    const long long ps = D.ps;
    const Cell<T> C(D, i, j, k);
    const long long q = C.at(0, j, 0);
    const T idx = (T)D.idx, idy = (T)D.idy, idz = (T)D.idz;

    // ---- velocity gradient L_ab = du_a/dx_b and velocity at the cell centre
    T L[3][3];
    L[0][0] = (T)(C.U(0, 0, 0) - C.U(-1, 0, 0)) * idx;
    L[0][1] = (T)(C.U(0, 1, 0) + C.U(-1, 1, 0) - C.U(0, -1, 0) - C.U(-1, -1, 0)) * ((T)0.25 * idy);
    L[0][2] = (T)(C.U(0, 0, 1) + C.U(-1, 0, 1) - C.U(0, 0, -1) - C.U(-1, 0, -1)) * ((T)0.25 * idz);
    L[1][0] = (T)(C.V(1, 0, 0) + C.V(1, -1, 0) - C.V(-1, 0, 0) - C.V(-1, -1, 0)) * ((T)0.25 * idx);
    L[1][1] = (T)(C.V(0, 0, 0) - C.V(0, -1, 0)) * idy;
    L[1][2] = (T)(C.V(0, 0, 1) + C.V(0, -1, 1) - C.V(0, 0, -1) - C.V(0, -1, -1)) * ((T)0.25 * idz);
    L[2][0] = (T)(C.W(1, 0, 0) + C.W(1, 0, -1) - C.W(-1, 0, 0) - C.W(-1, 0, -1)) * ((T)0.25 * idx);
    L[2][1] = (T)(C.W(0, 1, 0) + C.W(0, 1, -1) - C.W(0, -1, 0) - C.W(0, -1, -1)) * ((T)0.25 * idy);
    L[2][2] = (T)(C.W(0, 0, 0) - C.W(0, 0, -1)) * idz;
    const T uc = (T)(0.5 * (C.U(0, 0, 0) + C.U(-1, 0, 0)));
    const T vc = (T)(0.5 * (C.V(0, 0, 0) + C.V(0, -1, 0)));
    const T wc = (T)(0.5 * (C.W(0, 0, 0) + C.W(0, 0, -1)));

    // ---- Table 1 closure at this cell
    T bt[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) bt[c] = Bin[c * ps + q];
    T F = (T)1, a = (T)1;
    if (D.model == EVP_FENE_P) {
        const T L2 = (T)D.L2;
        F = L2 / (L2 - (bt[0] + bt[3] + bt[5] + (T)3));
        a = (T)D.a_fene;
    } else if (D.model == EVP_SARAMITO) {
        const T G = (T)D.G;
        const T t3 = G * (bt[0] + bt[3] + bt[5]) * (T)(1.0 / 3.0);
        const T dxx = G * bt[0] - t3, dyy = G * bt[3] - t3, dzz = G * bt[5] - t3;
        const T txy = G * bt[1], txz = G * bt[2], tyz = G * bt[4];
        const T nrm = sqrt((T)0.5 * (dxx * dxx + dyy * dyy + dzz * dzz)
                           + txy * txy + txz * txz + tyz * tyz);
        const T ty = (T)D.tau_y;
        F = (ty == (T)0) ? (T)1 : (nrm > ty ? (T)1 - ty / nrm : (T)0);
        a = F;
    }
    const T il = (T)D.inv_lam;

    // ---- stress right-hand side, Eq. (rt), and AB2 update, Eq. (ab2tau)
    const int pa[6] = {0, 0, 0, 1, 1, 2}, pb[6] = {0, 1, 2, 1, 2, 2};
    const int cmat[3][3] = {{0, 1, 2}, {1, 3, 4}, {2, 4, 5}};
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        const T* b = Bin + c * ps;
        T fx[7], fy[7], fz[7];
#pragma unroll
        for (int o = 0; o < 7; ++o) {
            fx[o] = b[C.at(o - 3, j, 0)];
            fy[o] = C.Bt(b, 0, o - 3, 0);
            fz[o] = b[C.at(0, j, o - 3)];
        }
        const T adv = uc * weno_upwind<T>(fx, idx, uc) + vc * weno_upwind<T>(fy, idy, vc)
                    + wc * weno_upwind<T>(fz, idz, wc);
        const int p = pa[c], r = pb[c];
        T ucv = L[p][r] + L[r][p];                 // (L.I + I.L^T)_pr
#pragma unroll
        for (int m = 0; m < 3; ++m) ucv += L[p][m] * bt[cmat[m][r]] + bt[cmat[p][m]] * L[r][m];
        const T relax = (((p == r) ? (a - F) : (T)0) - F * bt[c]) * il;
        const T rt = relax - adv + ucv;
        const T old = euler ? (T)0 : RT[c * ps + q];
        Bout[c * ps + q] = bt[c] + dt * (c1 * rt + c2 * old);
        RT[c * ps + q] = rt;
    }

    if (freeze) {
        D.us[q] = D.u[q]; D.vs[q] = D.v[q]; D.ws[q] = D.w[q];
        RU[q] = (T)0; RU[ps + q] = (T)0; RU[2 * ps + q] = (T)0;
        return;
    }

    // ---- momentum right-hand side, Eq. (ru), and predictor, Eq. (ab2)
    const T ms = (T)D.mu_s, irho = (T)D.inv_rho;
    const T idx2 = idx * idx, idy2 = idy * idy, idz2 = idz * idz;
    const T h = (T)0.5;
    // x-face (i+1/2, j, k)
    T rux;
    {
        const T u0 = (T)C.U(0, 0, 0), ue = (T)C.U(1, 0, 0), uw = (T)C.U(-1, 0, 0);
        const T un = (T)C.U(0, 1, 0), us = (T)C.U(0, -1, 0), uf = (T)C.U(0, 0, 1), ub = (T)C.U(0, 0, -1);
        const T cR = h * (u0 + ue), cL = h * (uw + u0);
        const T vT = h * (T)(C.V(0, 0, 0) + C.V(1, 0, 0)), vB = h * (T)(C.V(0, -1, 0) + C.V(1, -1, 0));
        const T wF = h * (T)(C.W(0, 0, 0) + C.W(1, 0, 0)), wB = h * (T)(C.W(0, 0, -1) + C.W(1, 0, -1));
        const T adv = (cR * cR - cL * cL) * idx + (vT * h * (u0 + un) - vB * h * (us + u0)) * idy
                    + (wF * h * (u0 + uf) - wB * h * (ub + u0)) * idz;
        const T lap = (ue - (T)2 * u0 + uw) * idx2 + (un - (T)2 * u0 + us) * idy2
                    + (uf - (T)2 * u0 + ub) * idz2;
        const T dtau = (tau_at(C, Bin, ps, 0, 1, 0, 0) - tau_at(C, Bin, ps, 0, 0, 0, 0)) * idx
                     + (tau_edge(C, Bin, ps, 1, 1, 0, 0, 0, 1, 0) - tau_edge(C, Bin, ps, 1, 1, 0, 0, 0, -1, 0)) * idy
                     + (tau_edge(C, Bin, ps, 2, 1, 0, 0, 0, 0, 1) - tau_edge(C, Bin, ps, 2, 1, 0, 0, 0, 0, -1)) * idz;
        T f = (T)0;
        if (D.force_kind == EVP_FORCE_CONST_X) f = (T)D.force_amp;
        else if (D.force_kind == EVP_FORCE_SIN_X_OF_Y)
            f = (T)(D.force_amp * sin(D.force_ky * (D.y0 + (j + 0.5) * D.dy)));
        rux = -adv + (ms * lap + dtau + f) * irho;
    }
    // y-face (i, j+1/2, k); the top wall face stays at rest
    T ruy = (T)0;
    const bool vwall = D.walls && j == ny - 1;
    if (!vwall) {
        const T v0 = (T)C.V(0, 0, 0), vn = (T)C.V(0, 1, 0), vs = (T)C.V(0, -1, 0);
        const T ve = (T)C.V(1, 0, 0), vw = (T)C.V(-1, 0, 0), vf = (T)C.V(0, 0, 1), vb = (T)C.V(0, 0, -1);
        const T cT = h * (v0 + vn), cB = h * (vs + v0);
        const T uR = h * (T)(C.U(0, 0, 0) + C.U(0, 1, 0)), uL = h * (T)(C.U(-1, 0, 0) + C.U(-1, 1, 0));
        const T wF = h * (T)(C.W(0, 0, 0) + C.W(0, 1, 0)), wB = h * (T)(C.W(0, 0, -1) + C.W(0, 1, -1));
        const T adv = (uR * h * (v0 + ve) - uL * h * (vw + v0)) * idx + (cT * cT - cB * cB) * idy
                    + (wF * h * (v0 + vf) - wB * h * (vb + v0)) * idz;
        const T lap = (ve - (T)2 * v0 + vw) * idx2 + (vn - (T)2 * v0 + vs) * idy2
                    + (vf - (T)2 * v0 + vb) * idz2;
        const T dtau = (tau_edge(C, Bin, ps, 1, 0, 1, 0, 1, 0, 0) - tau_edge(C, Bin, ps, 1, 0, 1, 0, -1, 0, 0)) * idx
                     + (tau_at(C, Bin, ps, 3, 0, 1, 0) - tau_at(C, Bin, ps, 3, 0, 0, 0)) * idy
                     + (tau_edge(C, Bin, ps, 4, 0, 1, 0, 0, 0, 1) - tau_edge(C, Bin, ps, 4, 0, 1, 0, 0, 0, -1)) * idz;
        ruy = -adv + (ms * lap + dtau) * irho;
    }
    // z-face (i, j, k+1/2)
    T ruz;
    {
        const T w0 = (T)C.W(0, 0, 0), wf = (T)C.W(0, 0, 1), wb = (T)C.W(0, 0, -1);
        const T we = (T)C.W(1, 0, 0), ww = (T)C.W(-1, 0, 0), wn = (T)C.W(0, 1, 0), ws = (T)C.W(0, -1, 0);
        const T cF = h * (w0 + wf), cB = h * (wb + w0);
        const T uR = h * (T)(C.U(0, 0, 0) + C.U(0, 0, 1)), uL = h * (T)(C.U(-1, 0, 0) + C.U(-1, 0, 1));
        const T vT = h * (T)(C.V(0, 0, 0) + C.V(0, 0, 1)), vB = h * (T)(C.V(0, -1, 0) + C.V(0, -1, 1));
        const T adv = (uR * h * (w0 + we) - uL * h * (ww + w0)) * idx
                    + (vT * h * (w0 + wn) - vB * h * (ws + w0)) * idy + (cF * cF - cB * cB) * idz;
        const T lap = (we - (T)2 * w0 + ww) * idx2 + (wn - (T)2 * w0 + ws) * idy2
                    + (wf - (T)2 * w0 + wb) * idz2;
        const T dtau = (tau_edge(C, Bin, ps, 2, 0, 0, 1, 1, 0, 0) - tau_edge(C, Bin, ps, 2, 0, 0, 1, -1, 0, 0)) * idx
                     + (tau_edge(C, Bin, ps, 4, 0, 0, 1, 0, 1, 0) - tau_edge(C, Bin, ps, 4, 0, 0, 1, 0, -1, 0)) * idy
                     + (tau_at(C, Bin, ps, 5, 0, 0, 1) - tau_at(C, Bin, ps, 5, 0, 0, 0)) * idz;
        ruz = -adv + (ms * lap + dtau) * irho;
    }
    const T ox = euler ? (T)0 : RU[q], oy = euler ? (T)0 : RU[ps + q], oz = euler ? (T)0 : RU[2 * ps + q];
    D.us[q] = D.u[q] + (double)(dt * (c1 * rux + c2 * ox));
    D.vs[q] = vwall ? 0.0 : D.v[q] + (double)(dt * (c1 * ruy + c2 * oy));
    D.ws[q] = D.w[q] + (double)(dt * (c1 * ruz + c2 * oz));
    RU[q] = rux; RU[ps + q] = ruy; RU[2 * ps + q] = ruz;
}

}  // namespace

hipError_t launch_predictor_ref(const Batch& b, int precision, int nx, int ny, int nz, bool freeze,
                                hipStream_t s)
{
    dim3 block(BX, BY);
    dim3 grid((nx + BX - 1) / BX, ((ny + BY - 1) / BY) * nz, b.count);
    if (precision == EVP_MIXED)
        hipLaunchKernelGGL(k_predictor<float>, grid, block, 0, s, b, freeze ? 1 : 0);
    else
        hipLaunchKernelGGL(k_predictor<double>, grid, block, 0, s, b, freeze ? 1 : 0);
    return hipGetLastError();
}

}  // namespace evp
