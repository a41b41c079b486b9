// Predictor of the Adams-Bashforth step (Sec. 3.2.2, Eqs. (rt), (ab2tau), (ru), (ab2)) -- or of
// one Runge-Kutta substep (Sec. 3.3.1) -- as a z-marching LDS-tiled kernel laid out for CDNA4:
//   * a block of 32 x 8 threads owns a 32 x 8 column of cells and marches along z over a chunk of
//     planes, so every field is read from HBM about once;
//   * the seven planes k-3..k+3 that the z-direction WENO needs for the thread's own cell live in
//     registers (a sliding window);
//   * plane k of B - I, with the 3-cell cross halo of the x/y WENO stencils (ghost rows beyond a
//     wall extrapolated at load time), sits in LDS;
//   * three-plane rings in LDS hold the velocities and the stress components tau_xz, tau_yz,
//     tau_zz of planes k-1, k, k+1 on the tile plus a 1-cell halo (momentum stencils and the
//     velocity gradient);
//   * FENE-P stress factors G F and G (F - a) of plane k are staged once per cell.
// Block ids are remapped so consecutive tiles land on the same XCD (shared L2 for halo reads).
#include <cstdlib>

#include "evp_internal.h"
#include "weno.h"

namespace evp {

namespace {

constexpr int TX = 32, TY = 8, NTH = TX * TY;
constexpr int RW = TX + 6, RH = TY + 6;    // B plane with a 3-cell halo
constexpr int BW = TX + 2, BH = TY + 2;    // 1-cell halo box
constexpr int BOX = BW * BH;

// The tile rows (in y) one launch covers: rows.first + r for r < rows.count, shifted up by
// rows.skip once they reach rows.skip_from (so one launch can take the bottom and top rows of a
// channel and leave out the interior ones).
struct Rows { int first, count, skip_from, skip; };

__device__ __forceinline__ int modp(int i, int n)
{
    int r = i % n;
    return r < 0 ? r + n : r;
}

// Loads and stores at a wave-uniform base plus a per-thread byte offset that fits 32 bits
// (within one plane of one field).  BUF: as raw buffer instructions, whose descriptor (base, no
// stride, 2^31 - 1 bytes; fourth word the raw-buffer format of CDNA, 32-bit data, no swizzle)
// lives in scalar registers, so an access costs no vector arithmetic and no 64-bit address
// registers (this lets the FP32 kernel run four waves per SIMD); otherwise as global
// instructions on the base plus the zero-extended offset (measured faster for the FP64 kernel).
constexpr int kRawBufferWord3 = 0x00020000;
// Cache policy of an access.  kKeep: data that neighbouring tiles read again as their halo
// (B - I, u, v, w).  kStream: data that only this cell touches in this kernel (the history it
// reads, every result it writes); the non-temporal bit lets L2 evict those lines first, so the
// halo lines of a plane survive until the neighbouring tiles have read them.  The value is the
// non-temporal bit of the buffer instructions' cache-policy operand.
constexpr int kKeep = 0, kStream = 2;
template <bool BUF, typename T, int POL = kKeep>
__device__ __forceinline__ T ldx(gptr<const T> base, unsigned boff)
{
    if constexpr (BUF) {
        const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc((EVP_GLOBAL void*)base, (short)0, 0x7fffffff, kRawBufferWord3);
        if constexpr (sizeof(T) == 4) return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, boff, 0, POL));
        else return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, boff, 0, POL));
    } else {
        const gptr<const T> a = (gptr<const T>)((gptr<const char>)base + boff);
        if constexpr (POL == kStream) return __builtin_nontemporal_load(a);
        else return *a;
    }
}
template <bool BUF, typename T, int POL = kStream>
__device__ __forceinline__ void stx(gptr<T> base, unsigned boff, T v)
{
    if constexpr (BUF) {
        typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
        const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc((EVP_GLOBAL void*)base, (short)0, 0x7fffffff, kRawBufferWord3);
        if constexpr (sizeof(T) == 4) __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, boff, 0, POL);
        else __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, boff, 0, POL);
    } else {
        const gptr<T> a = (gptr<T>)((gptr<char>)base + boff);
        if constexpr (POL == kStream) __builtin_nontemporal_store(v, a);
        else *a = v;
    }
}

template <typename T> struct Smem {
    T B[6][RH][RW];      // B - I of plane k
    T gf[BH][BW];        // G F of plane k (G for Oldroyd-B / Saramito)
    T ga[BH][BW];        // G (F - a) of plane k (0 for Oldroyd-B / Saramito)
    T Z[3][3][BH][BW];   // ring slot, (tau_xz, tau_yz, tau_zz)
    T V[3][3][BH][BW];   // ring slot, (u, v, w)
};

// upwind derivative (times h) at the middle of f0..f6: WENO5, or HOUC5 (the fifth-order linear
// upwind-biased combination)
template <typename T, bool HOUC>
__device__ __forceinline__ T weno_up(T f0, T f1, T f2, T f3, T f4, T f5, T f6, T vel, T eps2)
{
    const T d0 = f1 - f0, d1 = f2 - f1, d2 = f3 - f2, d3 = f4 - f3, d4 = f5 - f4, d5 = f6 - f5;
    // pick the upwind-side differences with selects, then evaluate one WENO (no divergence)
    const bool pos = vel >= (T)0;
    const T v1 = pos ? d0 : d5, v2 = pos ? d1 : d4, v3 = pos ? d2 : d3;
    const T v4 = pos ? d3 : d2, v5 = pos ? d4 : d1;
    if constexpr (HOUC)
        return (T)(2.0 / 60.0) * v1 - (T)(13.0 / 60.0) * v2 + (T)(47.0 / 60.0) * v3
             + (T)(27.0 / 60.0) * v4 - (T)(3.0 / 60.0) * v5;
    else
        return weno5u<T>(v1, v2, v3, v4, v5, eps2);
}

// upwind derivative (times h) from six values g0..g5 already in upwind order (for a negative
// velocity the caller passes the stencil mirrored, f6..f1, and gets minus the derivative: the
// scheme is odd in its differences, and every step of it is sign-symmetric in floating point)
template <typename T, bool HOUC>
__device__ __forceinline__ T weno_dir(T g0, T g1, T g2, T g3, T g4, T g5, T eps2)
{
    const T v1 = g1 - g0, v2 = g2 - g1, v3 = g3 - g2, v4 = g4 - g3, v5 = g5 - g4;
    if constexpr (HOUC)
        return (T)(2.0 / 60.0) * v1 - (T)(13.0 / 60.0) * v2 + (T)(47.0 / 60.0) * v3
             + (T)(27.0 / 60.0) * v4 - (T)(3.0 / 60.0) * v5;
    else
        return weno5u<T>(v1, v2, v3, v4, v5, eps2);
}

// RK3: the substep of Sec. 3.3.1 instead of AB2.  B^k = B^{k-1} + dt (zeta RT^{k-1} + xi RT^{k-2});
// the momentum part leaves out the stress divergence at the new level (added by k_stress_div once
// B^k is complete) and the pressure gradient (the projection then yields p^k itself), and keeps
// the advection term as the history: u~ = u + dt [-zeta A^{k-1} - xi A^{k-2}
// + (2 alpha (mu_s lap u + f) + alpha div tau^{k-1}) / rho].
// HOUC: fifth-order upstream-central advection instead of WENO5 (a separate instantiation, so
// the WENO kernel's register allocation is not shared with the other scheme).
// TWOPH: two-phase mode (Sec. 3.2, FP64, AB2): lambda and G = mu_p/lambda of the cell come from
// the mixture at phi^{n+1}; only the stress is advanced (the momentum has its own kernel).
// The block's work: tile `bid` of the tile rows `rows`, z-chunks of kc planes.
template <typename T, bool WALLS, int MODEL, bool RK3, bool HOUC, bool TWOPH>
__device__ __forceinline__ void pred_block(Smem<T>& S, const Batch& B, int freeze, int kc, Rows rows, int bid)
{
    // buffer-instruction accesses in the FP32 kernels and the FP64 wall kernel (which then keeps
    // its ghost-row state in registers without spilling)
    constexpr bool BUF = sizeof(T) == 4 || WALLS;
    const int b = blockIdx.y;
    const Desc& D = *B.d[b];
    const int nx = D.nx, ny = D.ny, nz = D.nz;
    const int sxy = nx * ny;
    const int ps = (int)D.ps;
    const int ntx = (nx + TX - 1) / TX, nty = rows.count, nch = (nz + kc - 1) / kc;
    const int nblk = ntx * nty * nch;
    if ((nblk & 7) == 0) bid = (bid & 7) * (nblk >> 3) + (bid >> 3);     // XCD-contiguous tiles
    const int tile_x = bid % ntx, ch = bid / (ntx * nty);
    int tile_y = rows.first + (bid / ntx) % nty;
    if (tile_y >= rows.skip_from) tile_y += rows.skip;
    const int i0 = tile_x * TX, j0 = tile_y * TY, k0 = ch * kc;
    const int k1 = min(k0 + kc, nz);
    const int tx = threadIdx.x % TX, ty = threadIdx.x / TX;
    const int i = i0 + tx, j = j0 + ty;
    const bool valid = i < nx && j < ny;
    const int ic = min(i, nx - 1), jc = min(j, ny - 1);
    const int oij = jc * nx + ic;

    const int st = B.state[b];
    const gptr<const T> __restrict__ Bin = (gptr<const T>)D.Bt[st & 1];
    const gptr<T> __restrict__ Bout = (gptr<T>)D.Bt[(st & 1) ^ 1];
    const gptr<T> __restrict__ RT = (gptr<T>)D.RT;
    const gptr<T> __restrict__ RU = (gptr<T>)D.RU;
    const bool euler = (st & ST_EULER) != 0;
    const T dt = (T)B.dt[b];
    // history weights: AB2 (3/2, -1/2; Euler start 1, 0) or the substep's (zeta, xi)
    const T c1 = RK3 ? (T)B.rk[0] : (euler ? (T)1 : (T)1.5);
    const T c2 = euler ? (T)0 : (RK3 ? (T)B.rk[1] : (T)-0.5);
    constexpr bool fene = MODEL == EVP_FENE_P, sara = MODEL == EVP_SARAMITO, neo = MODEL == EVP_NEO_HOOKEAN;
    const T kap = (T)D.kappa;
    const T G = (T)D.G, L2 = (T)D.L2, afene = (T)D.a_fene, il = (T)D.inv_lam, tyld = (T)D.tau_y;
    const T idx = (T)D.idx, idy = (T)D.idy, idz = (T)D.idz;
    const T e2x = (T)(1e-6 * D.dx * D.dx), e2y = (T)(1e-6 * D.dy * D.dy), e2z = (T)(1e-6 * D.dz * D.dz);
    const gptr<const double> __restrict__ gu = (gptr<const double>)D.u;
    const gptr<const double> __restrict__ gv = (gptr<const double>)D.v;
    const gptr<const double> __restrict__ gw = (gptr<const double>)D.w;
    const gptr<double> __restrict__ gus = (gptr<double>)D.us;
    const gptr<double> __restrict__ gvs = (gptr<double>)D.vs;
    const gptr<double> __restrict__ gws = (gptr<double>)D.ws;

    // ---- staging descriptors, computed once: the per-plane offsets do not depend on k ----
    // Interior slots (the block's own cells) are filled from the thread's register window; only
    // halo slots, and interior slots of threads whose cell lies outside the domain (ragged
    // tiles: periodic image or wall ghost), are read from global memory.
    // B-plane halo: rows j0-1 and j0+TY over the full width, columns i0-3..i0-1 and
    // i0+TX..i0+TX+2 of the tile's rows, and the arm rows j0-3, j0-2, j0+TY+1, j0+TY+2 over the
    // tile's columns.  Box halo: the 1-cell ring.
    constexpr int NHB = 2 * RW + 6 * TY + 4 * TX;
    constexpr int NHX = 2 * BW + 2 * TY;
    static_assert(NHB <= NTH && NHX <= NTH, "one halo slot per thread");
    // row map of a (possibly ghost) centre row jg: value = wa B[ja] + wb B[jb]
    auto rowmap = [&](int jg, int& ja, int& jb, T& wa, T& wb) {
        if (!WALLS) { ja = modp(jg, ny); jb = ja; wa = (T)1; wb = (T)0; return; }
        if (jg < 0) { const T g = (T)(-jg); ja = 0; jb = 1; wa = (T)1 + g; wb = -g; return; }
        if (jg >= ny) { const T g = (T)(jg - ny + 1); ja = ny - 1; jb = ny - 2; wa = (T)1 + g; wb = -g; return; }
        ja = jg; jb = jg; wa = (T)1; wb = (T)0;
    };
    struct Src { int a, b; T wa, wb; };          // B value = wa B[a] + wb B[b] (plane-relative)
    struct VSrc { int o, kind; };                  // velocity row offset; 0 inner, 1/2 ghost, 3 top v-face
    auto bsrc = [&](int ig, int jg) {
        Src q; int ja, jb; rowmap(jg, ja, jb, q.wa, q.wb);
        q.a = ja * nx + ig; q.b = jb * nx + ig; return q;
    };
    auto vsrc = [&](int ig, int jg) {
        VSrc q;
        if (!WALLS) { q.o = modp(jg, ny) * nx + ig; q.kind = 0; }
        else if (jg < 0) { q.o = min(-1 - jg, ny - 1) * nx + ig; q.kind = 1; }
        else if (jg >= ny) { q.o = max(2 * ny - 1 - jg, 0) * nx + ig; q.kind = 2; }
        else { q.o = jg * nx + ig; q.kind = (jg == ny - 1) ? 3 : 0; }
        return q;
    };
    const int t = threadIdx.x;
    int hb_l = -1;
    Src hb{0, 0, (T)1, (T)0};
    if (t < NHB) {
        int r, c;
        if (t < 2 * RW) { r = t < RW ? 2 : TY + 3; c = t % RW; }
        else if (t < 2 * RW + 6 * TY) { const int u = t - 2 * RW, c6 = u % 6; r = 3 + u / 6; c = c6 < 3 ? c6 : TX + c6; }
        else { const int u = t - 2 * RW - 6 * TY, qq = u / TX; r = qq < 2 ? qq : TY + 2 + qq; c = 3 + u % TX; }
        hb_l = r * RW + c;
        hb = bsrc(modp(i0 + c - 3, nx), j0 + r - 3);
    }
    int hx_l = -1;
    Src hx{0, 0, (T)1, (T)0};
    VSrc hv{0, 0};
    if (t < NHX) {
        int r, c;
        if (t < 2 * BW) { r = t < BW ? 0 : TY + 1; c = t % BW; }
        else { const int u = t - 2 * BW; r = 1 + u / 2; c = (u & 1) ? TX + 1 : 0; }
        hx_l = r * BW + c;
        hx = bsrc(modp(i0 + c - 1, nx), j0 + r - 1);
        hv = vsrc(modp(i0 + c - 1, nx), j0 + r - 1);
    }
    const int own_b = (ty + 3) * RW + (tx + 3), own_x = (ty + 1) * BW + (tx + 1);
    const Src os = bsrc(modp(i, nx), j);           // used only when the cell is outside the domain
    const VSrc ov = vsrc(modp(i, nx), j);

    constexpr unsigned TS = sizeof(T);
    auto bload = [&](gptr<const T> p, int cc, const Src& q) {
        T x = ldx<BUF, T>(p + cc * ps, (unsigned)q.a * TS);
        if (WALLS) x = q.wa * x + q.wb * ldx<BUF, T>(p + cc * ps, (unsigned)q.b * TS);
        return x;
    };
    auto vload = [&](int kv, const VSrc& q, T* out) {
        const unsigned o8 = (unsigned)q.o * 8u;
        const double uu = ldx<BUF, double>(gu + kv, o8), vv = ldx<BUF, double>(gv + kv, o8), ww = ldx<BUF, double>(gw + kv, o8);
        if (!WALLS || q.kind == 0) { out[0] = (T)uu; out[1] = (T)vv; out[2] = (T)ww; }
        else if (q.kind == 3) { out[0] = (T)uu; out[1] = (T)0; out[2] = (T)ww; }
        else {
            const bool bot = q.kind == 1;
            out[0] = (T)(2.0 * (bot ? D.u_bot : D.u_top) - uu);
            out[1] = (T)0;
            out[2] = (T)(2.0 * (bot ? D.w_bot : D.w_top) - ww);
        }
    };
    // stress factors G F, G (F - a) of a B - I value set
    auto factors = [&](T b0, T b3, T b5, T& gfo, T& gao) {
        gfo = G; gao = (T)0;
        if (fene) {
            const T F = L2 / (L2 - (b0 + b3 + b5 + (T)3));
            gfo = G * F; gao = G * (F - afene);
        }
    };

    T* const sB = &S.B[0][0][0];
    // B - I of plane kk with the cross halo into S.B (own value: the window entry of plane kk)
    auto load_bplane = [&](int kk, const T* own) {
        const gptr<const T> bk = Bin + kk * sxy;
        T hvv[6], ovv[6];
#pragma unroll
        for (int cc = 0; cc < 6; ++cc) {
            hvv[cc] = (hb_l >= 0) ? bload(bk, cc, hb) : (T)0;
            ovv[cc] = valid ? own[cc] : bload(bk, cc, os);
        }
#pragma unroll
        for (int cc = 0; cc < 6; ++cc) {
            if (hb_l >= 0) sB[cc * (RH * RW) + hb_l] = hvv[cc];
            sB[cc * (RH * RW) + own_b] = ovv[cc];
        }
    };

    // ring slot sl <- tau_xz, tau_yz, tau_zz and u, v, w of plane kz (own B - I values: ownz);
    // if ownk != nullptr also the stress factors of plane k (own values: ownk)
    auto load_box = [&](int kz, const T* ownz, int sl, int kg, const T* ownk) {
        const gptr<const T> bz = Bin + kz * sxy;
        const gptr<const T> bg = Bin + kg * sxy;
        const int kv = kz * sxy;
        // halo slot
        T hz[3], hvel[3], hgf = G, hga = (T)0;
        if (hx_l >= 0) {
            T gf, ga;
            if (fene) factors(bload(bz, 0, hx), bload(bz, 3, hx), bload(bz, 5, hx), gf, ga);
            else { gf = G; ga = (T)0; }
            hz[0] = gf * bload(bz, 2, hx); hz[1] = gf * bload(bz, 4, hx); hz[2] = gf * bload(bz, 5, hx) + ga;
            vload(kv, hv, hvel);
            if (ownk && fene) factors(bload(bg, 0, hx), bload(bg, 3, hx), bload(bg, 5, hx), hgf, hga);
        }
        // own slot
        T oz[3], ovel[3], ogf = G, oga = (T)0;
        {
            T zb[6];
#pragma unroll
            for (int cc = 0; cc < 6; ++cc) zb[cc] = (cc == 1) ? (T)0 : (valid ? ownz[cc] : bload(bz, cc, os));
            T gf, ga;
            factors(zb[0], zb[3], zb[5], gf, ga);
            oz[0] = gf * zb[2]; oz[1] = gf * zb[4]; oz[2] = gf * zb[5] + ga;
            vload(kv, ov, ovel);
            if (ownk && fene) {
                if (valid) factors(ownk[0], ownk[3], ownk[5], ogf, oga);
                else factors(bload(bg, 0, os), bload(bg, 3, os), bload(bg, 5, os), ogf, oga);
            }
        }
        T* zs = &S.Z[sl][0][0][0];
        T* vs = &S.V[sl][0][0][0];
        if (hx_l >= 0) {
            zs[hx_l] = hz[0]; zs[BOX + hx_l] = hz[1]; zs[2 * BOX + hx_l] = hz[2];
            vs[hx_l] = hvel[0]; vs[BOX + hx_l] = hvel[1]; vs[2 * BOX + hx_l] = hvel[2];
            if (ownk) { (&S.gf[0][0])[hx_l] = hgf; (&S.ga[0][0])[hx_l] = hga; }
        }
        zs[own_x] = oz[0]; zs[BOX + own_x] = oz[1]; zs[2 * BOX + own_x] = oz[2];
        vs[own_x] = ovel[0]; vs[BOX + own_x] = ovel[1]; vs[2 * BOX + own_x] = ovel[2];
        if (ownk) { (&S.gf[0][0])[own_x] = ogf; (&S.ga[0][0])[own_x] = oga; }
    };

    // forcing on this thread's x-face row
    T fx = (T)0;
    if (D.force_kind == EVP_FORCE_CONST_X) fx = (T)D.force_amp;
    else if (D.force_kind == EVP_FORCE_SIN_X_OF_Y) fx = (T)(D.force_amp * sin(D.force_ky * (D.y0 + (jc + 0.5) * D.dy)));

    // prologue: register window planes k0-3..k0+2, rings for planes k0-1 and k0
    T win[7][6];
#pragma unroll
    for (int m = 0; m < 6; ++m) {
        const gptr<const T> p = Bin + modp(k0 - 3 + m, nz) * sxy;
#pragma unroll
        for (int cc = 0; cc < 6; ++cc) win[m][cc] = ldx<BUF, T>(p + cc * ps, (unsigned)oij * TS);
    }
    load_box(modp(k0 - 1, nz), win[2], (k0 + 2) % 3, 0, nullptr);
    load_box(k0, win[3], (k0 + 3) % 3, 0, nullptr);

    const T ms = (T)D.mu_s, irho = (T)D.inv_rho;
    const T idx2 = idx * idx, idy2 = idy * idy, idz2 = idz * idz;
    const T h = (T)0.5, qt = (T)0.25;
    const bool vwall = WALLS && j == ny - 1;

    for (int k = k0; k < k1; ++k) {
        const int kp = modp(k + 1, nz);
        {
            const gptr<const T> p = Bin + modp(k + 3, nz) * sxy;
#pragma unroll
            for (int cc = 0; cc < 6; ++cc) win[6][cc] = ldx<BUF, T>(p + cc * ps, (unsigned)oij * TS);
        }
        load_bplane(k, win[3]);
        load_box(kp, win[4], (k + 4) % 3, k, win[3]);
        __syncthreads();

        if (valid) {
            const int q = k * sxy + j * nx + i;
            const int r = ty + 3, c = tx + 3, rb = ty + 1, cb = tx + 1;
            const int sm = (k + 2) % 3, s0 = (k + 3) % 3, sp = (k + 4) % 3;
#define VU(s, di, dj) S.V[s][0][rb + (dj)][cb + (di)]
#define VV(s, di, dj) S.V[s][1][rb + (dj)][cb + (di)]
#define VW(s, di, dj) S.V[s][2][rb + (dj)][cb + (di)]
            // velocity gradient L_ab = du_a/dx_b at the centre, and the centre velocity
            T L[3][3];
            L[0][0] = (VU(s0, 0, 0) - VU(s0, -1, 0)) * idx;
            L[0][1] = (VU(s0, 0, 1) + VU(s0, -1, 1) - VU(s0, 0, -1) - VU(s0, -1, -1)) * (qt * idy);
            L[0][2] = (VU(sp, 0, 0) + VU(sp, -1, 0) - VU(sm, 0, 0) - VU(sm, -1, 0)) * (qt * idz);
            L[1][0] = (VV(s0, 1, 0) + VV(s0, 1, -1) - VV(s0, -1, 0) - VV(s0, -1, -1)) * (qt * idx);
            L[1][1] = (VV(s0, 0, 0) - VV(s0, 0, -1)) * idy;
            L[1][2] = (VV(sp, 0, 0) + VV(sp, 0, -1) - VV(sm, 0, 0) - VV(sm, 0, -1)) * (qt * idz);
            L[2][0] = (VW(s0, 1, 0) + VW(sm, 1, 0) - VW(s0, -1, 0) - VW(sm, -1, 0)) * (qt * idx);
            L[2][1] = (VW(s0, 0, 1) + VW(sm, 0, 1) - VW(s0, 0, -1) - VW(sm, 0, -1)) * (qt * idy);
            L[2][2] = (VW(s0, 0, 0) - VW(sm, 0, 0)) * idz;
            const T uc = h * (VU(s0, 0, 0) + VU(s0, -1, 0));
            const T vc = h * (VV(s0, 0, 0) + VV(s0, 0, -1));
            const T wc = h * (VW(s0, 0, 0) + VW(sm, 0, 0));

            // Table 1 closure of this cell
            const T* bt = win[3];
            T Gc = G, ilc = il;
            if constexpr (TWOPH) {
                const double hh = heaviside(((gptr<const double>)D.phi)[q], D.eps_if);
                const double lam = D.lam1 * hh + D.lam2 * (1.0 - hh), mup = D.mup1 * hh + D.mup2 * (1.0 - hh);
                Gc = (T)(mup / lam);
                ilc = (T)(1.0 / lam);
            }
            T F = (T)1, a = (T)1;
            if (fene) {
                F = L2 / (L2 - (bt[0] + bt[3] + bt[5] + (T)3));
                a = afene;
            } else if (sara) {
                const T t3 = Gc * (bt[0] + bt[3] + bt[5]) * (T)(1.0 / 3.0);
                const T dxx = Gc * bt[0] - t3, dyy = Gc * bt[3] - t3, dzz = Gc * bt[5] - t3;
                const T txy = Gc * bt[1], txz = Gc * bt[2], tyz = Gc * bt[4];
                const T nrm = sqrt((T)0.5 * (dxx * dxx + dyy * dyy + dzz * dzz)
                                   + txy * txy + txz * txz + tyz * tyz);
                F = (tyld == (T)0) ? (T)1 : (nrm > tyld ? (T)1 - tyld / nrm : (T)0);
                a = F;
            } else if (neo) {
                F = (T)0;
                a = (T)0;
            }
            // local artificial diffusion (Sec. 3.1): det B < 0, or tr B >= 0.95 L^2 (FENE-P)
            bool diffon = false;
            if (kap > (T)0) {
                const T b0 = bt[0] + (T)1, b3 = bt[3] + (T)1, b5 = bt[5] + (T)1;
                const T det = b0 * (b3 * b5 - bt[4] * bt[4]) - bt[1] * (bt[1] * b5 - bt[4] * bt[2])
                            + bt[2] * (bt[1] * bt[4] - b3 * bt[2]);
                diffon = det < (T)0 || (fene && b0 + b3 + b5 >= (T)0.95 * L2);
            }

            // stress right-hand side (Eq. rt) and AB2 update (Eq. ab2tau)
            const int pa[6] = {0, 0, 0, 1, 1, 2}, pb[6] = {0, 1, 2, 1, 2, 2};
            const int cm[3][3] = {{0, 1, 2}, {1, 3, 4}, {2, 4, 5}};
            T rtv[6];
            {
                // FP64: x and y stencils read from LDS in upwind order: element m of the x stencil
                // is column c + sx (m - 3), of the y stencil row r + sy (m - 3), with s = +1 for a
                // non-negative velocity and -1 otherwise; the sign of the derivative then comes
                // with |velocity| in the advection term (no selects; bitwise the same numbers).
                // FP32 keeps the selects: the per-thread LDS addresses cost it registers at four
                // waves per SIMD.
                constexpr bool MIRROR = sizeof(T) == 8;
                const int sx = uc >= (T)0 ? 1 : -1, sy = vc >= (T)0 ? RW : -RW;
                const T* const bx = &S.B[0][r][c];
                const T auc = uc >= (T)0 ? uc : -uc, avc = vc >= (T)0 ? vc : -vc;
#pragma unroll
                for (int cc = 0; cc < 6; ++cc) {
                    T gx, gy;
                    if constexpr (MIRROR) {
                        const T* const pc = bx + cc * (RH * RW);
                        gx = weno_dir<T, HOUC>(pc[-3 * sx], pc[-2 * sx], pc[-sx], pc[0], pc[sx], pc[2 * sx], e2x);
                        gy = weno_dir<T, HOUC>(pc[-3 * sy], pc[-2 * sy], pc[-sy], pc[0], pc[sy], pc[2 * sy], e2y);
                    } else {
                        gx = weno_up<T, HOUC>(S.B[cc][r][c - 3], S.B[cc][r][c - 2], S.B[cc][r][c - 1], S.B[cc][r][c],
                                              S.B[cc][r][c + 1], S.B[cc][r][c + 2], S.B[cc][r][c + 3], uc, e2x);
                        gy = weno_up<T, HOUC>(S.B[cc][r - 3][c], S.B[cc][r - 2][c], S.B[cc][r - 1][c], S.B[cc][r][c],
                                              S.B[cc][r + 1][c], S.B[cc][r + 2][c], S.B[cc][r + 3][c], vc, e2y);
                    }
                    const T gz = weno_up<T, HOUC>(win[0][cc], win[1][cc], win[2][cc], win[3][cc], win[4][cc],
                                                  win[5][cc], win[6][cc], wc, e2z);
                    const T adv = MIRROR ? auc * gx * idx + avc * gy * idy + wc * gz * idz
                                         : uc * gx * idx + vc * gy * idy + wc * gz * idz;
                    const int p = pa[cc], rr = pb[cc];
                    T ucv = L[p][rr] + L[rr][p];
#pragma unroll
                    for (int m = 0; m < 3; ++m) ucv += L[p][m] * bt[cm[m][rr]] + bt[cm[p][m]] * L[rr][m];
                    const T relax = (((p == rr) ? (a - F) : (T)0) - F * bt[cc]) * ilc;
                    rtv[cc] = relax - adv + ucv;
                    // bound live ranges: finish this component before the next one's LDS reads
                    __asm__ volatile("" ::"v"(rtv[cc]) : "memory");
                }
            }
            if (diffon) {
#pragma unroll
                for (int cc = 0; cc < 6; ++cc)
                    rtv[cc] += kap * ((S.B[cc][r][c - 1] - (T)2 * bt[cc] + S.B[cc][r][c + 1]) * (idx * idx)
                                      + (S.B[cc][r - 1][c] - (T)2 * bt[cc] + S.B[cc][r + 1][c]) * (idy * idy)
                                      + (win[2][cc] - (T)2 * bt[cc] + win[4][cc]) * (idz * idz));
            }
            // every load of this cell's history and velocity is issued before any store: the
            // compiler cannot move a load above a store it cannot prove disjoint, and a wait for
            // a load also waits for the stores issued before it
            // plane bases (uniform) and this cell's byte offsets within a plane
            const int kq = k * sxy;
            const unsigned ob = (unsigned)(j * nx + i) * TS, o8 = (unsigned)(j * nx + i) * 8u;
            T old[6];
#pragma unroll
            for (int cc = 0; cc < 6; ++cc) old[cc] = euler ? (T)0 : ldx<BUF, T, kStream>(RT + (kq + cc * ps), ob);
            double u0, v0, w0;
            if constexpr (!WALLS && sizeof(T) == 8) {
                // this cell's velocities are in the ring slot of plane k (in FP64 the loaded values
                // themselves), so they need no second load
                u0 = VU(s0, 0, 0); v0 = VV(s0, 0, 0); w0 = VW(s0, 0, 0);
            } else {
                u0 = ldx<BUF, double>(gu + kq, o8); v0 = ldx<BUF, double>(gv + kq, o8); w0 = ldx<BUF, double>(gw + kq, o8);
            }
            T ox = (T)0, oy = (T)0, oz = (T)0;
            if (!euler && !freeze) {
                ox = ldx<BUF, T, kStream>(RU + kq, ob); oy = ldx<BUF, T, kStream>(RU + (kq + ps), ob);
                oz = ldx<BUF, T, kStream>(RU + (kq + 2 * ps), ob);
            }
            // the stress results are stored after the momentum part, so that the history loads
            // above are in flight during it
            auto store_stress = [&]() {
#pragma unroll
                for (int cc = 0; cc < 6; ++cc) {
                    stx<BUF, T>(Bout + (kq + cc * ps), ob, bt[cc] + dt * (c1 * rtv[cc] + c2 * old[cc]));
                    stx<BUF, T>(RT + (kq + cc * ps), ob, rtv[cc]);
                }
            };
            if constexpr (!(sizeof(T) == 8 && !WALLS)) {
                store_stress();
                __asm__ volatile("" ::: "memory");
            }
            if constexpr (TWOPH) {
                // the two-phase momentum follows in k_momentum_two_phase
            } else if (freeze) {
                stx<BUF, double>(gus + kq, o8, u0); stx<BUF, double>(gvs + kq, o8, v0); stx<BUF, double>(gws + kq, o8, w0);
                stx<BUF, T>(RU + kq, ob, (T)0); stx<BUF, T>(RU + (kq + ps), ob, (T)0); stx<BUF, T>(RU + (kq + 2 * ps), ob, (T)0);
            } else {
                // stresses of plane k from B - I and the staged factors
#define TK(cc, di, dj) (fene ? (S.gf[rb + (dj)][cb + (di)] * S.B[cc][r + (dj)][c + (di)] + \
                        (((cc) == 0 || (cc) == 3 || (cc) == 5) ? S.ga[rb + (dj)][cb + (di)] : (T)0)) \
                        : G * S.B[cc][r + (dj)][c + (di)])
#define TZ(s, zc, di, dj) S.Z[s][zc][rb + (dj)][cb + (di)]
                // face terms; RK3 keeps the advection (history) apart from the rest (mx, my, mz)
                const T cal = RK3 ? (T)B.rk[2] : (T)0;
                T mx = (T)0, my = (T)0, mz = (T)0;
                // x-face (i+1/2, j, k)
                T rux;
                {
                    const T u0 = VU(s0, 0, 0), ue = VU(s0, 1, 0), uw = VU(s0, -1, 0);
                    const T un = VU(s0, 0, 1), us = VU(s0, 0, -1), uf = VU(sp, 0, 0), ub = VU(sm, 0, 0);
                    const T cR = h * (u0 + ue), cL = h * (uw + u0);
                    const T vT = h * (VV(s0, 0, 0) + VV(s0, 1, 0)), vB = h * (VV(s0, 0, -1) + VV(s0, 1, -1));
                    const T wF = h * (VW(s0, 0, 0) + VW(s0, 1, 0)), wB = h * (VW(sm, 0, 0) + VW(sm, 1, 0));
                    const T adv = (cR * cR - cL * cL) * idx + (vT * h * (u0 + un) - vB * h * (us + u0)) * idy
                                + (wF * h * (u0 + uf) - wB * h * (ub + u0)) * idz;
                    const T lap = (ue - (T)2 * u0 + uw) * idx2 + (un - (T)2 * u0 + us) * idy2
                                + (uf - (T)2 * u0 + ub) * idz2;
                    const T dtau = (TK(0, 1, 0) - TK(0, 0, 0)) * idx
                                 + qt * (TK(1, 0, 1) + TK(1, 1, 1) - TK(1, 0, -1) - TK(1, 1, -1)) * idy
                                 + qt * (TZ(sp, 0, 0, 0) + TZ(sp, 0, 1, 0) - TZ(sm, 0, 0, 0) - TZ(sm, 0, 1, 0)) * idz;
                    if constexpr (RK3) { rux = adv; mx = (T)2 * cal * (ms * lap + fx) + cal * dtau; }
                    else rux = -adv + (ms * lap + dtau + fx) * irho;
                }
                // y-face (i, j+1/2, k)
                T ruy = (T)0;
                if (!vwall) {
                    const T v0 = VV(s0, 0, 0), vn = VV(s0, 0, 1), vs = VV(s0, 0, -1);
                    const T ve = VV(s0, 1, 0), vw = VV(s0, -1, 0), vf = VV(sp, 0, 0), vb = VV(sm, 0, 0);
                    const T cT = h * (v0 + vn), cB = h * (vs + v0);
                    const T uR = h * (VU(s0, 0, 0) + VU(s0, 0, 1)), uL = h * (VU(s0, -1, 0) + VU(s0, -1, 1));
                    const T wF = h * (VW(s0, 0, 0) + VW(s0, 0, 1)), wB = h * (VW(sm, 0, 0) + VW(sm, 0, 1));
                    const T adv = (uR * h * (v0 + ve) - uL * h * (vw + v0)) * idx + (cT * cT - cB * cB) * idy
                                + (wF * h * (v0 + vf) - wB * h * (vb + v0)) * idz;
                    const T lap = (ve - (T)2 * v0 + vw) * idx2 + (vn - (T)2 * v0 + vs) * idy2
                                + (vf - (T)2 * v0 + vb) * idz2;
                    const T dtau = qt * (TK(1, 1, 0) + TK(1, 1, 1) - TK(1, -1, 0) - TK(1, -1, 1)) * idx
                                 + (TK(3, 0, 1) - TK(3, 0, 0)) * idy
                                 + qt * (TZ(sp, 1, 0, 0) + TZ(sp, 1, 0, 1) - TZ(sm, 1, 0, 0) - TZ(sm, 1, 0, 1)) * idz;
                    if constexpr (RK3) { ruy = adv; my = (T)2 * cal * (ms * lap) + cal * dtau; }
                    else ruy = -adv + (ms * lap + dtau) * irho;
                }
                // z-face (i, j, k+1/2)
                T ruz;
                {
                    const T w0 = VW(s0, 0, 0), wf = VW(sp, 0, 0), wb = VW(sm, 0, 0);
                    const T we = VW(s0, 1, 0), ww = VW(s0, -1, 0), wn = VW(s0, 0, 1), wsv = VW(s0, 0, -1);
                    const T cF = h * (w0 + wf), cB = h * (wb + w0);
                    const T uR = h * (VU(s0, 0, 0) + VU(sp, 0, 0)), uL = h * (VU(s0, -1, 0) + VU(sp, -1, 0));
                    const T vT = h * (VV(s0, 0, 0) + VV(sp, 0, 0)), vB = h * (VV(s0, 0, -1) + VV(sp, 0, -1));
                    const T adv = (uR * h * (w0 + we) - uL * h * (ww + w0)) * idx
                                + (vT * h * (w0 + wn) - vB * h * (wsv + w0)) * idy + (cF * cF - cB * cB) * idz;
                    const T lap = (we - (T)2 * w0 + ww) * idx2 + (wn - (T)2 * w0 + wsv) * idy2
                                + (wf - (T)2 * w0 + wb) * idz2;
                    const T dtau = qt * (TZ(s0, 0, 1, 0) + TZ(sp, 0, 1, 0) - TZ(s0, 0, -1, 0) - TZ(sp, 0, -1, 0)) * idx
                                 + qt * (TZ(s0, 1, 0, 1) + TZ(sp, 1, 0, 1) - TZ(s0, 1, 0, -1) - TZ(sp, 1, 0, -1)) * idy
                                 + (TZ(sp, 2, 0, 0) - TZ(s0, 2, 0, 0)) * idz;
                    if constexpr (RK3) { ruz = adv; mz = (T)2 * cal * (ms * lap) + cal * dtau; }
                    else ruz = -adv + (ms * lap + dtau) * irho;
                }
#undef TK
#undef TZ
                if constexpr (RK3) {
                    // the stress divergence at B^k and any solid penalisation follow in k_stress_div
                    stx<BUF, double>(gus + kq, o8, u0 + (double)(dt * (mx * irho - c1 * rux - c2 * ox)));
                    stx<BUF, double>(gvs + kq, o8, vwall ? 0.0 : v0 + (double)(dt * (my * irho - c1 * ruy - c2 * oy)));
                    stx<BUF, double>(gws + kq, o8, w0 + (double)(dt * (mz * irho - c1 * ruz - c2 * oz)));
                } else {
                    // a solid, if any, is applied by k_penalise once u* is complete
                    stx<BUF, double>(gus + kq, o8, u0 + (double)(dt * (c1 * rux + c2 * ox)));
                    stx<BUF, double>(gvs + kq, o8, vwall ? 0.0 : v0 + (double)(dt * (c1 * ruy + c2 * oy)));
                    stx<BUF, double>(gws + kq, o8, w0 + (double)(dt * (c1 * ruz + c2 * oz)));
                }
                stx<BUF, T>(RU + kq, ob, rux); stx<BUF, T>(RU + (kq + ps), ob, ruy); stx<BUF, T>(RU + (kq + 2 * ps), ob, ruz);
            }
            if constexpr (sizeof(T) == 8 && !WALLS) store_stress();
#undef VU
#undef VV
#undef VW
        }
        __syncthreads();
#pragma unroll
        for (int m = 0; m < 6; ++m)
#pragma unroll
            for (int cc = 0; cc < 6; ++cc) win[m][cc] = win[m + 1][cc];
    }
}

template <typename T, bool WALLS, int MODEL, bool RK3, bool HOUC, bool TWOPH>
__global__ __launch_bounds__(NTH, (sizeof(T) == 4 && !WALLS) ? 4 : 2) void k_pred_zm(Batch B, int freeze, int kc, Rows rows)
{
    __shared__ Smem<T> S;
    pred_block<T, WALLS, MODEL, RK3, HOUC, TWOPH>(S, B, freeze, kc, rows, blockIdx.x);
}

// FP64 channel: the rows next to the walls and the interior tile rows (periodic-in-y code) in one
// grid, the first n_wall blocks the wall rows (the heavier blocks start first), the rest the
// interior.  Both parts run two blocks per CU and take the same planes per block, so the blocks
// of both parts share the rounds instead of the wall rows running after the interior.
template <int MODEL, bool RK3, bool HOUC>
__global__ __launch_bounds__(NTH, 2) void k_pred_zm_channel(Batch B, int freeze, int kc, Rows rows_int, Rows rows_wall, int n_wall)
{
    __shared__ Smem<double> S;
    if ((int)blockIdx.x < n_wall) pred_block<double, true, MODEL, RK3, HOUC, false>(S, B, freeze, kc, rows_wall, blockIdx.x);
    else pred_block<double, false, MODEL, RK3, HOUC, false>(S, B, freeze, kc, rows_int, blockIdx.x - n_wall);
}

}  // namespace

// planes per block: `target` blocks per grid in total (EVP_PRED_BLOCKS overrides it), at least 4
// planes per block.  Measured on one MI355X (blocks resident at once: two per CU for FP64, four
// for the FP32 periodic kernel): periodic grids run best with about one round of resident blocks
// (512 FP64, 1024 FP32), channels with about four rounds (2048), whose shorter z-chunks leave a
// shorter last round
int predictor_chunk_tiles(int tiles, int nz, int target)
{
    static const int target_env = [] {
        const char* e = std::getenv("EVP_PRED_BLOCKS");
        return e ? std::atoi(e) : 0;
    }();
    if (target_env > 0) target = target_env;
    int nch = (target + tiles - 1) / tiles;
    nch = max(1, min(nch, nz / 4));
    return (nz + nch - 1) / nch;
}


hipError_t launch_predictor_zm(const Batch& b, int precision, int nx, int ny, int nz, bool freeze,
                               hipStream_t s, bool walls, int model, bool rk3, bool houc,
                               bool two_phase, const Side* side)
{
    const int ntx = (nx + TX - 1) / TX, nty = (ny + TY - 1) / TY;
    // Channel: tile rows whose whole stencil (B rows j0-3 .. j0+TY+2, velocity rows j0-1 ..
    // j0+TY) lies in rows 0 .. ny-3 never see a ghost row or the top wall face; they run the
    // periodic instantiation (same arithmetic there, and no spills of the ghost-row state), the
    // rows next to the walls the wall instantiation.
    int in_lo = 1, in_hi = walls ? (ny - 3) / TY : 0;
    if (in_hi <= in_lo) in_lo = in_hi = 0;
    const int fz = freeze ? 1 : 0;
    struct Part { bool w; Rows rows; };
    Part parts[2];
    int np = 0;
    if (!walls) parts[np++] = {false, {0, nty, 1 << 30, 0}};
    else {
        if (in_hi > in_lo) parts[np++] = {false, {in_lo, in_hi - in_lo, 1 << 30, 0}};
        if (in_hi > in_lo) parts[np++] = {true, {0, nty - (in_hi - in_lo), in_lo, in_hi - in_lo}};
        else parts[np++] = {true, {0, nty, 1 << 30, 0}};
    }
    // FP64 channels run both parts in one grid (k_pred_zm_channel).  In the mixed form the rows
    // next to the walls run beside the interior on the side stream (measured faster for
    // 256x128x128 and 512x256x256 channels: the FP32 wall and interior kernels differ in
    // occupancy, so one grid would run both at the wall kernel's).  The two-phase mode launches
    // the parts one after the other.
    if (np == 2 && precision == EVP_FP64 && !two_phase) {
        // one grid for both parts, chunked over all tile rows (see k_pred_zm_channel)
        const int kc = predictor_chunk_tiles(ntx * nty, nz, 2048);
        const int nch = (nz + kc - 1) / kc;
        const int n_int = ntx * parts[0].rows.count * nch, n_wall = ntx * parts[1].rows.count * nch;
        dim3 grid(n_int + n_wall, b.count);
#define EVP_LAUNCH_C(MM, RR)                                                                       \
    do {                                                                                           \
        if (houc) hipLaunchKernelGGL((k_pred_zm_channel<MM, RR, true>), grid, dim3(NTH), 0, s, b, fz, kc, parts[0].rows, parts[1].rows, n_wall); \
        else hipLaunchKernelGGL((k_pred_zm_channel<MM, RR, false>), grid, dim3(NTH), 0, s, b, fz, kc, parts[0].rows, parts[1].rows, n_wall); \
    } while (0)
#define EVP_LAUNCH_CR(MM)                                                                          \
    do {                                                                                           \
        if (rk3) EVP_LAUNCH_C(MM, true);                                                           \
        else EVP_LAUNCH_C(MM, false);                                                              \
    } while (0)
        switch (model) {
        case EVP_FENE_P: EVP_LAUNCH_CR(EVP_FENE_P); break;
        case EVP_SARAMITO: EVP_LAUNCH_CR(EVP_SARAMITO); break;
        case EVP_NEO_HOOKEAN: EVP_LAUNCH_CR(EVP_NEO_HOOKEAN); break;
        default: EVP_LAUNCH_CR(EVP_OLDROYD_B); break;
        }
#undef EVP_LAUNCH_CR
#undef EVP_LAUNCH_C
        return hipGetLastError();
    }
    const bool fork = np == 2 && side != nullptr && precision == EVP_MIXED;
    if (fork) {
        hipError_t e = hipEventRecord(side->fork, s);
        if (e == hipSuccess) e = hipStreamWaitEvent(side->s, side->fork, 0);
        if (e != hipSuccess) return e;
    }
    for (int ip = 0; ip < np; ++ip) {
    const bool pw = parts[ip].w;
    const Rows rows = parts[ip].rows;
    const hipStream_t ls = (fork && pw) ? side->s : s;
    const int kc = predictor_chunk_tiles(ntx * rows.count, nz, walls ? 2048 : (precision == EVP_MIXED ? 1024 : 512));
    const int nblk = ntx * rows.count * ((nz + kc - 1) / kc);
    dim3 grid(nblk, b.count);
#define EVP_LAUNCH2(TT, WW, MM, RR)                                                                \
    do {                                                                                           \
        if (houc) hipLaunchKernelGGL((k_pred_zm<TT, WW, MM, RR, true, false>), grid, dim3(NTH), 0, ls, b, fz, kc, rows); \
        else hipLaunchKernelGGL((k_pred_zm<TT, WW, MM, RR, false, false>), grid, dim3(NTH), 0, ls, b, fz, kc, rows); \
    } while (0)
#define EVP_LAUNCH_TP(WW, MM)                                                                      \
    do {                                                                                           \
        if (houc) hipLaunchKernelGGL((k_pred_zm<double, WW, MM, false, true, true>), grid, dim3(NTH), 0, ls, b, fz, kc, rows); \
        else hipLaunchKernelGGL((k_pred_zm<double, WW, MM, false, false, true>), grid, dim3(NTH), 0, ls, b, fz, kc, rows); \
    } while (0)
#define EVP_LAUNCH(TT, WW, MM)                                                                     \
    do {                                                                                           \
        if (rk3) EVP_LAUNCH2(TT, WW, MM, true);                                                    \
        else EVP_LAUNCH2(TT, WW, MM, false);                                                       \
    } while (0)
#define EVP_BY_MODEL(TT, WW)                                                                       \
    switch (model) {                                                                               \
    case EVP_FENE_P: EVP_LAUNCH(TT, WW, EVP_FENE_P); break;                                       \
    case EVP_SARAMITO: EVP_LAUNCH(TT, WW, EVP_SARAMITO); break;                                   \
    case EVP_NEO_HOOKEAN: EVP_LAUNCH(TT, WW, EVP_NEO_HOOKEAN); break;                             \
    default: EVP_LAUNCH(TT, WW, EVP_OLDROYD_B); break;                                            \
    }
    if (two_phase) {
        if (precision != EVP_FP64 || rk3) return hipErrorInvalidValue;
#define EVP_TP_BY_MODEL(WW)                                                                        \
    switch (model) {                                                                               \
    case EVP_FENE_P: EVP_LAUNCH_TP(WW, EVP_FENE_P); break;                                        \
    case EVP_SARAMITO: EVP_LAUNCH_TP(WW, EVP_SARAMITO); break;                                    \
    case EVP_NEO_HOOKEAN: EVP_LAUNCH_TP(WW, EVP_NEO_HOOKEAN); break;                              \
    default: EVP_LAUNCH_TP(WW, EVP_OLDROYD_B); break;                                             \
    }
        if (pw) { EVP_TP_BY_MODEL(true) } else { EVP_TP_BY_MODEL(false) }
#undef EVP_TP_BY_MODEL
    } else if (precision == EVP_MIXED) {
        if (pw) { EVP_BY_MODEL(float, true) } else { EVP_BY_MODEL(float, false) }
    } else {
        if (pw) { EVP_BY_MODEL(double, true) } else { EVP_BY_MODEL(double, false) }
    }
    }
    if (fork) {
        hipError_t e = hipEventRecord(side->join, side->s);
        if (e == hipSuccess) e = hipStreamWaitEvent(s, side->join, 0);
        if (e != hipSuccess) return e;
    }
#undef EVP_BY_MODEL
#undef EVP_LAUNCH
#undef EVP_LAUNCH2
#undef EVP_LAUNCH_TP
    return hipGetLastError();
}

}  // namespace evp
