/*
 * ORACLE -- test infrastructure only.  Only tests/, the smoke check and the CPU-baseline leg
 * of the benchmark may load this library.  It shares no source with the HIP path.
 *
 * Plain, slow, FP64 evaluation of the explicit part of one time step of the paper's Eulerian
 * solver (Izbassarov et al., "Computational modeling of multiphase viscoelastic and
 * elastoviscoplastic flows"):
 *   - the generic conformation-tensor transport, Sec. 2 Eq. (SRM2), closed per model by Table 1;
 *   - the deviatoric stress norm of the Saramito model, Sec. 2 (the |tau^d| definition);
 *   - the spatial discretisation of Sec. 3 (staggered uniform grid, second-order central
 *     differences, fifth-order WENO or HOUC for the stress advection, Sec. 3 and 3.1);
 *   - the local artificial diffusion of Sec. 3.1, added to Eq. (SRM2) where det B < 0 or, for
 *     FENE-P, tr B >= 0.95 L^2, with a caller-given coefficient (the paper tunes it per case);
 *   - the Adams-Bashforth predictor of Sec. 3.2.2, Eqs. (ab2tau), (ab2), (rt), (ru), with rho
 *     constant, g = 0 (absorbed in the pressure) and f a prescribed body force.
 * The pressure projection, Eqs. (var poisson) and (projection), is done by the Python side of
 * the oracle (oracle/__init__.py) from its plain definition.
 *
 * Readings of points the paper leaves open (they are listed with reasons in the design notes):
 *   velocity gradient L_ij = du_i/dx_j, upper-convected terms L.B + B.L^T;
 *   HJ-WENO5 with Jiang-Shu weights, eps = 1e-6, upwinding on the cell-centre velocity,
 *   velocity >= 0 takes the left-biased stencil;
 *   Saramito: tau^d = tau - tr(tau)/3 I, F = 1 when tau_y == 0, else F = 0 when |tau^d| <= tau_y;
 *   FENE-P stress tau = (mu_p/lambda)(F B - a I), Table 1 solved for tau;
 *   Neo-Hookean: F = a = 0 and tau = G B with G = mu_p/lambda (Table 1; lambda enters nowhere
 *   else);
 *   HOUC: the fifth-order upstream-central stencil, upwinded like the WENO scheme;
 *   artificial diffusion: kappa times the 7-point Laplacian of each component of B (ghost rows
 *   as for the advection), switched on per cell by the state at the start of the step;
 *   walls in y: u, w reflected about the wall velocity, v = 0 on wall faces, B extrapolated
 *   linearly into ghost cells;
 *   AB2 starts with a forward-Euler step when no history exists.
 *
 * Field layout: every field is a dense [nz][ny][nx] FP64 array, x fastest.  u[k][j][i] sits on
 * the +x face of cell (i,j,k), v on its +y face, w on its +z face; B is six such arrays in the
 * order xx, xy, xz, yy, yz, zz at cell centres.
 */
#include <math.h>
#include <stddef.h>

enum { M_OLDROYD_B = 0, M_FENE_P = 1, M_SARAMITO = 2, M_NEO_HOOKEAN = 3 };
enum { ADV_WENO5 = 0, ADV_HOUC5 = 1 };
enum { XX = 0, XY = 1, XZ = 2, YY = 3, YZ = 4, ZZ = 5 };

typedef struct {
    int nx, ny, nz;
    int walls;            /* 0: periodic in y; 1: no-slip walls at y = y0 and y = y0 + ny*dy */
    double dx, dy, dz, y0;
    int model;            /* 0 Oldroyd-B, 1 FENE-P, 2 Saramito */
    double rho, mu_s, mu_p, lam, tau_y, L2;
    int force_kind;       /* 0 none, 1 f_x = amp, 2 f_x = amp*sin(ky*y) */
    double force_amp, force_ky;
    double u_bot, u_top, w_bot, w_top;
    int adv_scheme;       /* 0 WENO5, 1 HOUC5 */
    double kappa;         /* artificial diffusion coefficient (0: off) */
    /* two-phase mixture (Sec. 3.2.1): per-cell lambda, mu_p, mu_s, rho at cell centres (NULL:
     * the constants above; a per-cell mu_s selects the full div(mu_s (grad u + grad u^T))) and an
     * extra force density on the faces, three planes x, y, z (NULL: none).  Ghost rows beyond a
     * wall take the properties of the adjacent interior row. */
    const double* lam_c;
    const double* mup_c;
    const double* mus_c;
    const double* rho_c;
    const double* fs;
} oracle_params;

static int wrap(int i, int n) { i %= n; return i < 0 ? i + n : i; }

static size_t at(const oracle_params* P, int i, int j, int k)
{
    return ((size_t)k * P->ny + (size_t)j) * P->nx + (size_t)i;
}

/* x-velocity on the face (i+1/2, j, k), ghost rows by reflection about the wall velocity. */
static double U(const oracle_params* P, const double* u, int i, int j, int k)
{
    i = wrap(i, P->nx); k = wrap(k, P->nz);
    if (!P->walls) return u[at(P, i, wrap(j, P->ny), k)];
    if (j < 0) return 2.0 * P->u_bot - u[at(P, i, -1 - j, k)];
    if (j >= P->ny) return 2.0 * P->u_top - u[at(P, i, 2 * P->ny - 1 - j, k)];
    return u[at(P, i, j, k)];
}

static double W(const oracle_params* P, const double* w, int i, int j, int k)
{
    i = wrap(i, P->nx); k = wrap(k, P->nz);
    if (!P->walls) return w[at(P, i, wrap(j, P->ny), k)];
    if (j < 0) return 2.0 * P->w_bot - w[at(P, i, -1 - j, k)];
    if (j >= P->ny) return 2.0 * P->w_top - w[at(P, i, 2 * P->ny - 1 - j, k)];
    return w[at(P, i, j, k)];
}

/* y-velocity on the face (i, j+1/2, k).  With walls the faces j = -1 and j = ny-1 are the walls
 * (no penetration); beyond them the field is reflected with a sign change. */
static double V(const oracle_params* P, const double* v, int i, int j, int k)
{
    i = wrap(i, P->nx); k = wrap(k, P->nz);
    if (!P->walls) return v[at(P, i, wrap(j, P->ny), k)];
    if (j == -1 || j == P->ny - 1) return 0.0;
    if (j < -1) return -v[at(P, i, -2 - j, k)];
    if (j > P->ny - 1) return -v[at(P, i, 2 * P->ny - 2 - j, k)];
    return v[at(P, i, j, k)];
}

/* Component c of B at the centre of cell (i,j,k); ghost rows beyond a wall are the linear
 * extrapolation of the two nearest interior rows. */
static double Bc(const oracle_params* P, const double* B, int c, int i, int j, int k)
{
    const size_t n = (size_t)P->nx * P->ny * P->nz;
    const double* b = B + (size_t)c * n;
    i = wrap(i, P->nx); k = wrap(k, P->nz);
    if (!P->walls) return b[at(P, i, wrap(j, P->ny), k)];
    if (j < 0) {
        double g = (double)(-j);
        return (1.0 + g) * b[at(P, i, 0, k)] - g * b[at(P, i, 1, k)];
    }
    if (j >= P->ny) {
        double g = (double)(j - (P->ny - 1));
        return (1.0 + g) * b[at(P, i, P->ny - 1, k)] - g * b[at(P, i, P->ny - 2, k)];
    }
    return b[at(P, i, j, k)];
}

/* Material property of cell (i,j,k): per-cell array if given, else the constant; ghost rows
 * copy the nearest interior row. */
static double prop(const oracle_params* P, const double* arr, double c, int i, int j, int k)
{
    if (!arr) return c;
    i = wrap(i, P->nx); k = wrap(k, P->nz);
    if (P->walls) j = j < 0 ? 0 : (j >= P->ny ? P->ny - 1 : j);
    else j = wrap(j, P->ny);
    return arr[at(P, i, j, k)];
}

static double G_at(const oracle_params* P, int i, int j, int k)
{
    return prop(P, P->mup_c, P->mu_p, i, j, k) / prop(P, P->lam_c, P->lam, i, j, k);
}

/* Table 1: the factors F and a of Eq. (SRM2) for the given B; G = mu_p / lambda of the cell. */
static void closure(const oracle_params* P, const double b[6], double G, double* F, double* a)
{
    if (P->model == M_OLDROYD_B) {
        *F = 1.0; *a = 1.0;
    } else if (P->model == M_NEO_HOOKEAN) {
        *F = 0.0; *a = 0.0;
    } else if (P->model == M_FENE_P) {
        double tr = b[XX] + b[YY] + b[ZZ];
        *F = P->L2 / (P->L2 - tr);
        *a = P->L2 / (P->L2 - 3.0);
    } else {
        /* Saramito: tau = (mu_p/lambda)(B - I); von Mises switch on |tau^d| (Sec. 2). */
        double t[6];
        for (int c = 0; c < 6; ++c) t[c] = G * b[c];
        t[XX] -= G; t[YY] -= G; t[ZZ] -= G;
        double tr3 = (t[XX] + t[YY] + t[ZZ]) / 3.0;
        double dxx = t[XX] - tr3, dyy = t[YY] - tr3, dzz = t[ZZ] - tr3;
        double sum = dxx * dxx + dyy * dyy + dzz * dzz
                   + 2.0 * (t[XY] * t[XY] + t[XZ] * t[XZ] + t[YZ] * t[YZ]);
        double norm = sqrt(0.5 * sum);
        double f;
        if (P->tau_y == 0.0) f = 1.0;
        else if (norm > P->tau_y) f = 1.0 - P->tau_y / norm;
        else f = 0.0;
        *F = f; *a = f;
    }
}

/* Extra stress tau from B by inverting the B-definitions of Table 1. */
static void stress_from_B(const oracle_params* P, const double b[6], double G, double t[6])
{
    if (P->model == M_FENE_P) {
        double F, a;
        closure(P, b, G, &F, &a);
        for (int c = 0; c < 6; ++c) t[c] = G * F * b[c];
        t[XX] -= G * a; t[YY] -= G * a; t[ZZ] -= G * a;
    } else if (P->model == M_NEO_HOOKEAN) {
        for (int c = 0; c < 6; ++c) t[c] = G * b[c];
    } else {
        for (int c = 0; c < 6; ++c) t[c] = G * b[c];
        t[XX] -= G; t[YY] -= G; t[ZZ] -= G;
    }
}

static void stress_at(const oracle_params* P, const double* B, int i, int j, int k, double t[6])
{
    double b[6];
    for (int c = 0; c < 6; ++c) b[c] = Bc(P, B, c, i, j, k);
    stress_from_B(P, b, G_at(P, i, j, k), t);
}

/* Fifth-order WENO derivative from the five one-sided difference quotients v1..v5 (the
 * Hamilton-Jacobi form of Jiang & Peng with the smoothness indicators and linear weights of
 * Jiang & Shu), the scheme Sec. 3.1 names for the stress advection. */
static double weno5(double v1, double v2, double v3, double v4, double v5)
{
    const double eps = 1e-6;
    double phi1 = v1 / 3.0 - 7.0 * v2 / 6.0 + 11.0 * v3 / 6.0;
    double phi2 = -v2 / 6.0 + 5.0 * v3 / 6.0 + v4 / 3.0;
    double phi3 = v3 / 3.0 + 5.0 * v4 / 6.0 - v5 / 6.0;
    double s1 = 13.0 / 12.0 * (v1 - 2.0 * v2 + v3) * (v1 - 2.0 * v2 + v3)
              + 0.25 * (v1 - 4.0 * v2 + 3.0 * v3) * (v1 - 4.0 * v2 + 3.0 * v3);
    double s2 = 13.0 / 12.0 * (v2 - 2.0 * v3 + v4) * (v2 - 2.0 * v3 + v4)
              + 0.25 * (v2 - v4) * (v2 - v4);
    double s3 = 13.0 / 12.0 * (v3 - 2.0 * v4 + v5) * (v3 - 2.0 * v4 + v5)
              + 0.25 * (3.0 * v3 - 4.0 * v4 + v5) * (3.0 * v3 - 4.0 * v4 + v5);
    double a1 = 0.1 / ((eps + s1) * (eps + s1));
    double a2 = 0.6 / ((eps + s2) * (eps + s2));
    double a3 = 0.3 / ((eps + s3) * (eps + s3));
    return (a1 * phi1 + a2 * phi2 + a3 * phi3) / (a1 + a2 + a3);
}

/* Upwind WENO5 derivative at the middle of seven consecutive values f[0..6] (offsets -3..+3)
 * with spacing h; vel >= 0 takes backward differences at offsets -2..+2, vel < 0 forward
 * differences at offsets +2..-2. */
static double weno_upwind(const double f[7], double h, double vel)
{
    if (vel >= 0.0)
        return weno5((f[1] - f[0]) / h, (f[2] - f[1]) / h, (f[3] - f[2]) / h,
                     (f[4] - f[3]) / h, (f[5] - f[4]) / h);
    return weno5((f[6] - f[5]) / h, (f[5] - f[4]) / h, (f[4] - f[3]) / h,
                 (f[3] - f[2]) / h, (f[2] - f[1]) / h);
}

/* Fifth-order upstream-central (HOUC) derivative at the middle of f[0..6] (offsets -3..+3):
 * the six-point stencil (-2, 15, -60, 20, 30, -3)/60h on offsets -3..+2 for vel >= 0, and its
 * mirror image on offsets +3..-2 for vel < 0. */
static double houc_upwind(const double f[7], double h, double vel)
{
    if (vel >= 0.0)
        return (-2.0 * f[0] + 15.0 * f[1] - 60.0 * f[2] + 20.0 * f[3] + 30.0 * f[4] - 3.0 * f[5])
               / (60.0 * h);
    return (2.0 * f[6] - 15.0 * f[5] + 60.0 * f[4] - 20.0 * f[3] - 30.0 * f[2] + 3.0 * f[1])
           / (60.0 * h);
}

static double adv_upwind(const oracle_params* P, const double f[7], double h, double vel)
{
    return P->adv_scheme == ADV_HOUC5 ? houc_upwind(f, h, vel) : weno_upwind(f, h, vel);
}

/* Exported for the advection pins: periodic 1D derivative of f (length n, spacing h),
 * upwinded for a uniform velocity of sign vel, with WENO5 (scheme 0) or HOUC5 (scheme 1). */
void oracle_upwind_line(const double* f, int n, double h, double vel, int scheme, double* out)
{
    for (int i = 0; i < n; ++i) {
        double s[7];
        for (int m = 0; m < 7; ++m) s[m] = f[wrap(i + m - 3, n)];
        out[i] = scheme == ADV_HOUC5 ? houc_upwind(s, h, vel) : weno_upwind(s, h, vel);
    }
}

void oracle_weno5_line(const double* f, int n, double h, double vel, double* out)
{
    oracle_upwind_line(f, n, h, vel, ADV_WENO5, out);
}

/* det B of a symmetric tensor stored as xx, xy, xz, yy, yz, zz */
static double det6(const double b[6])
{
    return b[XX] * (b[YY] * b[ZZ] - b[YZ] * b[YZ]) - b[XY] * (b[XY] * b[ZZ] - b[YZ] * b[XZ])
         + b[XZ] * (b[XY] * b[YZ] - b[YY] * b[XZ]);
}

/* Sec. 3.1: local artificial diffusion where B loses positive definiteness (det B < 0) or, for
 * FENE-P, where tr B reaches 95 % of L^2. */
static int diffusion_on(const oracle_params* P, const double b[6])
{
    if (P->kappa <= 0.0) return 0;
    if (det6(b) < 0.0) return 1;
    return P->model == M_FENE_P && b[XX] + b[YY] + b[ZZ] >= 0.95 * P->L2;
}

/* Exported: extra stress from B on every cell (six planes in, six planes out). */
void oracle_stress(const oracle_params* P, const double* B, double* tau)
{
    const size_t n = (size_t)P->nx * P->ny * P->nz;
    for (size_t q = 0; q < n; ++q) {
        double b[6], t[6];
        for (int c = 0; c < 6; ++c) b[c] = B[c * n + q];
        stress_from_B(P, b, (P->mup_c ? P->mup_c[q] : P->mu_p) / (P->lam_c ? P->lam_c[q] : P->lam), t);
        for (int c = 0; c < 6; ++c) tau[c * n + q] = t[c];
    }
}

/* Exported: the closure factors F (and a) of Table 1 on every cell. */
void oracle_closure(const oracle_params* P, const double* B, double* F, double* a)
{
    const size_t n = (size_t)P->nx * P->ny * P->nz;
    for (size_t q = 0; q < n; ++q) {
        double b[6];
        for (int c = 0; c < 6; ++c) b[c] = B[c * n + q];
        closure(P, b, (P->mup_c ? P->mup_c[q] : P->mu_p) / (P->lam_c ? P->lam_c[q] : P->lam),
                &F[q], &a[q]);
    }
}

/* Right-hand side RT of Eq. (rt) at cell (i,j,k): relaxation / yield, WENO advection and the
 * upper-convected terms. */
static void stress_rhs(const oracle_params* P, const double* u, const double* v, const double* w,
                       const double* B, int i, int j, int k, double rt[6])
{
    const double dx = P->dx, dy = P->dy, dz = P->dz;
    /* velocity gradient L[a][b] = du_a/dx_b at the cell centre */
    double L[3][3];
    L[0][0] = (U(P, u, i, j, k) - U(P, u, i - 1, j, k)) / dx;
    L[0][1] = (U(P, u, i, j + 1, k) + U(P, u, i - 1, j + 1, k)
             - U(P, u, i, j - 1, k) - U(P, u, i - 1, j - 1, k)) / (4.0 * dy);
    L[0][2] = (U(P, u, i, j, k + 1) + U(P, u, i - 1, j, k + 1)
             - U(P, u, i, j, k - 1) - U(P, u, i - 1, j, k - 1)) / (4.0 * dz);
    L[1][0] = (V(P, v, i + 1, j, k) + V(P, v, i + 1, j - 1, k)
             - V(P, v, i - 1, j, k) - V(P, v, i - 1, j - 1, k)) / (4.0 * dx);
    L[1][1] = (V(P, v, i, j, k) - V(P, v, i, j - 1, k)) / dy;
    L[1][2] = (V(P, v, i, j, k + 1) + V(P, v, i, j - 1, k + 1)
             - V(P, v, i, j, k - 1) - V(P, v, i, j - 1, k - 1)) / (4.0 * dz);
    L[2][0] = (W(P, w, i + 1, j, k) + W(P, w, i + 1, j, k - 1)
             - W(P, w, i - 1, j, k) - W(P, w, i - 1, j, k - 1)) / (4.0 * dx);
    L[2][1] = (W(P, w, i, j + 1, k) + W(P, w, i, j + 1, k - 1)
             - W(P, w, i, j - 1, k) - W(P, w, i, j - 1, k - 1)) / (4.0 * dy);
    L[2][2] = (W(P, w, i, j, k) - W(P, w, i, j, k - 1)) / dz;

    /* cell-centre velocity (upwinding and advection speed) */
    double uc = 0.5 * (U(P, u, i, j, k) + U(P, u, i - 1, j, k));
    double vc = 0.5 * (V(P, v, i, j, k) + V(P, v, i, j - 1, k));
    double wc = 0.5 * (W(P, w, i, j, k) + W(P, w, i, j, k - 1));

    double b[6];
    for (int c = 0; c < 6; ++c) b[c] = Bc(P, B, c, i, j, k);
    double Bm[3][3] = { { b[XX], b[XY], b[XZ] }, { b[XY], b[YY], b[YZ] }, { b[XZ], b[YZ], b[ZZ] } };
    static const int ia[6] = { 0, 0, 0, 1, 1, 2 }, ib[6] = { 0, 1, 2, 1, 2, 2 };

    double F, a;
    closure(P, b, G_at(P, i, j, k), &F, &a);
    const int diff = diffusion_on(P, b);
    const double lam = prop(P, P->lam_c, P->lam, i, j, k);

    for (int c = 0; c < 6; ++c) {
        double sx[7], sy[7], sz[7];
        for (int m = 0; m < 7; ++m) {
            sx[m] = Bc(P, B, c, i + m - 3, j, k);
            sy[m] = Bc(P, B, c, i, j + m - 3, k);
            sz[m] = Bc(P, B, c, i, j, k + m - 3);
        }
        double adv = uc * adv_upwind(P, sx, dx, uc) + vc * adv_upwind(P, sy, dy, vc)
                   + wc * adv_upwind(P, sz, dz, wc);
        int p = ia[c], q = ib[c];
        double ucv = 0.0;   /* (L.B + B.L^T)_pq */
        for (int m = 0; m < 3; ++m) ucv += L[p][m] * Bm[m][q] + Bm[p][m] * L[q][m];
        double relax = ((p == q ? a : 0.0) - F * b[c]) / lam;
        rt[c] = relax - adv + ucv;
        if (diff) {
            double lap = (sx[2] - 2.0 * sx[3] + sx[4]) / (dx * dx)
                       + (sy[2] - 2.0 * sy[3] + sy[4]) / (dy * dy)
                       + (sz[2] - 2.0 * sz[3] + sz[4]) / (dz * dz);
            rt[c] += P->kappa * lap;
        }
    }
}

/* Body force f_x on the x-face row j (Eq. NS, the term f). */
static double force_x(const oracle_params* P, int j)
{
    if (P->force_kind == 1) return P->force_amp;
    if (P->force_kind == 2) return P->force_amp * sin(P->force_ky * (P->y0 + (j + 0.5) * P->dy));
    return 0.0;
}

/* Viscous term div(mu_s (grad u + grad u^T)) of Eq. (ru) with a per-cell mu_s (two-phase
 * mixture): normal viscous stresses 2 mu du_a/dx_a at cell centres, shear stresses
 * mu (du_a/dx_b + du_b/dx_a) on cell edges with mu the average of the four cells around the edge;
 * the face value is their difference across the face. */
static double mu_c(const oracle_params* P, int i, int j, int k)
{
    return prop(P, P->mus_c, P->mu_s, i, j, k);
}

static void viscous_variable(const oracle_params* P, const double* u, const double* v,
                             const double* w, int i, int j, int k, double Vv[3])
{
    const double dx = P->dx, dy = P->dy, dz = P->dz;
    /* x-face (i+1/2, j, k) */
    {
        double t1 = 2.0 * mu_c(P, i + 1, j, k) * (U(P, u, i + 1, j, k) - U(P, u, i, j, k)) / dx;
        double t0 = 2.0 * mu_c(P, i, j, k) * (U(P, u, i, j, k) - U(P, u, i - 1, j, k)) / dx;
        double mT = 0.25 * (mu_c(P, i, j, k) + mu_c(P, i + 1, j, k) + mu_c(P, i, j + 1, k) + mu_c(P, i + 1, j + 1, k));
        double mB = 0.25 * (mu_c(P, i, j, k) + mu_c(P, i + 1, j, k) + mu_c(P, i, j - 1, k) + mu_c(P, i + 1, j - 1, k));
        double mF = 0.25 * (mu_c(P, i, j, k) + mu_c(P, i + 1, j, k) + mu_c(P, i, j, k + 1) + mu_c(P, i + 1, j, k + 1));
        double mK = 0.25 * (mu_c(P, i, j, k) + mu_c(P, i + 1, j, k) + mu_c(P, i, j, k - 1) + mu_c(P, i + 1, j, k - 1));
        double sT = mT * ((U(P, u, i, j + 1, k) - U(P, u, i, j, k)) / dy + (V(P, v, i + 1, j, k) - V(P, v, i, j, k)) / dx);
        double sB = mB * ((U(P, u, i, j, k) - U(P, u, i, j - 1, k)) / dy + (V(P, v, i + 1, j - 1, k) - V(P, v, i, j - 1, k)) / dx);
        double sF = mF * ((U(P, u, i, j, k + 1) - U(P, u, i, j, k)) / dz + (W(P, w, i + 1, j, k) - W(P, w, i, j, k)) / dx);
        double sK = mK * ((U(P, u, i, j, k) - U(P, u, i, j, k - 1)) / dz + (W(P, w, i + 1, j, k - 1) - W(P, w, i, j, k - 1)) / dx);
        Vv[0] = (t1 - t0) / dx + (sT - sB) / dy + (sF - sK) / dz;
    }
    /* y-face (i, j+1/2, k) */
    if (P->walls && j == P->ny - 1) {
        Vv[1] = 0.0;
    } else {
        double t1 = 2.0 * mu_c(P, i, j + 1, k) * (V(P, v, i, j + 1, k) - V(P, v, i, j, k)) / dy;
        double t0 = 2.0 * mu_c(P, i, j, k) * (V(P, v, i, j, k) - V(P, v, i, j - 1, k)) / dy;
        double mR = 0.25 * (mu_c(P, i, j, k) + mu_c(P, i + 1, j, k) + mu_c(P, i, j + 1, k) + mu_c(P, i + 1, j + 1, k));
        double mL = 0.25 * (mu_c(P, i, j, k) + mu_c(P, i - 1, j, k) + mu_c(P, i, j + 1, k) + mu_c(P, i - 1, j + 1, k));
        double mF = 0.25 * (mu_c(P, i, j, k) + mu_c(P, i, j + 1, k) + mu_c(P, i, j, k + 1) + mu_c(P, i, j + 1, k + 1));
        double mK = 0.25 * (mu_c(P, i, j, k) + mu_c(P, i, j + 1, k) + mu_c(P, i, j, k - 1) + mu_c(P, i, j + 1, k - 1));
        double sR = mR * ((U(P, u, i, j + 1, k) - U(P, u, i, j, k)) / dy + (V(P, v, i + 1, j, k) - V(P, v, i, j, k)) / dx);
        double sL = mL * ((U(P, u, i - 1, j + 1, k) - U(P, u, i - 1, j, k)) / dy + (V(P, v, i, j, k) - V(P, v, i - 1, j, k)) / dx);
        double sF = mF * ((V(P, v, i, j, k + 1) - V(P, v, i, j, k)) / dz + (W(P, w, i, j + 1, k) - W(P, w, i, j, k)) / dy);
        double sK = mK * ((V(P, v, i, j, k) - V(P, v, i, j, k - 1)) / dz + (W(P, w, i, j + 1, k - 1) - W(P, w, i, j, k - 1)) / dy);
        Vv[1] = (t1 - t0) / dy + (sR - sL) / dx + (sF - sK) / dz;
    }
    /* z-face (i, j, k+1/2) */
    {
        double t1 = 2.0 * mu_c(P, i, j, k + 1) * (W(P, w, i, j, k + 1) - W(P, w, i, j, k)) / dz;
        double t0 = 2.0 * mu_c(P, i, j, k) * (W(P, w, i, j, k) - W(P, w, i, j, k - 1)) / dz;
        double mR = 0.25 * (mu_c(P, i, j, k) + mu_c(P, i + 1, j, k) + mu_c(P, i, j, k + 1) + mu_c(P, i + 1, j, k + 1));
        double mL = 0.25 * (mu_c(P, i, j, k) + mu_c(P, i - 1, j, k) + mu_c(P, i, j, k + 1) + mu_c(P, i - 1, j, k + 1));
        double mT = 0.25 * (mu_c(P, i, j, k) + mu_c(P, i, j + 1, k) + mu_c(P, i, j, k + 1) + mu_c(P, i, j + 1, k + 1));
        double mB = 0.25 * (mu_c(P, i, j, k) + mu_c(P, i, j - 1, k) + mu_c(P, i, j, k + 1) + mu_c(P, i, j - 1, k + 1));
        double sR = mR * ((U(P, u, i, j, k + 1) - U(P, u, i, j, k)) / dz + (W(P, w, i + 1, j, k) - W(P, w, i, j, k)) / dx);
        double sL = mL * ((U(P, u, i - 1, j, k + 1) - U(P, u, i - 1, j, k)) / dz + (W(P, w, i, j, k) - W(P, w, i - 1, j, k)) / dx);
        double sT = mT * ((V(P, v, i, j, k + 1) - V(P, v, i, j, k)) / dz + (W(P, w, i, j + 1, k) - W(P, w, i, j, k)) / dy);
        double sB = mB * ((V(P, v, i, j - 1, k + 1) - V(P, v, i, j - 1, k)) / dz + (W(P, w, i, j, k) - W(P, w, i, j - 1, k)) / dy);
        Vv[2] = (t1 - t0) / dz + (sR - sL) / dx + (sT - sB) / dy;
    }
}

/* The three momentum terms of Eq. (ru) on the three faces owned by cell (i,j,k): A =
 * divergence-form advection div(uu), Vv = mu_s times the 7-point Laplacian, T = divergence of the
 * extra stress from centre and edge-averaged values.  The top wall face of a channel gets 0. */
static void momentum_parts(const oracle_params* P, const double* u, const double* v,
                           const double* w, const double* B, int i, int j, int k, double A[3],
                           double Vv[3], double T[3])
{
    const double dx = P->dx, dy = P->dy, dz = P->dz;
    const double ms = P->mu_s;
    double t00[6], t[6];

    /* ---- x-face (i+1/2, j, k) ---- */
    {
        double ucR = 0.5 * (U(P, u, i, j, k) + U(P, u, i + 1, j, k));
        double ucL = 0.5 * (U(P, u, i - 1, j, k) + U(P, u, i, j, k));
        double fxx = ucR * ucR - ucL * ucL;
        double vT = 0.5 * (V(P, v, i, j, k) + V(P, v, i + 1, j, k));
        double vB = 0.5 * (V(P, v, i, j - 1, k) + V(P, v, i + 1, j - 1, k));
        double uT = 0.5 * (U(P, u, i, j, k) + U(P, u, i, j + 1, k));
        double uB = 0.5 * (U(P, u, i, j - 1, k) + U(P, u, i, j, k));
        double wF = 0.5 * (W(P, w, i, j, k) + W(P, w, i + 1, j, k));
        double wK = 0.5 * (W(P, w, i, j, k - 1) + W(P, w, i + 1, j, k - 1));
        double uF = 0.5 * (U(P, u, i, j, k) + U(P, u, i, j, k + 1));
        double uK = 0.5 * (U(P, u, i, j, k - 1) + U(P, u, i, j, k));
        double adv = fxx / dx + (vT * uT - vB * uB) / dy + (wF * uF - wK * uK) / dz;
        double c0 = U(P, u, i, j, k);
        double lap = (U(P, u, i + 1, j, k) - 2.0 * c0 + U(P, u, i - 1, j, k)) / (dx * dx)
                   + (U(P, u, i, j + 1, k) - 2.0 * c0 + U(P, u, i, j - 1, k)) / (dy * dy)
                   + (U(P, u, i, j, k + 1) - 2.0 * c0 + U(P, u, i, j, k - 1)) / (dz * dz);
        /* divergence of tau at the x-face */
        stress_at(P, B, i, j, k, t00);
        stress_at(P, B, i + 1, j, k, t);
        double dtxx = (t[XX] - t00[XX]) / dx;
        double s[4];
        double e_top, e_bot, e_fr, e_bk;
        stress_at(P, B, i, j + 1, k, t); s[0] = t[XY];
        stress_at(P, B, i + 1, j + 1, k, t); s[1] = t[XY];
        stress_at(P, B, i + 1, j, k, t); s[2] = t[XY];
        e_top = 0.25 * (t00[XY] + s[0] + s[1] + s[2]);
        stress_at(P, B, i, j - 1, k, t); s[0] = t[XY];
        stress_at(P, B, i + 1, j - 1, k, t); s[1] = t[XY];
        e_bot = 0.25 * (t00[XY] + s[0] + s[1] + s[2]);
        stress_at(P, B, i, j, k + 1, t); s[0] = t[XZ];
        stress_at(P, B, i + 1, j, k + 1, t); s[1] = t[XZ];
        stress_at(P, B, i + 1, j, k, t); s[2] = t[XZ];
        e_fr = 0.25 * (t00[XZ] + s[0] + s[1] + s[2]);
        stress_at(P, B, i, j, k - 1, t); s[0] = t[XZ];
        stress_at(P, B, i + 1, j, k - 1, t); s[1] = t[XZ];
        e_bk = 0.25 * (t00[XZ] + s[0] + s[1] + s[2]);
        double divt = dtxx + (e_top - e_bot) / dy + (e_fr - e_bk) / dz;
        A[0] = adv; Vv[0] = ms * lap; T[0] = divt;
    }

    /* ---- y-face (i, j+1/2, k) ---- */
    if (P->walls && j == P->ny - 1) {
        A[1] = 0.0; Vv[1] = 0.0; T[1] = 0.0;   /* top wall face: no penetration */
    } else {
        double vcT = 0.5 * (V(P, v, i, j, k) + V(P, v, i, j + 1, k));
        double vcB = 0.5 * (V(P, v, i, j - 1, k) + V(P, v, i, j, k));
        double fyy = vcT * vcT - vcB * vcB;
        double uR = 0.5 * (U(P, u, i, j, k) + U(P, u, i, j + 1, k));
        double uL = 0.5 * (U(P, u, i - 1, j, k) + U(P, u, i - 1, j + 1, k));
        double vR = 0.5 * (V(P, v, i, j, k) + V(P, v, i + 1, j, k));
        double vL = 0.5 * (V(P, v, i - 1, j, k) + V(P, v, i, j, k));
        double wF = 0.5 * (W(P, w, i, j, k) + W(P, w, i, j + 1, k));
        double wK = 0.5 * (W(P, w, i, j, k - 1) + W(P, w, i, j + 1, k - 1));
        double vF = 0.5 * (V(P, v, i, j, k) + V(P, v, i, j, k + 1));
        double vK = 0.5 * (V(P, v, i, j, k - 1) + V(P, v, i, j, k));
        double adv = (uR * vR - uL * vL) / dx + fyy / dy + (wF * vF - wK * vK) / dz;
        double c0 = V(P, v, i, j, k);
        double lap = (V(P, v, i + 1, j, k) - 2.0 * c0 + V(P, v, i - 1, j, k)) / (dx * dx)
                   + (V(P, v, i, j + 1, k) - 2.0 * c0 + V(P, v, i, j - 1, k)) / (dy * dy)
                   + (V(P, v, i, j, k + 1) - 2.0 * c0 + V(P, v, i, j, k - 1)) / (dz * dz);
        stress_at(P, B, i, j, k, t00);
        stress_at(P, B, i, j + 1, k, t);
        double dtyy = (t[YY] - t00[YY]) / dy;
        double s[4], eR, eL, eF, eK;
        stress_at(P, B, i + 1, j, k, t); s[0] = t[XY];
        stress_at(P, B, i + 1, j + 1, k, t); s[1] = t[XY];
        stress_at(P, B, i, j + 1, k, t); s[2] = t[XY];
        eR = 0.25 * (t00[XY] + s[0] + s[1] + s[2]);
        stress_at(P, B, i - 1, j, k, t); s[0] = t[XY];
        stress_at(P, B, i - 1, j + 1, k, t); s[1] = t[XY];
        eL = 0.25 * (t00[XY] + s[0] + s[1] + s[2]);
        stress_at(P, B, i, j, k + 1, t); s[0] = t[YZ];
        stress_at(P, B, i, j + 1, k + 1, t); s[1] = t[YZ];
        stress_at(P, B, i, j + 1, k, t); s[2] = t[YZ];
        eF = 0.25 * (t00[YZ] + s[0] + s[1] + s[2]);
        stress_at(P, B, i, j, k - 1, t); s[0] = t[YZ];
        stress_at(P, B, i, j + 1, k - 1, t); s[1] = t[YZ];
        eK = 0.25 * (t00[YZ] + s[0] + s[1] + s[2]);
        double divt = (eR - eL) / dx + dtyy + (eF - eK) / dz;
        A[1] = adv; Vv[1] = ms * lap; T[1] = divt;
    }

    /* ---- z-face (i, j, k+1/2) ---- */
    {
        double wcF = 0.5 * (W(P, w, i, j, k) + W(P, w, i, j, k + 1));
        double wcK = 0.5 * (W(P, w, i, j, k - 1) + W(P, w, i, j, k));
        double fzz = wcF * wcF - wcK * wcK;
        double uR = 0.5 * (U(P, u, i, j, k) + U(P, u, i, j, k + 1));
        double uL = 0.5 * (U(P, u, i - 1, j, k) + U(P, u, i - 1, j, k + 1));
        double wR = 0.5 * (W(P, w, i, j, k) + W(P, w, i + 1, j, k));
        double wL = 0.5 * (W(P, w, i - 1, j, k) + W(P, w, i, j, k));
        double vT = 0.5 * (V(P, v, i, j, k) + V(P, v, i, j, k + 1));
        double vB = 0.5 * (V(P, v, i, j - 1, k) + V(P, v, i, j - 1, k + 1));
        double wT = 0.5 * (W(P, w, i, j, k) + W(P, w, i, j + 1, k));
        double wB = 0.5 * (W(P, w, i, j - 1, k) + W(P, w, i, j, k));
        double adv = (uR * wR - uL * wL) / dx + (vT * wT - vB * wB) / dy + fzz / dz;
        double c0 = W(P, w, i, j, k);
        double lap = (W(P, w, i + 1, j, k) - 2.0 * c0 + W(P, w, i - 1, j, k)) / (dx * dx)
                   + (W(P, w, i, j + 1, k) - 2.0 * c0 + W(P, w, i, j - 1, k)) / (dy * dy)
                   + (W(P, w, i, j, k + 1) - 2.0 * c0 + W(P, w, i, j, k - 1)) / (dz * dz);
        stress_at(P, B, i, j, k, t00);
        stress_at(P, B, i, j, k + 1, t);
        double dtzz = (t[ZZ] - t00[ZZ]) / dz;
        double s[4], eR, eL, eT, eB;
        stress_at(P, B, i + 1, j, k, t); s[0] = t[XZ];
        stress_at(P, B, i + 1, j, k + 1, t); s[1] = t[XZ];
        stress_at(P, B, i, j, k + 1, t); s[2] = t[XZ];
        eR = 0.25 * (t00[XZ] + s[0] + s[1] + s[2]);
        stress_at(P, B, i - 1, j, k, t); s[0] = t[XZ];
        stress_at(P, B, i - 1, j, k + 1, t); s[1] = t[XZ];
        eL = 0.25 * (t00[XZ] + s[0] + s[1] + s[2]);
        stress_at(P, B, i, j + 1, k, t); s[0] = t[YZ];
        stress_at(P, B, i, j + 1, k + 1, t); s[1] = t[YZ];
        stress_at(P, B, i, j, k + 1, t); s[2] = t[YZ];
        eT = 0.25 * (t00[YZ] + s[0] + s[1] + s[2]);
        stress_at(P, B, i, j - 1, k, t); s[0] = t[YZ];
        stress_at(P, B, i, j - 1, k + 1, t); s[1] = t[YZ];
        eB = 0.25 * (t00[YZ] + s[0] + s[1] + s[2]);
        double divt = (eR - eL) / dx + (eT - eB) / dy + dtzz;
        A[2] = adv; Vv[2] = ms * lap; T[2] = divt;
    }
    if (P->mus_c) viscous_variable(P, u, v, w, i, j, k, Vv);
}

/* Momentum right-hand side RU of Eq. (ru) (g = 0): RU = -A + (Vv + T + f + fs)/rho_face, with
 * the body force f on the x-faces, the extra face force fs (surface tension) and rho_face the
 * mean of the two cells beside the face (constant rho for a single phase). */
static void momentum_rhs(const oracle_params* P, const double* u, const double* v, const double* w,
                         const double* B, int i, int j, int k, double ru[3])
{
    double A[3], Vv[3], T[3], f[3] = { force_x(P, j), 0.0, 0.0 };
    momentum_parts(P, u, v, w, B, i, j, k, A, Vv, T);
    const double r0 = prop(P, P->rho_c, P->rho, i, j, k);
    const double rf[3] = { 0.5 * (r0 + prop(P, P->rho_c, P->rho, i + 1, j, k)),
                           0.5 * (r0 + prop(P, P->rho_c, P->rho, i, j + 1, k)),
                           0.5 * (r0 + prop(P, P->rho_c, P->rho, i, j, k + 1)) };
    if (P->fs) {
        const size_t n = (size_t)P->nx * P->ny * P->nz, q = at(P, i, j, k);
        for (int c = 0; c < 3; ++c) f[c] += P->fs[c * n + q];
    }
    for (int c = 0; c < 3; ++c)
        ru[c] = -A[c] + (Vv[c] + T[c] + f[c]) / (P->rho_c ? rf[c] : P->rho);
    if (P->walls && j == P->ny - 1) ru[1] = 0.0;
}

/*
 * Exported: the predictor of Sec. 3.2.2.  From u^n, B^n and the previous right-hand sides
 * computes RT^n (Eq. rt), B^{n+1} (Eq. ab2tau), RU^n (Eq. ru) and u* (Eq. ab2).  euler != 0
 * replaces the AB2 weights (3/2, -1/2) by (1, 0) (first step, no history).  freeze != 0 leaves
 * the velocity unchanged (u* = u^n, RU^n = 0): the paper's "uncoupled" homogeneous-shear test
 * of Sec. 4.1.3.  B_new, RT, us, vs, ws, RU must not alias the inputs.
 */
void oracle_predictor(const oracle_params* P, const double* u, const double* v, const double* w,
                      const double* B, const double* RT_old, const double* RU_old,
                      int euler, int freeze, double dt,
                      double* B_new, double* RT, double* us, double* vs, double* ws, double* RU)
{
    const int nx = P->nx, ny = P->ny, nz = P->nz;
    const size_t n = (size_t)nx * ny * nz;
    const double c1 = euler ? 1.0 : 1.5, c2 = euler ? 0.0 : -0.5;
    #pragma omp parallel for schedule(static)
    for (int k = 0; k < nz; ++k) {
        for (int j = 0; j < ny; ++j) {
            for (int i = 0; i < nx; ++i) {
                size_t q = at(P, i, j, k);
                double rt[6], ru[3];
                stress_rhs(P, u, v, w, B, i, j, k, rt);
                for (int c = 0; c < 6; ++c) {
                    RT[c * n + q] = rt[c];
                    B_new[c * n + q] = B[c * n + q] + dt * (c1 * rt[c] + c2 * RT_old[c * n + q]);
                }
                if (freeze) {
                    us[q] = u[q]; vs[q] = v[q]; ws[q] = w[q];
                    RU[q] = 0.0; RU[n + q] = 0.0; RU[2 * n + q] = 0.0;
                    continue;
                }
                momentum_rhs(P, u, v, w, B, i, j, k, ru);
                RU[q] = ru[0]; RU[n + q] = ru[1]; RU[2 * n + q] = ru[2];
                us[q] = u[q] + dt * (c1 * ru[0] + c2 * RU_old[q]);
                vs[q] = v[q] + dt * (c1 * ru[1] + c2 * RU_old[n + q]);
                ws[q] = w[q] + dt * (c1 * ru[2] + c2 * RU_old[2 * n + q]);
                if (P->walls && j == ny - 1) vs[q] = 0.0;
            }
        }
    }
}

/*
 * Exported for the Runge-Kutta integrator of Sec. 3.3.1: the separate terms of Eqs. (RK-rt) and
 * (NS-num1) at one state, on every cell.
 *   RT: the bracket of Eq. (RK-rt) (the right-hand side of Eq. SRM2), six planes;
 *   A : the advection term div(uu) on the three faces of each cell, three planes;
 *   V : mu_s times the 7-point Laplacian of the face velocities, three planes;
 *   T : div(tau) on the faces (centre and edge-averaged stresses), three planes.
 * The top wall face of a channel gets 0 in A, V and T.
 */
void oracle_terms(const oracle_params* P, const double* u, const double* v, const double* w,
                  const double* B, double* RT, double* A, double* V, double* T)
{
    const int nx = P->nx, ny = P->ny, nz = P->nz;
    const size_t n = (size_t)nx * ny * nz;
    #pragma omp parallel for schedule(static)
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                const size_t q = at(P, i, j, k);
                double rt[6], a[3], vv[3], t[3];
                stress_rhs(P, u, v, w, B, i, j, k, rt);
                for (int c = 0; c < 6; ++c) RT[c * n + q] = rt[c];
                momentum_parts(P, u, v, w, B, i, j, k, a, vv, t);
                for (int c = 0; c < 3; ++c) {
                    A[c * n + q] = a[c]; V[c * n + q] = vv[c]; T[c * n + q] = t[c];
                }
            }
}
