// Internal declarations of libevp.so: the per-grid device descriptor, the batch argument block
// passed by value to every kernel, and the host-side launchers of each kernel family.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

#include "../../include/evp.h"

namespace evp {

// Per-grid constants and pointers.  Lives at the start of the grid's workspace (device) and is
// mirrored in the host-side grid; kernels read it through a uniform pointer (scalar loads).
struct Desc {
    int nx, ny, nz, nh;          // cells; nh = nx/2 + 1 complex values per x-spectrum line
    int walls;                   // EVP_WALLS in y?
    int precision;               // EVP_FP64 or EVP_MIXED
    int model;                   // EVP_OLDROYD_B / EVP_FENE_P / EVP_SARAMITO / EVP_NEO_HOOKEAN
    int force_kind;              // EVP_FORCE_*
    int adv;                     // EVP_WENO5 / EVP_HOUC5
    int sh;                      // row stride of the half spectrum and the pivots: nh rounded up
                                 // to 8 complex values, so every row starts on a 128-byte line
    double kappa;                // artificial diffusion coefficient (0: off)
    const double* alpha[3];      // solid volume fractions at u, v, w points (caller's; null: none)
    // two-phase (bubbly-flow) mode, Sec. 3.2: properties of fluid 1 (phi > 0) and fluid 2, the
    // surface tension, the interface half-width eps of H(phi), rho_0 = min(rho1, rho2), and the
    // level-set fields in the caller's second workspace (null when off)
    int two_phase;
    double rho1, rho2, mus1, mus2, mup1, mup2, lam1, lam2, sigma, eps_if, rho0;
    double *phi, *phi1, *phi2, *sgn, *kap, *p_old, *p_hat;
    long long ncell;             // nx*ny*nz
    long long ps;                // element stride between planes of B, RT, RU (256-byte padded)
    double dx, dy, dz, idx, idy, idz, y0;
    double rho, inv_rho, mu_s, mu_p, lam, inv_lam, G, tau_y, L2, a_fene;
    double force_amp, force_ky;
    double u_bot, u_top, w_bot, w_top;
    double *u, *v, *w;           // velocity u^n (FP64)
    double *us, *vs, *ws;        // predicted velocity u* (FP64)
    void* Bt[2];                 // B - I, six planes each, ping-pong (double or float)
    void* RT;                    // stress right-hand side history, six planes (double or float)
    void* RU;                    // momentum right-hand side history, three planes
    double* p;                   // pressure
    double2* spec;               // half spectrum [nz][ny][sh] (kx < nh used)
    const double2 *twx, *twy, *twz;        // W_N^n = exp(-2 pi i n / N), n < N, per direction
    const double *eigx, *eigy, *eigz;      // -(4/h^2) sin^2(pi k / N) per direction
    const double* piv;           // walls: Thomas pivots 1/(b_j - a c'_{j-1}) [nz/2+1][ny][sh]
    const int* pvj;              // walls, per 64-mode wave of the Thomas solve: the row from which
                                 // every pivot of its modes below row ny-1 equals row ny-2's
    double* red;                 // reduction partials (health)
    double* gauge;               // walls: volume mean of p before the zero-mean gauge (one value)
};

// Argument block of every batched kernel (by value; < 1 KiB).
struct Batch {
    const Desc* d[EVP_MAX_BATCH];
    double dt[EVP_MAX_BATCH];
    int state[EVP_MAX_BATCH];    // bit 0: index of the current B buffer; bit 1: no history term
    int count;
    double rk[3];                // Runge-Kutta substep: zeta, xi, alpha (Eq. RK); unused by AB2
};

// Pointers into the workspace as global-memory (address space 1) pointers: accesses through them
// compile to global_* instructions, which count only against the vector-memory counter, so a
// wait for LDS results does not also wait for global loads in flight (flat instructions, which
// generic pointers produce, count against both).
#define EVP_GLOBAL __attribute__((address_space(1)))
template <typename T> using gptr = EVP_GLOBAL T*;

constexpr int ST_PARITY = 1;
constexpr int ST_EULER = 2;
constexpr int ST_PZERO = 4;      // two-phase: no pressure history yet (2 p^n - p^{n-1} := 0)
constexpr int ST_REINIT = 8;     // two-phase: this grid reinitialises its level set now

// Host-side launchers (one per kernel family); shape is common to the whole batch.
// A second stream with a fork and a join event: work launched there runs beside the main
// stream's and is joined back before the main stream goes on.
struct Side { hipStream_t s; hipEvent_t fork, join; };
hipError_t launch_predictor_zm(const Batch& b, int precision, int nx, int ny, int nz, bool freeze,
                               hipStream_t s, bool walls, int model, bool rk3, bool houc,
                               bool two_phase, const Side* side = nullptr);
// two-phase path (k_two_phase.hip)
hipError_t launch_level_set_stage(const Batch& b, int nx, int ny, int nz, bool walls, bool reinit,
                                  int stage, hipStream_t s);
hipError_t launch_reinit_sign(const Batch& b, int nx, int ny, int nz, hipStream_t s);
hipError_t launch_curvature(const Batch& b, int nx, int ny, int nz, bool walls, hipStream_t s);
hipError_t launch_momentum_two_phase(const Batch& b, int nx, int ny, int nz, bool walls, int model,
                                     bool freeze, hipStream_t s);
hipError_t launch_split_pressure(const Batch& b, int nx, int ny, int nz, bool walls, hipStream_t s);
hipError_t launch_fill(double* p, long long n, double value, hipStream_t s);
hipError_t launch_stress_div(const Batch& b, int precision, int nx, int ny, int nz, bool walls,
                             hipStream_t s);
hipError_t launch_penalise(const Batch& b, int nx, int ny, int nz, hipStream_t s);
hipError_t launch_div_fftx(const Batch& b, int nx, int ny, int nz, hipStream_t s);
// periodic grids with nx == ny <= 128 and at least 256 z planes over the batch: divergence + x
// and y transforms, and inverse y and x transforms, one block per z plane with the plane's half
// spectrum in LDS
bool plane_transforms(int nx, int ny, int nz, int count);
hipError_t launch_div_fftxy(const Batch& b, int n, int nz, hipStream_t s);
hipError_t launch_ifftxy(const Batch& b, int n, int nz, hipStream_t s);
hipError_t launch_fft_strided(const Batch& b, int nx, int ny, int nz, int axis, bool inverse,
                              hipStream_t s);
hipError_t launch_solve_periodic(const Batch& b, int nx, int ny, int nz, hipStream_t s);
hipError_t launch_thomas(const Batch& b, int nx, int ny, int nz, hipStream_t s);
hipError_t launch_ifftx(const Batch& b, int nx, int ny, int nz, hipStream_t s);
hipError_t launch_correct(const Batch& b, int nx, int ny, int nz, hipStream_t s);
hipError_t launch_copy_ustar(const Batch& b, int nx, int ny, int nz, bool to_u, hipStream_t s);
hipError_t launch_write_fields(const Desc* d, int precision, long long ncell, int ny, int nx,
                               int walls, int parity, const double* u, const double* v,
                               const double* w, const double* B6, const double* hist,
                               hipStream_t s);
hipError_t launch_read_fields(const Desc* d, int precision, long long ncell, int parity,
                              unsigned mask, double* u, double* v, double* w, double* p,
                              double* B6, double* hist, hipStream_t s);
hipError_t launch_health(const Desc* d, int precision, int parity, double* out5, hipStream_t s);

// Guard words after every region of a workspace: a fixed 64-bit pattern, a quiet NaN, so that a
// stray read of one also shows up as a non-finite value.  table: n pairs (byte offset from ws,
// number of 8-byte words), in device memory.  The check writes the number of words that no
// longer hold the pattern to *out (as a double).
constexpr unsigned long long kGuardWord = 0x7FF8DEADC0DE5AFEull;
hipError_t launch_guard_fill(char* ws, const long long* table, int n, hipStream_t s);
hipError_t launch_guard_check(const char* ws, const long long* table, int n, double* out, hipStream_t s);

bool fft_size_supported(int n);

}  // namespace evp
