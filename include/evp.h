/*
 * evp.h -- C-ABI of libevp.so: one time step of incompressible flow of an Oldroyd-B, FENE-P or
 * Saramito elastoviscoplastic fluid on a uniform staggered grid, on one MI355X (gfx950).
 *
 * The method is the single-phase Eulerian part of Izbassarov et al., "Computational modeling of
 * multiphase viscoelastic and elastoviscoplastic flows":
 *   - unknowns u, p and the conformation tensor B of Sec. 2, Eqs. (mainNS) and (SRM2);
 *   - the closures F, a and the B <-> tau relation of Table 1 (Oldroyd-B, FENE-P, Saramito,
 *     Neo-Hookean);
 *   - the staggered grid and differences of Sec. 3 (velocities on faces; p and B at centres;
 *     second-order central differences; fifth-order WENO or HOUC for u.grad(B), Sec. 3 and
 *     3.1; optional local artificial diffusion of B, Sec. 3.1);
 *   - the Adams-Bashforth step and Chorin projection of Sec. 3.2.2, Eqs. (ab2tau), (ab2), (rt),
 *     (ru), (var poisson), (projection), with constant rho, g = 0 and f a body force; the pressure
 *     equation is solved with FFTs in periodic directions and a tridiagonal solve across walls;
 *   - fixed obstacles by the volume-penalisation immersed boundary of Sec. 3.3.2, Eqs. (Vol) and
 *     (forceAdded);
 *   - two-phase (bubbly) flow, Sec. 3.2: a level set transported by Eq. (ls adv) and
 *     reinitialised by Eq. (reinit), mixture properties (Eq. mat prop), the surface-tension force
 *     of Eq. (fLS) and the pressure splitting of Eq. (poisson LS);
 *   - alternatively the low-storage three-substep Runge-Kutta step of Sec. 3.3.1, Eqs. (RK-rt),
 *     (NS-num1), (rk3tau), (rk3), (NS-num2), (NS-num3), with the coefficients of Eq. (RK).
 *
 * Conventions shared by every call
 *   - Status: 0 (EVP_OK) or a negative EVP_ERR_* code.  No call throws, aborts or prints;
 *     evp_last_error() returns a thread-local text describing the last failure.
 *   - Memory: the caller owns all device memory (the workspace and every I/O buffer); the library
 *     never allocates or frees device memory.  It owns only the opaque host-side evp_grid, and
 *     one fixed-size static device array per GPU for evp_create_grid_static.
 *   - Streams: every call enqueues work on the HIP stream given at creation (or by
 *     evp_set_stream) and returns without waiting, except evp_health and evp_profile_read,
 *     which wait for the stream.  The caller synchronises before reading output buffers.
 *   - I/O arrays are device pointers to dense FP64 arrays [nz][ny][nx] (x fastest) in every
 *     precision mode.  u[k][j][i] is the x-velocity on the +x face of cell (i,j,k) (x = (i+1)dx,
 *     y = y0 + (j+1/2)dy, z = (k+1/2)dz); v and w sit on the +y and +z faces likewise; p and the
 *     six planes of B (order xx, xy, xz, yy, yz, zz) sit at cell centres.  With walls, y0 =
 *     -ly/2, the bottom wall face is implicit and v[k][ny-1][i] is the top wall face (always 0);
 *     periodic y has y0 = 0.
 */
#ifndef EVP_H
#define EVP_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define EVP_OK             0
#define EVP_ERR_ARG       -1   /* bad size, spacing, parameter, pointer or flag */
#define EVP_ERR_WORKSPACE -2   /* workspace too small or not 256-byte aligned */
#define EVP_ERR_STATE     -3   /* step/project/read before set_rheology or write_fields */
#define EVP_ERR_SHAPE     -4   /* grids of one batch differ in shape, precision, stream or
                                  time integrator */
#define EVP_ERR_HIP       -5   /* a HIP runtime call or kernel launch failed */
#define EVP_ERR_DISABLED  -6   /* the entry point is compiled but switched off (see its comment) */

/* boundary condition in y */
#define EVP_PERIODIC 0         /* periodic in x, y, z */
#define EVP_WALLS    1         /* periodic in x, z; no-slip walls at y = -ly/2 and y = +ly/2 */

/* precision of the stress transport and momentum stencils (the projection is always FP64) */
#define EVP_FP64  0
#define EVP_MIXED 1            /* B - I, RT, RU stored and computed in FP32; u, u*, p in FP64 */

/* constitutive models, Table 1 */
#define EVP_OLDROYD_B 0
#define EVP_FENE_P    1
#define EVP_SARAMITO  2
#define EVP_NEO_HOOKEAN 3      /* elastic solid: F = a = 0, G = mu_p / lambda (Table 1) */

/* advection scheme for u.grad(B) (Sec. 3) */
#define EVP_WENO5 0            /* fifth-order WENO (default) */
#define EVP_HOUC5 1            /* fifth-order upstream-central (linear) */

/* body force f of Eq. (NS) */
#define EVP_FORCE_NONE       0
#define EVP_FORCE_CONST_X    1 /* f_x = amp */
#define EVP_FORCE_SIN_X_OF_Y 2 /* f_x = amp * sin(ky * y), sampled at the u-face y */

/* time integrators (evp_set_integrator) */
#define EVP_AB2 0              /* Adams-Bashforth, Sec. 3.2.2 (default) */
#define EVP_RK3 1              /* low-storage Runge-Kutta, three substeps, Sec. 3.3.1 */

/* evp_step flags */
#define EVP_FREEZE_VELOCITY      1u  /* advance B only, u unchanged: the "uncoupled" shear test
                                        of Sec. 4.1.3 */
#define EVP_STOP_AFTER_PREDICTOR 2u  /* skip the projection: u <- u* (stage check; AB2 only) */

/* evp_read_fields mask bits */
#define EVP_READ_U    1u
#define EVP_READ_V    2u
#define EVP_READ_W    4u
#define EVP_READ_P    8u
#define EVP_READ_B   16u
#define EVP_READ_HIST 32u

/* largest batch of evp_step_batch */
#define EVP_MAX_BATCH 32

/* kernel classes reported by evp_profile_read */
#define EVP_K_PREDICTOR 0      /* fused stress + momentum stencil */
#define EVP_K_DIV_FFTX  1      /* Poisson right-hand side + forward x transform */
#define EVP_K_FFT_FWD   2      /* forward transform along y (periodic) or z (walls) */
#define EVP_K_SOLVE     3      /* z transform + spectral division (periodic) / Thomas (walls) */
#define EVP_K_FFT_INV   4      /* inverse transform along y (periodic) or z (walls) */
#define EVP_K_IFFTX     5      /* inverse x transform -> p */
#define EVP_K_CORRECT   6      /* u = u* - (dt/rho) grad p */
#define EVP_K_STRESS_DIV 7     /* RK3: u* += dt (alpha/rho) div tau(B^k) */
#define EVP_K_PENALISE  8      /* AB2 with a solid: u** = (1 - alpha) u* */
#define EVP_K_LEVEL_SET 9      /* two-phase: level-set transport stages (TVD-RK3) */
#define EVP_K_REINIT    10     /* two-phase: reinitialisation stages */
#define EVP_K_CURVATURE 11     /* two-phase: interface curvature at cell centres */
#define EVP_K_MOMENTUM2 12     /* two-phase: momentum with mixture properties and surface tension */
#define EVP_K_SPLIT     13     /* two-phase: pressure extrapolation and split velocity update */
#define EVP_K_COUNT     14

typedef struct evp_grid evp_grid;

/* Two-phase (bubbly-flow) parameters, Sec. 3.2: fluid 1 where the level set phi > 0 (the bulk),
 * fluid 2 where phi < 0 (bubbles or drops).  rho_k > 0, mu_s_k >= 0, mu_p_k >= 0, lam_k > 0,
 * sigma >= 0; the level set is reinitialised every reinit_every steps with reinit_iters
 * pseudo-time iterations (either 0: never). */
typedef struct {
    double rho1, rho2, mu_s1, mu_s2, mu_p1, mu_p2, lam1, lam2, sigma;
    int reinit_every, reinit_iters;
} evp_two_phase_t;

typedef struct {
    long long nonfinite;   /* cells where B or a velocity component is not finite */
    long long det_le0;     /* cells with det(B) <= 0 (loss of positive definiteness, Sec. 3.1) */
    long long trace_ge95;  /* FENE-P cells with tr(B) >= 0.95 L^2 (Sec. 3.1); 0 for other models */
    double max_div;        /* max |D_h u| over cells */
    double energy;         /* 1/2 sum(u^2 + v^2 + w^2) dx dy dz over faces */
    long long guard_bad;   /* workspace guard words no longer holding their pattern (a write past
                              the end of a region); 0 on a sound grid */
} evp_health_t;

typedef struct {
    long long launches[EVP_K_COUNT];  /* launches timed since evp_profile(g, 1) */
    double ms[EVP_K_COUNT];           /* summed HIP-event time per kernel class, milliseconds */
} evp_profile_t;

/* Text for a status code (static storage). */
const char* evp_error_string(int status);

/* Thread-local description of the most recent failure on this thread ("" if none). */
const char* evp_last_error(void);

/* Bytes of device workspace a grid of this shape needs (0 if the arguments are invalid).
 * nx, nz (FFT directions): 2^a, 3 2^a, 5 2^a or 15 2^a in [8, 512] (8, 10, 12, 16, 20, 24, 30, 32,
 * 40, 48, 60, 64, 80, 96, 120, 128, 160, 192, 240, 256, 320, 384, 480, 512); ny: one of the same
 * sizes when bc_y is EVP_PERIODIC, 4..1024 (any) with EVP_WALLS. */
size_t evp_workspace_bytes(int nx, int ny, int nz, int bc_y, int precision);

/* Guard regions of the workspace layout of a grid of this shape (a check for out-of-bounds writes,
 * not part of the method): every region of the workspace is followed by 8-byte guard words that
 * evp_create_grid fills with a fixed pattern and evp_health counts in guard_bad when they no longer
 * hold it.  Writes up to max (byte offset from the workspace start, number of words) pairs into
 * offsets[] and words[] (host memory, owned by the caller) and returns the number of regions, or
 * EVP_ERR_ARG for an invalid shape.  Host only. */
int evp_guard_regions(int nx, int ny, int nz, int bc_y, int precision, long long* offsets,
                      long long* words, int max);

/* Create a grid of nx x ny x nz cells in a box lx x ly x lz.  dev_workspace: device memory of at
 * least evp_workspace_bytes() bytes, 256-byte aligned, owned by the caller and kept alive until
 * evp_destroy_grid.  hip_stream: a hipStream_t (NULL = the null stream).  On success *out holds a
 * new grid with u = 0, B = I, p = 0, no rheology set.  Enqueues table uploads on the stream. */
int evp_create_grid(int nx, int ny, int nz, double lx, double ly, double lz, int bc_y,
                    int precision, void* dev_workspace, size_t workspace_bytes, void* hip_stream,
                    evp_grid** out);

/* Size of the library's static device workspace (64 MiB per GPU), see evp_create_grid_static. */
#define EVP_STATIC_WORKSPACE_BYTES (64u << 20)

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): evp_create_grid with the workspace taken from a device
 * array inside the library instead of the caller's.  The array holds EVP_STATIC_WORKSPACE_BYTES
 * on every GPU the library runs on, until the process ends; a grid needing more
 * (evp_workspace_bytes > EVP_STATIC_WORKSPACE_BYTES, e.g. beyond about 64^3 in EVP_FP64) is
 * rejected with EVP_ERR_WORKSPACE.  The grid lives on the current device (which must be the
 * stream's).  One such grid per device at a time: while it exists another call on that device
 * returns EVP_ERR_STATE; evp_destroy_grid waits for its stream and frees the slot.  The state is
 * cleared on creation (u = 0, B = I, p = 0), whatever an earlier grid left there.  All other calls
 * work on it as on any grid; it calls no hipMalloc/hipFree, and a channel grid in EVP_MIXED runs
 * the predictor's wall rows on its own stream (no side stream is created).  Work that other
 * code enqueues on that device's static workspace would race with it; only this entry point uses
 * it.  Enqueues a fill kernel and table uploads, and waits for the stream. */
int evp_create_grid_static(int nx, int ny, int nz, double lx, double ly, double lz, int bc_y,
                           int precision, void* hip_stream, evp_grid** out);

/* Change the stream later calls enqueue on (the caller orders it after earlier work). */
int evp_set_stream(evp_grid* g, void* hip_stream);

/* Material of Eq. (NS) and Table 1: density rho > 0, solvent viscosity mu_s >= 0, polymer
 * viscosity mu_p >= 0, relaxation time lambda > 0, yield stress tau_y >= 0 (Saramito only),
 * extensibility L2 > 3 (FENE-P only).  Neo-Hookean: shear modulus G = mu_p / lambda (lambda
 * enters nowhere else). */
int evp_set_rheology(evp_grid* g, int model, double rho, double mu_s, double mu_p, double lambda,
                     double tau_y, double L2);

/* Stress transport options: the advection scheme (EVP_WENO5 or EVP_HOUC5, Sec. 3) and the
 * coefficient kappa >= 0 of the local artificial diffusion of Sec. 3.1, kappa lap(B) added to the
 * right-hand side of Eq. (SRM2) in cells where det B < 0 or (FENE-P) tr B >= 0.95 L^2, judged on
 * the state at the start of the step (kappa = 0: off, the default). */
int evp_set_transport(evp_grid* g, int scheme, double kappa);

/* Fixed obstacles (Sec. 3.3.2, volume-penalisation immersed boundary): alpha_u, alpha_v, alpha_w
 * are the solid volume fractions (0 fluid .. 1 solid) around the u-, v- and w-points, dense FP64
 * device arrays [nz][ny][nx] owned by the caller and read by every later step until replaced, so
 * they must stay valid and unchanged while set.  Each step then uses u** = (1 - alpha) u* (Eq.
 * forceAdded, solid velocity 0) in place of the predicted velocity u*; under RK3 the fraction
 * multiplies the prediction from the momentum terms (the projection then yields p^k).  All three
 * NULL removes the obstacle; values are not checked. */
int evp_set_solid(evp_grid* g, const double* alpha_u, const double* alpha_v, const double* alpha_w);

/* Bytes of the second device workspace a two-phase grid of this shape needs (0 if invalid). */
size_t evp_two_phase_bytes(int nx, int ny, int nz);

/* Switch the grid to the two-phase path of Sec. 3.2 (tp != NULL) or back to a single phase
 * (tp == NULL).  dev_workspace: device memory of evp_two_phase_bytes() bytes, 256-byte aligned,
 * owned by the caller and kept alive while the mode is on.  Requires EVP_FP64 and the AB2
 * integrator, and no solid.  Each step then: advances phi with u^n (TVD-RK3, WENO5) and
 * reinitialises it on schedule; takes rho, mu_s, mu_p, lambda from phi^{n+1} (linear in a
 * regularised Heaviside, Eq. mat prop; model, tau_y and L2 of evp_set_rheology hold in both
 * phases); advances B (per-cell lambda) and u* (variable-viscosity stress, surface tension
 * sigma kappa delta(phi) n, 1/rho at the faces, Eq. ru); projects with the splitting of Eq.
 * (poisson LS) around rho_0 = min(rho1, rho2).  The level set starts at phi = 1 (all fluid 1);
 * write it with evp_write_level_set.  The pressure history restarts (2 p^n - p^{n-1} := 0) after
 * evp_write_fields or evp_project.
 * SWITCHED OFF: with tp != NULL this returns EVP_ERR_DISABLED and changes nothing.  The first
 * device run of the two-phase step ended in a memory fault whose cause has not been identified
 * (bounds-checked CPU emulation of its kernels stays in bounds), so its kernels are compiled but
 * not launched; tp == NULL (single phase) works as described. */
int evp_set_two_phase(evp_grid* g, const evp_two_phase_t* tp, void* dev_workspace, size_t bytes);

/* Level set phi at cell centres (FP64 device array [nz][ny][nx]): load, or copy out. */
int evp_write_level_set(evp_grid* g, const double* phi);
int evp_read_level_set(evp_grid* g, double* phi);

/* Body force f of Eq. (NS), one of EVP_FORCE_*. */
int evp_set_forcing(evp_grid* g, int kind, double amp, double ky);

/* Wall velocities (EVP_WALLS only): x- and z-velocity of the bottom (y = -ly/2) and top walls,
 * the no-slip condition of the wall-bounded validation cases of Sec. 4 (walls at rest in the
 * Poiseuille flow of Sec. 4.1.1, the default; walls moving in opposite directions in the plane
 * Couette flow of the suspension case, Sec. 4.2).  The ghost velocities beyond a wall are
 * reflected about these values.  EVP_ERR_ARG on a periodic grid or for non-finite values. */
int evp_set_walls(evp_grid* g, double u_bot, double u_top, double w_bot, double w_top);

/* Load the state: u, v, w (FP64 device arrays, layout above), B6 (six FP64 planes).  hist, if not
 * NULL, holds the nine planes RT_xx..RT_zz, RU_x, RU_y, RU_z of the previous step (Eqs. rt, ru) so
 * that the next step is a full AB2 step; with NULL the history is cleared and the next step is a
 * forward-Euler start.  With walls v on the top wall face is forced to 0.  Pointers are read on
 * the stream; they must stay valid until it reaches this point. */
int evp_write_fields(evp_grid* g, const double* u, const double* v, const double* w,
                     const double* B6, const double* hist);

/* Project the current velocity onto discretely divergence-free fields (Eqs. var poisson and
 * projection with u* = u and dt = 1); p is set to the potential removed. */
int evp_project(evp_grid* g);

/* Time integrator of later evp_step calls: EVP_AB2 (default) or EVP_RK3.  A change of scheme
 * clears the AB2 history, so the first AB2 step after RK3 steps is a forward-Euler start.  Host
 * state only; enqueues nothing. */
int evp_set_integrator(evp_grid* g, int scheme);

/* Advance nsteps steps of size dt > 0.  AB2 (Sec. 3.2.2): predictor (stress transport, Eq.
 * ab2tau; momentum, Eq. ab2), then the Poisson solve and the velocity correction.  RK3 (Sec.
 * 3.3.1): three substeps k = 1, 2, 3, each B^k from Eq. (rk3tau), u* from Eq. (rk3) and the
 * projection of Eqs. (NS-num2), (NS-num3) with 2 alpha_k dt; p is p^k = p^{k-1} + psi^k.  flags:
 * EVP_FREEZE_VELOCITY, EVP_STOP_AFTER_PREDICTOR (AB2 only: EVP_ERR_ARG under RK3). */
int evp_step(evp_grid* g, double dt, int nsteps, unsigned flags);

/* The same for count <= EVP_MAX_BATCH grids of identical shape, boundary type, precision,
 * stream and time integrator, each with its own rheology, forcing, walls and state: every kernel is launched once for
 * the whole batch.  Results are identical to count separate evp_step calls. */
int evp_step_batch(evp_grid* const* grids, int count, double dt, int nsteps, unsigned flags);

/* Copy the selected fields (mask of EVP_READ_*) into FP64 device arrays (NULL for unselected):
 * u, v, w, p: one plane each; B6: six planes; hist: nine planes as in evp_write_fields. */
int evp_read_fields(evp_grid* g, unsigned mask, double* u, double* v, double* w, double* p,
                    double* B6, double* hist);

/* Bytes of an opaque checkpoint of this grid's state (u, v, w, p, B, AB2 history, step count). */
size_t evp_state_bytes(const evp_grid* g);

/* Copy the state, bit for bit, into dst (device memory of evp_state_bytes() bytes, 256-byte
 * aligned, owned by the caller).  Waits for the stream before returning. */
int evp_save_state(evp_grid* g, void* dst, size_t bytes);

/* Restore a state saved from a grid of the same shape, boundary type and precision; the next
 * step continues exactly as the saved grid would have.  Waits for the stream. */
int evp_load_state(evp_grid* g, const void* src, size_t bytes);

/* Diagnostics of the current state; waits for the stream, *out is host memory.  The counts
 * follow the trigger conditions of the local artificial diffusion of Sec. 3.1; guard_bad counts
 * overwritten workspace guard words (see evp_guard_regions). */
int evp_health(evp_grid* g, evp_health_t* out);

/* evp_health without waiting: enqueues the same diagnostics (all but guard_bad) on the grid's
 * stream and writes the five values, as doubles in the order nonfinite, det_le0, trace_ge95,
 * max_div, energy, into out5
 * (device memory of 5 doubles, owned by the caller).  out5 is valid once the stream has passed
 * this point (e.g. an event recorded after the call).  Same numbers as evp_health: the reduction
 * sums in a fixed order. */
int evp_health_enqueue(evp_grid* g, double* out5);

/* Steps taken since the last evp_write_fields (AB2 bookkeeping). */
int evp_step_count(evp_grid* g, long long* out);

/* Turn per-kernel HIP-event timing on (1, counters reset) or off (0).  While on, every kernel
 * launch of evp_step/evp_step_batch is bracketed by events on the grid's stream. */
int evp_profile(evp_grid* g, int enable);

/* Sum the recorded kernel times (waits for the stream). */
int evp_profile_read(evp_grid* g, evp_profile_t* out);

/* Release the host-side grid (the workspace stays the caller's).  NULL is accepted. */
int evp_destroy_grid(evp_grid* g);

#ifdef __cplusplus
}
#endif

#endif /* EVP_H */
