"""ORACLE -- test infrastructure only.  Only tests/, the smoke check and the CPU-baseline leg of the
benchmark may use this module.  It shares no code with the HIP path.

Two-phase (bubbly-flow) Eulerian path of Izbassarov et al., Sec. 3.2, in plain numpy on top of the
single-phase oracle:
  - level-set transport, Eq. (ls adv), with fifth-order WENO and the three-stage TVD Runge-Kutta
    scheme of Shu & Osher named in Sec. 3.2.1;
  - reinitialisation, Eq. (reinit), with the mollified sign function, every few steps;
  - mixture properties rho, mu_s, mu_p, lambda linear in a regularised Heaviside H(phi),
    Eq. (mat prop);
  - the continuum-surface-force term sigma kappa delta(phi) n, Eqs. (fLS), (normal), (curv);
  - the AB2 step of Sec. 3.2.2 with properties at the new level, Eq. (ru);
  - the pressure splitting of Dong & Shen, Eq. (poisson LS) and the matching velocity correction.

Readings of points the paper leaves open (listed with reasons in the design notes):
  H(phi) = 0 below -eps, 1 above eps, (1 + phi/eps + sin(pi phi/eps)/pi)/2 between, with
  eps = 1.5 max(dx, dy, dz); level-set ghost rows beyond a wall by linear extrapolation (as for
  B); reinitialisation with pseudo-time step 0.5 min(dx, dy, dz), sign S = phi0 / sqrt(phi0^2 +
  h^2) with h = min(dx, dy, dz) and Godunov upwinding of |grad phi| on WENO5 one-sided
  derivatives; no interface mass correction (the cited correction step is not given);
  delta(phi) n taken as grad H(phi) on the faces (equal for a signed-distance phi), kappa at cell
  centres as -div(n) with n = grad phi / |grad phi| from central differences, averaged to the
  faces; face density the mean of the two cells, edge viscosity the mean of four; properties of
  ghost rows copy the adjacent interior row; rho_0 = min(rho_1, rho_2); the pressure
  extrapolation 2 p^n - p^{n-1} starts from p = 0 after fields are written.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np

from . import (FORCE_NONE, Grid, Rheology, Solver, divergence, gradient, solve_poisson)


@dataclass
class TwoPhase:
    """Properties of fluid 1 (phi > 0, the bulk) and fluid 2 (phi < 0, bubbles or drops), the
    surface tension sigma and the reinitialisation schedule (every `reinit_every` steps,
    `reinit_iters` pseudo-time iterations; 0 = never)."""
    rho1: float = 1.0
    rho2: float = 1.0
    mu_s1: float = 0.0
    mu_s2: float = 0.0
    mu_p1: float = 0.0
    mu_p2: float = 0.0
    lam1: float = 1.0
    lam2: float = 1.0
    sigma: float = 0.0
    reinit_every: int = 10
    reinit_iters: int = 2


# ----------------------------------------------------------------------------------------------
# centre fields with ghost cells
# ----------------------------------------------------------------------------------------------

def pad(g: Grid, f, m=3):
    """Centre field with m ghost cells on every side: periodic in x and z; in y periodic or, with
    walls, linear extrapolation of the two nearest interior rows (ghost g: (1+g) f0 - g f1)."""
    f = np.pad(f, ((m, m), (0, 0), (m, m)), mode="wrap")
    if not g.walls:
        return np.pad(f, ((0, 0), (m, m), (0, 0)), mode="wrap")
    ny = f.shape[1]
    out = np.empty((f.shape[0], ny + 2 * m, f.shape[2]))
    out[:, m:m + ny, :] = f
    for gg in range(1, m + 1):
        out[:, m - gg, :] = (1 + gg) * f[:, 0, :] - gg * f[:, 1, :]
        out[:, m + ny - 1 + gg, :] = (1 + gg) * f[:, ny - 1, :] - gg * f[:, ny - 2, :]
    return out


def _shift(fp, axis, s, m=3):
    """Interior-sized view of a padded field shifted by s cells along axis (0 z, 1 y, 2 x)."""
    sl = [slice(m, fp.shape[a] - m) for a in range(3)]
    sl[axis] = slice(m + s, fp.shape[axis] - m + s)
    return fp[tuple(sl)]


# ----------------------------------------------------------------------------------------------
# fifth-order WENO (Hamilton-Jacobi form), vectorised
# ----------------------------------------------------------------------------------------------

def weno5(v1, v2, v3, v4, v5, eps=1e-6):
    """Jiang-Peng WENO5 from five one-sided difference quotients, Jiang-Shu indicators and linear
    weights (0.1, 0.6, 0.3)."""
    p1 = v1 / 3.0 - 7.0 * v2 / 6.0 + 11.0 * v3 / 6.0
    p2 = -v2 / 6.0 + 5.0 * v3 / 6.0 + v4 / 3.0
    p3 = v3 / 3.0 + 5.0 * v4 / 6.0 - v5 / 6.0
    s1 = 13.0 / 12.0 * (v1 - 2 * v2 + v3) ** 2 + 0.25 * (v1 - 4 * v2 + 3 * v3) ** 2
    s2 = 13.0 / 12.0 * (v2 - 2 * v3 + v4) ** 2 + 0.25 * (v2 - v4) ** 2
    s3 = 13.0 / 12.0 * (v3 - 2 * v4 + v5) ** 2 + 0.25 * (3 * v3 - 4 * v4 + v5) ** 2
    a1 = 0.1 / (eps + s1) ** 2
    a2 = 0.6 / (eps + s2) ** 2
    a3 = 0.3 / (eps + s3) ** 2
    return (a1 * p1 + a2 * p2 + a3 * p3) / (a1 + a2 + a3)


def one_sided(g: Grid, f, axis):
    """Left- and right-biased WENO5 derivatives of centre field f along axis."""
    h = (g.dz, g.dy, g.dx)[axis]
    fp = pad(g, f)
    F = [_shift(fp, axis, s) for s in range(-3, 4)]          # offsets -3..+3
    d = [(F[m + 1] - F[m]) / h for m in range(6)]            # d[m] between offsets m-3 and m-2
    minus = weno5(d[0], d[1], d[2], d[3], d[4])
    plus = weno5(d[5], d[4], d[3], d[2], d[1])
    return minus, plus


def centre_velocity(g: Grid, u, v, w):
    uc = 0.5 * (u + np.roll(u, 1, axis=2))
    wc = 0.5 * (w + np.roll(w, 1, axis=0))
    if g.walls:
        vm = np.concatenate([np.zeros_like(v[:, :1, :]), v[:, :-1, :]], axis=1)   # bottom wall 0
    else:
        vm = np.roll(v, 1, axis=1)
    return uc, 0.5 * (v + vm), wc


# ----------------------------------------------------------------------------------------------
# level set: transport (Eq. ls adv) and reinitialisation (Eq. reinit), TVD-RK3 in time
# ----------------------------------------------------------------------------------------------

def tvd_rk3(f, rhs, dt):
    f1 = f + dt * rhs(f)
    f2 = 0.75 * f + 0.25 * (f1 + dt * rhs(f1))
    return f / 3.0 + 2.0 / 3.0 * (f2 + dt * rhs(f2))


def advection_rhs(g: Grid, phi, vel):
    """-u . grad(phi) with WENO5 upwinded on the cell-centre velocity (velocity >= 0: left-biased)."""
    out = np.zeros_like(phi)
    for axis, c in zip((2, 1, 0), vel):
        m, p = one_sided(g, phi, axis)
        out -= c * np.where(c >= 0.0, m, p)
    return out


def advect(g: Grid, phi, u, v, w, dt):
    vel = centre_velocity(g, u, v, w)
    return tvd_rk3(phi, lambda f: advection_rhs(g, f, vel), dt)


def reinit_rhs(g: Grid, phi, S):
    """-S (|grad phi| - 1) with Godunov's upwinding of the one-sided WENO5 derivatives."""
    g2 = np.zeros_like(phi)
    for axis in (2, 1, 0):
        a, b = one_sided(g, phi, axis)
        pos = np.maximum(np.maximum(a, 0.0) ** 2, np.minimum(b, 0.0) ** 2)
        neg = np.maximum(np.minimum(a, 0.0) ** 2, np.maximum(b, 0.0) ** 2)
        g2 += np.where(S >= 0.0, pos, neg)
    return -S * (np.sqrt(g2) - 1.0)


def reinitialise(g: Grid, phi, iters):
    h = min(g.dx, g.dy, g.dz)
    S = phi / np.sqrt(phi * phi + h * h)
    dtau = 0.5 * h
    for _ in range(iters):
        phi = tvd_rk3(phi, lambda f: reinit_rhs(g, f, S), dtau)
    return phi


# ----------------------------------------------------------------------------------------------
# mixture (Eq. mat prop) and surface tension (Eqs. fLS, normal, curv)
# ----------------------------------------------------------------------------------------------

def interface_width(g: Grid):
    return 1.5 * max(g.dx, g.dy, g.dz)


def heaviside(g: Grid, phi):
    e = interface_width(g)
    mid = 0.5 * (1.0 + phi / e + np.sin(np.pi * phi / e) / np.pi)
    return np.where(phi < -e, 0.0, np.where(phi > e, 1.0, mid))


def delta(g: Grid, phi):
    e = interface_width(g)
    return np.where(np.abs(phi) > e, 0.0, (1.0 + np.cos(np.pi * phi / e)) / (2.0 * e))


def properties(g: Grid, tp: TwoPhase, phi):
    H = heaviside(g, phi)
    mix = lambda a, b: a * H + b * (1.0 - H)
    return {"rho": mix(tp.rho1, tp.rho2), "mu_s": mix(tp.mu_s1, tp.mu_s2),
            "mu_p": mix(tp.mu_p1, tp.mu_p2), "lam": mix(tp.lam1, tp.lam2)}


def curvature(g: Grid, phi):
    """kappa = -div(n), n = grad phi / |grad phi|, central differences at cell centres."""
    fp = pad(g, phi)
    hs = (g.dz, g.dy, g.dx)
    grads = []
    for axis in (0, 1, 2):
        sl_p = [slice(1, -1)] * 3
        sl_m = [slice(1, -1)] * 3
        sl_p[axis] = slice(2, None)
        sl_m[axis] = slice(0, -2)
        grads.append((fp[tuple(sl_p)] - fp[tuple(sl_m)]) / (2 * hs[axis]))   # on the 2-padded grid
    mag = np.sqrt(grads[0] ** 2 + grads[1] ** 2 + grads[2] ** 2)
    mag = np.maximum(mag, 1e-12)
    n = [gr / mag for gr in grads]
    div = 0.0
    for axis in (0, 1, 2):
        sl_p = [slice(1, -1)] * 3
        sl_m = [slice(1, -1)] * 3
        sl_p[axis] = slice(2, None)
        sl_m[axis] = slice(0, -2)
        d = (n[axis][tuple(sl_p)] - n[axis][tuple(sl_m)]) / (2 * hs[axis])
        div = div + d[1:-1, 1:-1, 1:-1]                       # back to the interior
    return -div


def surface_force(g: Grid, phi, sigma):
    """sigma kappa delta(phi) n on the faces, as sigma kappa_face grad_h H(phi) (balanced with
    the pressure gradient); zero on the top wall face of a channel."""
    H = heaviside(g, phi)
    kap = curvature(g, phi)
    fx = sigma * 0.5 * (kap + np.roll(kap, -1, axis=2)) * (np.roll(H, -1, axis=2) - H) / g.dx
    fz = sigma * 0.5 * (kap + np.roll(kap, -1, axis=0)) * (np.roll(H, -1, axis=0) - H) / g.dz
    if g.walls:
        fy = np.zeros_like(H)
        fy[:, :-1, :] = sigma * 0.5 * (kap[:, :-1, :] + kap[:, 1:, :]) * (H[:, 1:, :] - H[:, :-1, :]) / g.dy
    else:
        fy = sigma * 0.5 * (kap + np.roll(kap, -1, axis=1)) * (np.roll(H, -1, axis=1) - H) / g.dy
    return np.stack([fx, fy, fz])


def face_density(g: Grid, rho):
    rx = 0.5 * (rho + np.roll(rho, -1, axis=2))
    rz = 0.5 * (rho + np.roll(rho, -1, axis=0))
    if g.walls:
        ry = rho.copy()                                      # top wall face: unused
        ry[:, :-1, :] = 0.5 * (rho[:, :-1, :] + rho[:, 1:, :])
    else:
        ry = 0.5 * (rho + np.roll(rho, -1, axis=1))
    return rx, ry, rz


# ----------------------------------------------------------------------------------------------
# Dong-Shen pressure splitting (Eq. poisson LS and the correction that follows it)
# ----------------------------------------------------------------------------------------------

def project_split(g: Grid, us, vs, ws, rho, rho0, p_n, p_nm1, dt):
    """L p = div[(1 - rho0/rho_f) grad(2 p^n - p^{n-1})] + (rho0/dt) div u*;
    u = u* - dt [grad p / rho0 + (1/rho_f - 1/rho0) grad(2 p^n - p^{n-1})].  Returns (u, v, w, p)."""
    ph = 2.0 * p_n - p_nm1
    gph = gradient(g, ph)
    rf = face_density(g, rho)
    flux = [(1.0 - rho0 / r) * gp for r, gp in zip(rf, gph)]
    rhs = divergence(g, *flux) + (rho0 / dt) * divergence(g, us, vs, ws)
    p = solve_poisson(g, rhs)
    gp = gradient(g, p)
    out = [x - dt * (gq / rho0 + (1.0 / r - 1.0 / rho0) * gh)
           for x, gq, r, gh in zip((us, vs, ws), gp, rf, gph)]
    if g.walls:
        out[1][:, -1, :] = 0.0
    return out[0], out[1], out[2], p


# ----------------------------------------------------------------------------------------------
# the step of Sec. 3.2.2 for a bubbly (two-phase) flow
# ----------------------------------------------------------------------------------------------

class TwoPhaseSolver(Solver):
    """Per step: advance phi with u^n (and reinitialise on schedule); properties and surface force
    from phi^{n+1}; the AB2 predictor with those properties (Eqs. ab2tau, ab2, rt, ru); the
    Dong-Shen projection.  The rheology's model, tau_y and L^2 hold in both phases; rho, mu_s,
    mu_p and lambda come from `two_phase`."""

    def __init__(self, grid: Grid, rheology: Rheology, two_phase: TwoPhase,
                 forcing=(FORCE_NONE, 0.0, 0.0), walls_uv=(0.0, 0.0, 0.0, 0.0)):
        super().__init__(grid, rheology, forcing, walls_uv)
        self.tp = two_phase
        self.phi = np.ones(grid.shape)
        self.p_old = np.zeros(grid.shape)
        self._arrays = None

    def write_level_set(self, phi):
        self.phi = np.array(phi, dtype=np.float64, copy=True)

    def write_fields(self, u, v, w, B, hist=None):
        super().write_fields(u, v, w, B, hist)
        self.p = np.zeros(self.g.shape)
        self.p_old = np.zeros(self.g.shape)

    def project(self, dt: float = 1.0):
        super().project(dt)
        self.p = np.zeros(self.g.shape)
        self.p_old = np.zeros(self.g.shape)

    def _p(self):
        p = super()._p()
        if self._arrays is not None:
            lam, mup, mus, rho, fs = self._arrays
            p.lam_c = lam.ctypes.data
            p.mup_c = mup.ctypes.data
            p.mus_c = mus.ctypes.data
            p.rho_c = rho.ctypes.data
            p.fs = fs.ctypes.data
        return p

    def step(self, dt: float, nsteps: int = 1, flags: int = 0):
        g, tp = self.g, self.tp
        for _ in range(nsteps):
            phi = advect(g, self.phi, self.u, self.v, self.w, dt)
            if tp.reinit_every > 0 and tp.reinit_iters > 0 and (self.nstep + 1) % tp.reinit_every == 0:
                phi = reinitialise(g, phi, tp.reinit_iters)
            self.phi = phi
            pr = properties(g, tp, phi)
            fs = surface_force(g, phi, tp.sigma)
            self._arrays = [np.ascontiguousarray(a) for a in
                            (pr["lam"], pr["mu_p"], pr["mu_s"], pr["rho"], fs)]
            Bn, RT, us, vs, ws, RU = self.predictor(dt, flags)
            self._arrays = None
            self.B, self.RT, self.RU = Bn, RT, RU
            self.have_hist = True
            self.nstep += 1
            if flags & self.STOP_AFTER_PREDICTOR:
                self.u, self.v, self.w = us, vs, ws
                continue
            if flags & self.FREEZE_VELOCITY:
                continue
            rho0 = min(tp.rho1, tp.rho2)
            u, v, w, p = project_split(g, us, vs, ws, pr["rho"], rho0, self.p, self.p_old, dt)
            self.u, self.v, self.w = u, v, w
            self.p_old, self.p = self.p, p

    def step_rk3(self, *a, **k):
        raise NotImplementedError("the bubbly-flow path uses the AB2 step (Sec. 3.2.2)")
