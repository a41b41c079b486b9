"""Seeded synthetic workloads (shapes, parameters and initial fields).  Pure input generation:
no step of the method is computed here, so both the HIP path and the CPU oracle take their inputs
from this module and nothing else is shared between them.

Dimensionless groups follow Eq. (PRESS) with rho = 1 and unit length and velocity scales:
mu_s = beta/Re, mu_p = (1 - beta)/Re, lambda = Wi, tau_y = Bi (mu_s + mu_p).  Channels have walls
at y = -1, +1 (box 4 pi x 2 x 2 pi), laminar centreline velocity 1, driven by a constant
-dp/dx = 2/Re applied as a body force.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

OLDROYD_B, FENE_P, SARAMITO, NEO_HOOKEAN = 0, 1, 2, 3
WENO5, HOUC5 = 0, 1
FORCE_NONE, FORCE_CONST_X, FORCE_SIN_X_OF_Y = 0, 1, 2
SEED = 1803


def coefficients(Re: float, Wi: float, beta: float, Bi: float = 0.0):
    """(mu_s, mu_p, lambda, tau_y) for rho = 1, unit velocity and length scales."""
    mu0 = 1.0 / Re
    return beta * mu0, (1.0 - beta) * mu0, Wi, Bi * mu0


@dataclass
class Workload:
    name: str
    nx: int
    ny: int
    nz: int
    lx: float
    ly: float
    lz: float
    walls: bool
    model: int
    mu_s: float
    mu_p: float
    lam: float
    tau_y: float = 0.0
    L2: float = 1.0e4
    rho: float = 1.0
    force: tuple = (FORCE_NONE, 0.0, 0.0)
    wall_velocity: tuple = (0.0, 0.0, 0.0, 0.0)
    dt: float = 1e-3
    steps: int = 100
    precision: str = "fp64"
    init: str = "zero"
    noise: float = 0.0
    seed: int = SEED
    project_initial: bool = False
    adv: int = WENO5             # stress advection scheme
    kappa: float = 0.0           # artificial diffusion coefficient (0: off)
    extra: dict = field(default_factory=dict)

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def ncell(self):
        return self.nx * self.ny * self.nz

    @property
    def dx(self): return self.lx / self.nx

    @property
    def dy(self): return self.ly / self.ny

    @property
    def dz(self): return self.lz / self.nz

    @property
    def y0(self): return -0.5 * self.ly if self.walls else 0.0

    def rheology(self):
        return dict(model=self.model, rho=self.rho, mu_s=self.mu_s, mu_p=self.mu_p, lam=self.lam,
                    tau_y=self.tau_y, L2=self.L2)


def taylor_green_periodic(n: int = 32) -> Workload:
    """Triply periodic cube n^3, L = 2 pi, Oldroyd-B Wi = 1, beta = 0.5, Re = 100, Taylor-Green
    velocity, B = I, dt = 1e-3, 100 steps, FP64 (the small case the oracle finishes quickly)."""
    ms, mp, lam, _ = coefficients(100.0, 1.0, 0.5)
    L = 2 * math.pi
    return Workload("taylor_green_32_oldroyd_b", n, n, n, L, L, L, False, OLDROYD_B, ms, mp, lam,
                    dt=1e-3, steps=100, init="taylor_green")


def kolmogorov_saramito(n: int = 128, steps: int = 200) -> Workload:
    """Triply periodic n^3 (2 pi), Saramito Wi = 1, Bi = 0.5, beta = 0.5, Re = 1000, forcing
    f_x = sin 4y, u = sin 4y + uniform noise 1e-2, projected, B = I, FP64."""
    ms, mp, lam, ty = coefficients(1000.0, 1.0, 0.5, 0.5)
    L = 2 * math.pi
    return Workload(f"kolmogorov_{n}_saramito", n, n, n, L, L, L, False, SARAMITO, ms, mp, lam,
                    tau_y=ty, force=(FORCE_SIN_X_OF_Y, 1.0, 4.0), dt=1e-3, steps=steps,
                    init="kolmogorov", noise=1e-2, project_initial=True)


def channel_fene_p(nx=256, ny=128, nz=128, steps=500, precision="mixed") -> Workload:
    """Channel 4 pi x 2 x 2 pi, walls at y = -1, +1, FENE-P L^2 = 900, Wi = 5, beta = 0.9,
    Re = 2000, laminar parabola + 5 % noise, projected, B = I."""
    ms, mp, lam, _ = coefficients(2000.0, 5.0, 0.9)
    return Workload(f"channel_{nx}x{ny}x{nz}_fene_p", nx, ny, nz, 4 * math.pi, 2.0, 2 * math.pi,
                    True, FENE_P, ms, mp, lam, L2=900.0, force=(FORCE_CONST_X, 2.0 / 2000.0, 0.0),
                    dt=1e-3, steps=steps, precision=precision, init="parabola", noise=0.05,
                    project_initial=True)


def channel_saramito(nx=512, ny=256, nz=256, steps=200, precision="fp64") -> Workload:
    """Channel 4 pi x 2 x 2 pi, Saramito Wi = 2, Bi = 0.2, beta = 0.1, Re = 5000, constant
    pressure gradient, parabola + noise projected to a divergence-free field, B = I."""
    ms, mp, lam, ty = coefficients(5000.0, 2.0, 0.1, 0.2)
    return Workload(f"channel_{nx}x{ny}x{nz}_saramito", nx, ny, nz, 4 * math.pi, 2.0, 2 * math.pi,
                    True, SARAMITO, ms, mp, lam, tau_y=ty,
                    force=(FORCE_CONST_X, 2.0 / 5000.0, 0.0), dt=1e-3, steps=steps,
                    precision=precision, init="parabola", noise=0.05, project_initial=True)


def initial_fields(wl: Workload):
    """(u, v, w, B) as float64 numpy arrays, u/v/w of shape (nz, ny, nx), B (6, nz, ny, nx)."""
    nz, ny, nx = wl.shape
    dx, dy, dz = wl.dx, wl.dy, wl.dz
    xf = (np.arange(nx) + 1.0) * dx          # u-face x
    xc = (np.arange(nx) + 0.5) * dx          # centre x (v, w faces)
    yc = wl.y0 + (np.arange(ny) + 0.5) * dy  # centre y (u, w faces)
    yf = wl.y0 + (np.arange(ny) + 1.0) * dy  # v-face y
    zc = (np.arange(nz) + 0.5) * dz
    zf = (np.arange(nz) + 1.0) * dz
    u = np.zeros(wl.shape)
    v = np.zeros(wl.shape)
    w = np.zeros(wl.shape)
    if wl.init == "taylor_green":
        u = np.sin(xf)[None, None, :] * np.cos(yc)[None, :, None] * np.cos(zc)[:, None, None]
        v = -np.cos(xc)[None, None, :] * np.sin(yf)[None, :, None] * np.cos(zc)[:, None, None]
        w = np.zeros(wl.shape)
    elif wl.init == "kolmogorov":
        u = np.broadcast_to(np.sin(4.0 * yc)[None, :, None], wl.shape).copy()
    elif wl.init == "parabola":
        u = np.broadcast_to((1.0 - yc ** 2)[None, :, None], wl.shape).copy()
    u = np.ascontiguousarray(u, dtype=np.float64)
    v = np.ascontiguousarray(v, dtype=np.float64)
    w = np.ascontiguousarray(w, dtype=np.float64)
    if wl.noise > 0.0:
        rng = np.random.default_rng(wl.seed)
        u += rng.uniform(-wl.noise, wl.noise, wl.shape)
        v += rng.uniform(-wl.noise, wl.noise, wl.shape)
        w += rng.uniform(-wl.noise, wl.noise, wl.shape)
    if wl.walls:
        v[:, -1, :] = 0.0
    B = np.zeros((6,) + wl.shape)
    B[0] = B[3] = B[5] = 1.0
    return u, v, w, B


def solid_fractions(wl: Workload, inside, sub: int = 3):
    """Solid volume fractions (alpha_u, alpha_v, alpha_w) of a fixed obstacle around the u-, v-
    and w-points: the share of sub^3 sample points of each velocity point's cell-sized control
    volume for which inside(x, y, z) is true.  Pure geometry (input of the immersed boundary)."""
    nz, ny, nx = wl.shape
    dx, dy, dz = wl.dx, wl.dy, wl.dz
    off = (np.arange(sub) + 0.5) / sub - 0.5
    out = []
    for shift in ((1.0, 0.5, 0.5), (0.5, 1.0, 0.5), (0.5, 0.5, 1.0)):
        x = (np.arange(nx) + shift[0]) * dx
        y = wl.y0 + (np.arange(ny) + shift[1]) * dy
        a = np.zeros(wl.shape)
        for k in range(nz):
            z = (k + shift[2]) * dz
            cnt = np.zeros((ny, nx))
            for oz in off:
                for oy in off:
                    for ox in off:
                        cnt += inside(x[None, :] + ox * dx, y[:, None] + oy * dy, z + oz * dz)
            a[k] = cnt / sub ** 3
        out.append(a)
    if wl.walls:
        out[1][:, -1, :] = 0.0
    return out


def sphere(center, radius):
    """inside() of a sphere (no periodic images)."""
    cx, cy, cz = center
    return lambda x, y, z: (x - cx) ** 2 + (y - cy) ** 2 + (z - cz) ** 2 <= radius ** 2


def random_state(shape, seed, amp_u=0.3, amp_b=0.05, walls=False):
    """A generic random state (for parity tests on arbitrary shapes): noise velocities and a
    symmetric positive-definite perturbation of B = I."""
    rng = np.random.default_rng(seed)
    u = amp_u * rng.standard_normal(shape)
    v = amp_u * rng.standard_normal(shape)
    w = amp_u * rng.standard_normal(shape)
    if walls:
        v[:, -1, :] = 0.0
    B = amp_b * rng.standard_normal((6,) + tuple(shape))
    B[0] += 1.0
    B[3] += 1.0
    B[5] += 1.0
    return u, v, w, B


def serving_requests(n_requests=500, seed=SEED, sizes=(32, 48, 64, 96, 128), rate=None,
                     step_range=(100, 1000)):
    """Seeded request stream: Poisson arrivals (exponential gaps at `rate` per second, all at
    t = 0 when rate is None), n^3 periodic grids, model / Wi / Bi / beta drawn uniformly,
    Re = 1000 and L^2 = 900, Kolmogorov forcing, mixed precision."""
    rng = np.random.default_rng(seed)
    t = 0.0
    reqs = []
    for r in range(n_requests):
        if rate:
            t += rng.exponential(1.0 / rate)
        n = int(rng.choice(sizes))
        model = int(rng.integers(0, 3))
        Wi = float(rng.uniform(0.1, 10.0))
        Bi = float(rng.uniform(0.0, 1.0))
        beta = float(rng.uniform(0.1, 0.9))
        steps = int(rng.integers(step_range[0], step_range[1] + 1))
        ms, mp, lam, ty = coefficients(1000.0, Wi, beta, Bi if model == SARAMITO else 0.0)
        L = 2 * math.pi
        wl = Workload(f"req{r}", n, n, n, L, L, L, False, model, ms, mp, lam, tau_y=ty, L2=900.0,
                      force=(FORCE_SIN_X_OF_Y, 1.0, 4.0), dt=1e-3, steps=steps,
                      precision="mixed", init="kolmogorov", noise=1e-2, seed=seed + 1 + r,
                      project_initial=True)
        reqs.append((t, wl))
    return reqs
