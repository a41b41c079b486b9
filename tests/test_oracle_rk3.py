"""Pins of the oracle's low-storage Runge-Kutta step (Sec. 3.3.1, Eqs. RK-rt, NS-num1..3, eq:RK).

* the coefficients of Eq. (eq:RK) are consistent (sum of 2 alpha = 1, sum of zeta + xi = 1) and
  integrate dy/dt = y to third order;
* 2D Taylor-Green decay: the advection is a discrete gradient (removed by the projection), so the
  amplitude follows the product of (1 + 2 alpha_k dt mu_d) over the substeps exactly;
* viscoelastic shear wave: one exact 2x2 recurrence per substep;
* homogeneous shear with frozen velocity: third-order convergence of Oldroyd-B to its closed form;
* laminar Kolmogorov flow of Oldroyd-B: the exact discrete steady state is kept;
* the velocity is discretely solenoidal after every step.
"""
import numpy as np

import oracle
from oracle import Grid, Rheology, Solver

A, Z, X = oracle.RK3_ALPHA, oracle.RK3_ZETA, oracle.RK3_XI


def _identity_B(g):
    B = np.zeros((6,) + g.shape)
    B[0] = B[3] = B[5] = 1.0
    return B


def test_coefficients_consistent_and_third_order():
    assert abs(sum(2 * a for a in A) - 1.0) < 1e-15
    assert abs(sum(Z) + sum(X) - 1.0) < 1e-15
    # low-storage scheme on y' = y: the (zeta, xi) combination of the previous substep slopes
    errs = []
    for dt in (0.1, 0.05):
        y, T = 1.0, 1.0
        for _ in range(int(round(T / dt))):
            f2 = None
            for k in range(3):
                f1 = y
                y = y + dt * (Z[k] * f1 + (X[k] * f2 if f2 is not None else 0.0))
                f2 = f1
        errs.append(abs(y - np.e))
    assert 7.0 < errs[0] / errs[1] < 9.0, errs


def _taylor_green_2d(g):
    xf = (np.arange(g.nx) + 1) * g.dx
    xc = (np.arange(g.nx) + 0.5) * g.dx
    yf = (np.arange(g.ny) + 1) * g.dy
    yc = (np.arange(g.ny) + 0.5) * g.dy
    u = np.broadcast_to(np.sin(xf)[None, None, :] * np.cos(yc)[None, :, None], g.shape).copy()
    v = np.broadcast_to(-np.cos(xc)[None, None, :] * np.sin(yf)[None, :, None], g.shape).copy()
    return u, v


def test_taylor_green_rk3_exact_recurrence():
    n = 32
    g = Grid(n, n, 4, 2 * np.pi, 2 * np.pi, 2 * np.pi * 4 / n)
    nu, dt, nsteps = 0.05, 1e-2, 30
    s = Solver(g, Rheology(mu_s=nu, mu_p=0.0))
    u, v = _taylor_green_2d(g)
    s.write_fields(u, v, np.zeros(g.shape), _identity_B(g))
    mud = -nu * 2 * (4 / g.dx ** 2) * np.sin(g.dx / 2) ** 2
    a = 1.0
    for _ in range(nsteps):
        for k in range(3):
            a *= 1 + 2 * A[k] * dt * mud
    s.step_rk3(dt, nsteps)
    assert np.abs(s.u - a * u).max() < 1e-13 and np.abs(s.v - a * v).max() < 1e-13


def test_shear_wave_rk3_exact_recurrence():
    g = Grid(4, 32, 4, 1.0, 2 * np.pi, 1.0)
    mu_s, mu_p, lam, rho, eps, dt = 0.05, 0.2, 0.7, 1.0, 0.3, 4e-3
    s = Solver(g, Rheology(rho=rho, mu_s=mu_s, mu_p=mu_p, lam=lam))
    y = g.yc()
    z = np.zeros(g.shape)
    s.write_fields(np.broadcast_to((eps * np.sin(y))[None, :, None], g.shape).copy(), z, z,
                   _identity_B(g))
    dy, G = g.dy, mu_p / lam
    kc2 = 4 * np.sin(dy / 2) ** 2 / dy ** 2
    sg = np.sin(dy) / dy
    amp, C = eps, 0.0
    nsteps = 60
    for _ in range(nsteps):
        fC2 = None
        for k in range(3):
            fC1 = sg * amp - C / lam
            Cn = C + dt * (Z[k] * fC1 + (X[k] * fC2 if fC2 is not None else 0.0))
            amp = amp + dt * (2 * A[k] * (-mu_s * kc2 * amp) + A[k] * (-G * sg) * (Cn + C)) / rho
            C, fC2 = Cn, fC1
    s.step_rk3(dt, nsteps)
    assert np.abs(s.u - (amp * np.sin(y))[None, :, None]).max() < 1e-13
    assert np.abs(s.B[1] - (C * np.cos(y))[None, :, None]).max() < 1e-13


def test_homogeneous_shear_rk3_third_order():
    lam, gd, T = 0.5, 1.3, 1.0
    errs = []
    for dt in (0.04, 0.02):
        g = Grid(4, 8, 4, 1.0, 2.0, 1.0, walls=True)
        s = Solver(g, Rheology(mu_s=0.1, mu_p=0.4, lam=lam), walls_uv=(-gd, gd, 0.0, 0.0))
        u = np.broadcast_to((gd * g.yc())[None, :, None], g.shape).copy()
        s.write_fields(u, np.zeros(g.shape), np.zeros(g.shape), _identity_B(g))
        n = int(round(T / dt))
        s.step_rk3(dt, n, flags=Solver.FREEZE_VELOCITY)
        e = np.exp(-n * dt / lam)
        bxy = lam * gd * (1 - e)
        bxx = 1 + 2 * lam ** 2 * gd ** 2 * (1 - e) - 2 * lam * gd ** 2 * n * dt * e
        errs.append(max(abs(s.B[0, 0, 0, 0] - bxx), abs(s.B[1, 0, 0, 0] - bxy)))
    assert 7.0 < errs[0] / errs[1] < 9.0, errs


def test_kolmogorov_steady_state_rk3():
    g = Grid(4, 32, 4, 1.0, 2 * np.pi, 1.0)
    ms, mp, lam, F0, k = 0.1, 0.05, 0.7, 1.0, 4
    dy, yc = g.dy, g.yc()
    kc2 = 4 * np.sin(k * dy / 2) ** 2 / dy ** 2
    sg = np.sin(k * dy) / dy
    amp = F0 / (ms * kc2 + mp * sg ** 2)
    prof = lambda a: np.broadcast_to(a[None, :, None], g.shape).copy()
    u = prof(amp * np.sin(k * yc))
    B = _identity_B(g)
    B[0] = prof(1 + 2 * lam ** 2 * sg ** 2 * amp ** 2 * np.cos(k * yc) ** 2)
    B[1] = prof(lam * sg * amp * np.cos(k * yc))
    s = Solver(g, Rheology(mu_s=ms, mu_p=mp, lam=lam), forcing=(oracle.FORCE_SIN_X_OF_Y, F0, k))
    z = np.zeros(g.shape)
    s.write_fields(u, z, z, B)
    s.step_rk3(1e-3, 20)
    assert np.abs(s.u - u).max() < 1e-13 * amp and np.abs(s.B - B).max() < 1e-13


def test_rk3_solenoidal_random_flow():
    g = Grid(16, 12, 8, 2 * np.pi, 2.0, np.pi, walls=True)
    rng = np.random.default_rng(4)
    u, v, w = [0.3 * rng.standard_normal(g.shape) for _ in range(3)]
    v[:, -1, :] = 0.0
    u, v, w, _ = oracle.project(g, u, v, w, 1.0)
    B = _identity_B(g) + 0.05 * rng.standard_normal((6,) + g.shape)
    s = Solver(g, Rheology(model=oracle.FENE_P, mu_s=0.01, mu_p=0.02, lam=0.5, L2=50.0),
               walls_uv=(0.2, -0.1, 0.0, 0.3))
    s.write_fields(u, v, w, B)
    s.step_rk3(2e-3, 3)
    div = np.abs(oracle.divergence(g, s.u, s.v, s.w)).max()
    assert div * g.dy / np.abs(s.u).max() < 1e-12
