"""Pins of the oracle's full step (predictor of Sec. 3.2.2 + projection) on flows with known answers.

* viscoelastic shear wave (Oldroyd-B, periodic): the discrete problem is exactly linear, one
  2x2 AB2 recurrence per Fourier mode -- pins the coupling of div(tau) into momentum and of the
  velocity gradient into B, with their signs, edge averages and spacings;
* plane Couette start-up of an Oldroyd-B fluid between moving walls: second-order convergence to
  the continuum series solution (sine modes, each a 2x2 linear ODE solved by matrix exponential);
* 2D Taylor-Green decay (Newtonian limit): the staggered divergence-form advection of this field is
  a discrete gradient, so after projection the amplitude follows the scalar AB2 recurrence of the
  discrete viscous decay exactly;
* laminar Kolmogorov flow (Oldroyd-B): an exact discrete steady state;
* inviscid energy conservation of the advection (skew-symmetric on divergence-free fields);
* model reductions (Saramito tau_y = 0 is Oldroyd-B; FENE-P with huge L^2 tends to Oldroyd-B;
  mu_p = 0 decouples B) and equivariance (shift, x<->z exchange).
"""
import numpy as np
import pytest
import scipy.linalg

import oracle
from oracle import Grid, Rheology, Solver

I6 = np.array([1.0, 0, 0, 1.0, 0, 1.0])


def _identity_B(g):
    return np.broadcast_to(I6[:, None, None, None], (6,) + g.shape).copy()


def _yprofile(g, prof):
    return np.broadcast_to(prof[None, :, None], g.shape).copy()


def test_viscoelastic_shear_wave_recurrence():
    g = Grid(4, 32, 4, 1.0, 2 * np.pi, 1.0)
    mu_s, mu_p, lam, rho, eps, dt = 0.05, 0.2, 0.7, 1.0, 0.3, 2e-3
    r = Rheology(model=oracle.OLDROYD_B, rho=rho, mu_s=mu_s, mu_p=mu_p, lam=lam)
    s = Solver(g, r)
    y = g.yc()
    z = np.zeros(g.shape)
    s.write_fields(_yprofile(g, eps * np.sin(y)), z, z, _identity_B(g))
    dy, G = g.dy, mu_p / lam
    kc2 = 4 * np.sin(dy / 2) ** 2 / dy ** 2
    sg = np.sin(dy) / dy

    def rhs(A, C):
        return (-mu_s * kc2 * A - G * sg * C) / rho, sg * A - C / lam

    A, C = eps, 0.0
    fA_old = fC_old = None
    nsteps = 150
    for n in range(nsteps):
        fA, fC = rhs(A, C)
        if fA_old is None:
            A, C = A + dt * fA, C + dt * fC
        else:
            A, C = A + dt * (1.5 * fA - 0.5 * fA_old), C + dt * (1.5 * fC - 0.5 * fC_old)
        fA_old, fC_old = fA, fC
    s.step(dt, nsteps)
    assert np.abs(s.u - _yprofile(g, A * np.sin(y))).max() < 1e-13
    assert np.abs(s.B[1] - _yprofile(g, C * np.cos(y))).max() < 1e-13
    assert np.abs(s.v).max() < 1e-13 and np.abs(s.w).max() < 1e-13


def _couette_continuum(y, t, U, mu_s, mu_p, lam, rho, nmodes=400):
    """u and tau_xy of Oldroyd-B plane Couette start-up, walls y = -1, +1 moving at -U, +U, fluid
    initially at rest and stress-free.  u = U y + sum a_m sin(m pi y); tau_xy = mu_p U (1 -
    exp(-t/lam)) + sum s_m cos(m pi y);  rho a_m' = -mu_s (m pi)^2 a_m - m pi s_m,
    lam s_m' + s_m = mu_p m pi a_m; a_m(0) = 2 U (-1)^m / (m pi), s_m(0) = 0."""
    u = U * y.copy()
    tau = np.full_like(y, mu_p * U * (1 - np.exp(-t / lam)))
    for m in range(1, nmodes + 1):
        k = m * np.pi
        M = np.array([[-mu_s * k * k / rho, -k / rho], [mu_p * k / lam, -1.0 / lam]])
        a, s = scipy.linalg.expm(M * t) @ np.array([2 * U * (-1) ** m / k, 0.0])
        u += a * np.sin(k * y)
        tau += s * np.cos(k * y)
    return u, tau


def test_oldroyd_b_couette_startup_converges_second_order():
    U, mu_s, mu_p, lam, rho, T = 1.0, 0.5, 0.5, 0.5, 1.0, 0.5
    errs = []
    for ny, dt in ((16, 1e-3), (32, 5e-4)):
        g = Grid(4, ny, 4, 1.0, 2.0, 1.0, walls=True)
        r = Rheology(model=oracle.OLDROYD_B, rho=rho, mu_s=mu_s, mu_p=mu_p, lam=lam)
        s = Solver(g, r, walls_uv=(-U, U, 0.0, 0.0))
        z = np.zeros(g.shape)
        s.write_fields(z, z, z, _identity_B(g))
        s.step(dt, int(round(T / dt)))
        y = g.yc()
        u_ex, tau_ex = _couette_continuum(y, T, U, mu_s, mu_p, lam, rho)
        tau = oracle.stress(g, r, s.B)[1]
        e = max(np.abs(s.u[0, :, 0] - u_ex).max(), np.abs(tau[0, :, 0] - tau_ex).max())
        errs.append(e)
        # x- and z-independent, no wall-normal flow
        assert np.abs(s.u - s.u[:1, :, :1]).max() < 1e-13
        assert np.abs(s.v).max() < 1e-13 and np.abs(s.w).max() < 1e-13
    assert errs[1] < 2e-3 and 3.3 < errs[0] / errs[1] < 4.7, errs


def _taylor_green_2d(g):
    xf = (np.arange(g.nx) + 1) * g.dx
    xc = (np.arange(g.nx) + 0.5) * g.dx
    yf = (np.arange(g.ny) + 1) * g.dy
    yc = (np.arange(g.ny) + 0.5) * g.dy
    u = np.broadcast_to(np.sin(xf)[None, None, :] * np.cos(yc)[None, :, None], g.shape).copy()
    v = np.broadcast_to(-np.cos(xc)[None, None, :] * np.sin(yf)[None, :, None], g.shape).copy()
    return u, v


@pytest.mark.parametrize("n", [16, 32])
def test_taylor_green_2d_exact_discrete_decay(n):
    g = Grid(n, n, 4, 2 * np.pi, 2 * np.pi, 2 * np.pi * 4 / n)
    nu, dt, nsteps = 0.05, 1e-2, 60
    s = Solver(g, Rheology(model=oracle.OLDROYD_B, mu_s=nu, mu_p=0.0, lam=1.0))
    u, v = _taylor_green_2d(g)
    s.write_fields(u, v, np.zeros(g.shape), _identity_B(g))
    mud = -nu * 2 * (4 / g.dx ** 2) * np.sin(g.dx / 2) ** 2
    a = [1.0, 1.0 + dt * mud]
    for k in range(1, nsteps):
        a.append(a[k] + dt * mud * (1.5 * a[k] - 0.5 * a[k - 1]))
    s.step(dt, nsteps)
    assert np.abs(s.u - a[nsteps] * u).max() < 1e-13
    assert np.abs(s.v - a[nsteps] * v).max() < 1e-13


def test_taylor_green_2d_continuum_second_order():
    """The oracle's decaying Taylor-Green flow tends to the continuum exp(-2 nu t) at second order
    in h (dt small enough that the AB2 error is far below the spatial one)."""
    nu, dt, nsteps = 0.05, 5e-3, 100
    errs = []
    for n in (16, 32, 64):
        g = Grid(n, n, 4, 2 * np.pi, 2 * np.pi, 2 * np.pi * 4 / n)
        s = Solver(g, Rheology(model=oracle.OLDROYD_B, mu_s=nu, mu_p=0.0, lam=1.0))
        u, v = _taylor_green_2d(g)
        s.write_fields(u, v, np.zeros(g.shape), _identity_B(g))
        s.step(dt, nsteps)
        ex = np.exp(-2 * nu * dt * nsteps)
        errs.append(max(np.abs(s.u - ex * u).max(), np.abs(s.v - ex * v).max()))
    assert errs[0] < 2e-3 and 3.9 < errs[0] / errs[1] < 4.1 and 3.9 < errs[1] / errs[2] < 4.1, errs


def test_kolmogorov_oldroyd_b_exact_steady_state():
    g = Grid(4, 32, 4, 1.0, 2 * np.pi, 1.0)
    ms, mp, lam, F0, k = 0.1, 0.05, 0.7, 1.0, 4
    r = Rheology(model=oracle.OLDROYD_B, mu_s=ms, mu_p=mp, lam=lam)
    dy, yc = g.dy, g.yc()
    kc2 = 4 * np.sin(k * dy / 2) ** 2 / dy ** 2
    sg = np.sin(k * dy) / dy
    A = F0 / (ms * kc2 + mp * sg ** 2)
    u = _yprofile(g, A * np.sin(k * yc))
    B = _identity_B(g)
    B[0] = _yprofile(g, 1 + 2 * lam ** 2 * sg ** 2 * A ** 2 * np.cos(k * yc) ** 2)
    B[1] = _yprofile(g, lam * sg * A * np.cos(k * yc))
    s = Solver(g, r, forcing=(oracle.FORCE_SIN_X_OF_Y, F0, k))
    z = np.zeros(g.shape)
    s.write_fields(u, z, z, B)
    s.step(1e-3, 100)
    assert np.abs(s.u - u).max() < 1e-13 * A
    assert np.abs(s.B - B).max() < 1e-13 * np.abs(B).max()


def _random_solenoidal(g, rng, amp=1.0):
    u = amp * rng.standard_normal(g.shape)
    v = amp * rng.standard_normal(g.shape)
    w = amp * rng.standard_normal(g.shape)
    if g.walls:
        v[:, -1, :] = 0.0
    u, v, w, _ = oracle.project(g, u, v, w, 1.0)
    return u, v, w


def test_inviscid_advection_conserves_energy():
    """The divergence-form staggered advection is skew-symmetric on solenoidal fields: the
    semi-discrete energy is conserved, so over a fixed time the energy drift is the AB2 error,
    falling as dt^2.  A non-conservative term would leave a drift independent of dt."""
    g = Grid(16, 16, 16, 2 * np.pi, 2 * np.pi, 2 * np.pi)
    u, v, w = _random_solenoidal(g, np.random.default_rng(7), 0.3)
    drift = []
    for dt in (2e-3, 1e-3):
        s = Solver(g, Rheology(model=oracle.OLDROYD_B, mu_s=0.0, mu_p=0.0, lam=1.0))
        s.write_fields(u, v, w, _identity_B(g))
        e0 = s.health()["energy"]
        s.step(dt, int(round(0.04 / dt)))
        drift.append(abs(s.health()["energy"] - e0) / e0)
    assert drift[1] < 1e-6 and 3.6 < drift[0] / drift[1] < 4.4, drift


def _c1_like(n=12, model=oracle.OLDROYD_B, **kw):
    g = Grid(n, n, n, 2 * np.pi, 2 * np.pi, 2 * np.pi)
    rng = np.random.default_rng(42)
    u, v, w = _random_solenoidal(g, rng, 0.5)
    B = _identity_B(g)
    B += 0.05 * rng.standard_normal(B.shape)
    B[1] *= 0.5
    return g, (u, v, w, B), Rheology(model=model, **kw)


def test_saramito_without_yield_stress_is_oldroyd_b():
    g, f, _ = _c1_like()
    a = Solver(g, Rheology(model=oracle.OLDROYD_B, mu_s=0.01, mu_p=0.02, lam=0.8))
    b = Solver(g, Rheology(model=oracle.SARAMITO, mu_s=0.01, mu_p=0.02, lam=0.8, tau_y=0.0))
    for s in (a, b):
        s.write_fields(*f)
        s.step(1e-3, 5)
    assert np.array_equal(a.u, b.u) and np.array_equal(a.B, b.B)


def test_fene_p_large_extensibility_tends_to_oldroyd_b():
    g, f, _ = _c1_like()
    a = Solver(g, Rheology(model=oracle.OLDROYD_B, mu_s=0.01, mu_p=0.02, lam=0.8))
    b = Solver(g, Rheology(model=oracle.FENE_P, mu_s=0.01, mu_p=0.02, lam=0.8, L2=1e12))
    for s in (a, b):
        s.write_fields(*f)
        s.step(1e-3, 5)
    assert np.abs(a.u - b.u).max() < 1e-9 and np.abs(a.B - b.B).max() < 1e-9


def test_zero_polymer_viscosity_decouples_stress():
    g, (u, v, w, B), _ = _c1_like()
    r = Rheology(model=oracle.OLDROYD_B, mu_s=0.01, mu_p=0.0, lam=0.8)
    a, b = Solver(g, r), Solver(g, r)
    a.write_fields(u, v, w, B)
    b.write_fields(u, v, w, _identity_B(g))
    for s in (a, b):
        s.step(1e-3, 5)
    assert np.abs(a.u - b.u).max() < 1e-13


def test_shift_equivariance():
    g, (u, v, w, B), r = _c1_like(model=oracle.SARAMITO, mu_s=0.01, mu_p=0.02, lam=0.8,
                                  tau_y=0.002)
    a, b = Solver(g, r), Solver(g, r)
    a.write_fields(u, v, w, B)
    sh = lambda x: np.roll(x, (1, -2, 3), axis=(-3, -2, -1))
    b.write_fields(sh(u), sh(v), sh(w), sh(B))
    for s in (a, b):
        s.step(1e-3, 4)
    assert np.abs(sh(a.u) - b.u).max() < 1e-12
    assert np.abs(sh(a.B) - b.B).max() < 1e-12


def _swap_xz_fields(u, v, w, B):
    t = lambda x: np.ascontiguousarray(np.swapaxes(x, -1, -3))
    # xx<->zz, xy<->yz, xz stays
    Bs = np.stack([t(B[5]), t(B[4]), t(B[2]), t(B[3]), t(B[1]), t(B[0])])
    return t(w), t(v), t(u), Bs


@pytest.mark.parametrize("walls", [False, True])
def test_x_z_exchange_equivariance(walls):
    n = 10
    g = Grid(n, 8, n, 2.0, 2.0, 2.0, walls=walls)
    rng = np.random.default_rng(3)
    u, v, w = _random_solenoidal(g, rng, 0.5)
    B = _identity_B(g) + 0.05 * rng.standard_normal((6,) + g.shape)
    r = Rheology(model=oracle.FENE_P, mu_s=0.01, mu_p=0.03, lam=0.5, L2=50.0)
    wu = (0.3, -0.2, 0.1, 0.4)
    a = Solver(g, r, walls_uv=wu)
    b = Solver(g, r, walls_uv=(wu[2], wu[3], wu[0], wu[1]))
    a.write_fields(u, v, w, B)
    b.write_fields(*_swap_xz_fields(u, v, w, B))
    for s in (a, b):
        s.step(2e-3, 4)
    su, sv, sw, sB = _swap_xz_fields(a.u, a.v, a.w, a.B)
    for x, y in ((su, b.u), (sv, b.v), (sw, b.w), (sB, b.B)):
        assert np.abs(x - y).max() < 1e-12
