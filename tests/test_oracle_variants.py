"""Pins of the oracle's stress-transport variants: the HOUC advection named beside WENO in Sec. 3,
the Neo-Hookean closure of Table 1, the local artificial diffusion of Sec. 3.1, and two flow
checks of the closures: steady plane Poiseuille flow of Oldroyd-B and FENE-P (exact discrete
fixed points found by brute force) and oscillatory simple shear of the Saramito model (against a
high-accuracy ODE integration).

Independent references only: polynomial exactness and the exact truncation error of a six-point
stencil, closed forms and scalar recurrences, a nonlinear solve of the 1D steady equations
assembled here from the staggered-grid definitions, and scipy's ODE integrator.
"""
import numpy as np
import pytest
from scipy.integrate import solve_ivp
from scipy.optimize import brentq, fsolve

import oracle
from oracle import Grid, Rheology, Solver


def _identity_B(g):
    B = np.zeros((6,) + g.shape)
    B[0] = B[3] = B[5] = 1.0
    return B


def _yprofile(g, prof):
    return np.broadcast_to(np.asarray(prof)[None, :, None], g.shape).copy()


# ---------------------------------------------------------------------------------------------
# HOUC5
# ---------------------------------------------------------------------------------------------

@pytest.mark.parametrize("vel", [1.0, -1.0])
def test_houc5_exact_for_quintics(vel):
    """A six-point stencil exact for every polynomial of degree <= 5 is unique: this fixes all six
    weights of the upwind-biased stencil on each side."""
    h, n = 0.1, 40
    x = (np.arange(n) - 20) * h
    for deg in range(6):
        c = np.random.default_rng(deg).standard_normal(deg + 1)
        f = np.polyval(c, x)
        d = oracle.upwind_line(f, h, vel, oracle.HOUC5)
        ref = np.polyval(np.polyder(c), x) if deg > 0 else np.zeros(n)
        inner = slice(4, n - 4)
        assert np.abs(d[inner] - ref[inner]).max() < 1e-9 * max(1.0, np.abs(ref[inner]).max())


@pytest.mark.parametrize("vel, sign", [(1.0, -1.0), (-1.0, 1.0)])
def test_houc5_truncation_error_of_sextic(vel, sign):
    """For f = x^6 the stencil error is exactly the leading term: -/+ h^5 f^(6) / 60 = -/+ 12 h^5
    (upwind from the left / from the right)."""
    h, n = 0.05, 40
    x = (np.arange(n) - 20) * h
    d = oracle.upwind_line(x ** 6, h, vel, oracle.HOUC5)
    inner = slice(4, n - 4)
    err = d[inner] - 6 * x[inner] ** 5
    assert np.allclose(err, sign * 12 * h ** 5, rtol=1e-6, atol=1e-12)


def test_houc5_fifth_order_and_upwind_side():
    errs = []
    for n in (32, 64, 128):
        h = 2 * np.pi / n
        x = (np.arange(n) + 0.5) * h
        errs.append(np.abs(oracle.upwind_line(np.sin(x), h, 1.0, oracle.HOUC5) - np.cos(x)).max())
    assert 28 < errs[0] / errs[1] < 36 and 28 < errs[1] / errs[2] < 36, errs
    # vel >= 0 reads offsets -3..+2 only: a spike at +3 does not reach the cell
    f = np.zeros(16)
    f[8 + 3] = 1.0
    assert oracle.upwind_line(f, 1.0, 1.0, oracle.HOUC5)[8] == 0.0
    assert oracle.upwind_line(f, 1.0, -1.0, oracle.HOUC5)[8] != 0.0


def test_houc5_transport_fifth_order():
    """Uniform transport of a smooth B pattern (frozen velocity, no relaxation) with HOUC5."""
    def run(n, dt=1e-3, t_end=0.25):
        L = 2 * np.pi
        g = Grid(n, 4, 4, L, L * 4 / n, L * 4 / n)
        s = Solver(g, Rheology(mu_s=0.0, mu_p=0.0, lam=1e30, adv=oracle.HOUC5))
        c = (np.arange(n) + 0.5) * L / n
        prof = lambda xx: np.sin(xx) + 0.3 * np.cos(2 * xx)
        B = _identity_B(g)
        B[1] = 0.2 * prof(c)[None, None, :]
        u = np.full(g.shape, 1.0)
        z = np.zeros(g.shape)
        s.write_fields(u, z, z, B)
        m = int(round(t_end / dt))
        s.step(dt, m, flags=Solver.FREEZE_VELOCITY)
        return np.abs(s.B[1] - 0.2 * prof(c - m * dt)[None, None, :]).max()
    e32, e64 = run(32), run(64)
    assert e32 / e64 > 20, (e32, e64)


# ---------------------------------------------------------------------------------------------
# Neo-Hookean (Table 1: B = tau/G, F = a = 0)
# ---------------------------------------------------------------------------------------------

def _shear_solver(rheo, gd):
    g = Grid(4, 8, 4, 1.0, 2.0, 1.0, walls=True)
    s = Solver(g, rheo, walls_uv=(-gd, gd, 0.0, 0.0))
    s.write_fields(_yprofile(g, gd * g.yc()), np.zeros(g.shape), np.zeros(g.shape), _identity_B(g))
    return s


def test_neo_hookean_simple_shear_exact():
    """No relaxation: dB_xy/dt = gd, dB_xx/dt = 2 gd B_xy; Euler-started AB2 gives B_xy = gd t and
    B_xx = 1 + gd^2 (t^2 - dt^2) exactly; RK3 integrates these polynomials exactly."""
    gd, dt = 0.7, 0.01
    s = _shear_solver(Rheology(model=oracle.NEO_HOOKEAN, mu_s=0.1, mu_p=2.0, lam=1.0), gd)
    for n in range(1, 40):
        s.step(dt, 1, flags=Solver.FREEZE_VELOCITY)
        t = n * dt
        assert np.abs(s.B[1] - gd * t).max() < 1e-13
        assert np.abs(s.B[0] - (1 + gd ** 2 * (t * t - dt * dt))).max() < 1e-13
        assert np.abs(s.B[3] - 1).max() < 1e-14
    r = _shear_solver(Rheology(model=oracle.NEO_HOOKEAN, mu_s=0.1, mu_p=2.0, lam=1.0), gd)
    r.step_rk3(0.05, 10, flags=Solver.FREEZE_VELOCITY)
    assert np.abs(r.B[1] - gd * 0.5).max() < 1e-13
    assert np.abs(r.B[0] - (1 + gd ** 2 * 0.25)).max() < 1e-13


def test_neo_hookean_is_saramito_far_below_yield():
    """F = a = 0 in both; the stresses G B and G (B - I) differ by an isotropic constant, which
    has no divergence."""
    g = Grid(12, 10, 8, 2 * np.pi, 2.0, np.pi, walls=True)
    u, v, w, B = (np.asarray(a) for a in _random_state(g, 3))
    out = []
    for model, ty in ((oracle.NEO_HOOKEAN, 0.0), (oracle.SARAMITO, 1e30)):
        s = Solver(g, Rheology(model=model, mu_s=0.01, mu_p=0.05, lam=0.5, tau_y=ty),
                   walls_uv=(0.1, -0.2, 0.0, 0.05))
        s.write_fields(u, v, w, B)
        s.step(1e-3, 3, flags=Solver.STOP_AFTER_PREDICTOR)
        out.append(s)
    assert np.array_equal(out[0].B, out[1].B)
    assert np.abs(out[0].u - out[1].u).max() < 1e-12
    assert np.abs(out[0].v - out[1].v).max() < 1e-12


def _random_state(g, seed):
    rng = np.random.default_rng(seed)
    u, v, w = (0.3 * rng.standard_normal(g.shape) for _ in range(3))
    if g.walls:
        v[:, -1, :] = 0.0
    B = _identity_B(g) + 0.05 * rng.standard_normal((6,) + g.shape)
    return u, v, w, B


def test_neo_hookean_elastic_shear_wave_recurrence():
    """u = eps sin y, B = I in a Neo-Hookean solid: per mode dA/dt = (-mu_s kc^2 A - G s C)/rho,
    dC/dt = s A (no relaxation); AB2 on this 2x2 system is an exact recurrence."""
    g = Grid(4, 32, 4, 1.0, 2 * np.pi, 1.0)
    mu_s, G, rho, eps, dt = 0.02, 0.5, 1.0, 0.3, 2e-3
    s = Solver(g, Rheology(model=oracle.NEO_HOOKEAN, rho=rho, mu_s=mu_s, mu_p=G, lam=1.0))
    y = g.yc()
    z = np.zeros(g.shape)
    s.write_fields(_yprofile(g, eps * np.sin(y)), z, z, _identity_B(g))
    dy = g.dy
    kc2 = 4 * np.sin(dy / 2) ** 2 / dy ** 2
    sg = np.sin(dy) / dy
    A, C, old = eps, 0.0, None
    for _ in range(200):
        f = ((-mu_s * kc2 * A - G * sg * C) / rho, sg * A)
        c1, c2 = (1.0, 0.0) if old is None else (1.5, -0.5)
        o = old or (0.0, 0.0)
        A, C = A + dt * (c1 * f[0] + c2 * o[0]), C + dt * (c1 * f[1] + c2 * o[1])
        old = f
    s.step(dt, 200)
    assert np.abs(s.u - _yprofile(g, A * np.sin(y))).max() < 1e-13
    assert np.abs(s.B[1] - _yprofile(g, C * np.cos(y))).max() < 1e-13


# ---------------------------------------------------------------------------------------------
# local artificial diffusion (Sec. 3.1)
# ---------------------------------------------------------------------------------------------

def test_artificial_diffusion_decay_recurrence():
    """B_xx = -1 + eps cos x (det B < 0 in every cell), no flow, no relaxation: each cell gets
    kappa lap_h B, so the mode decays by the AB2 recurrence of mu = -kappa (4/h^2) sin^2(h/2)."""
    n, kappa, eps, dt = 32, 0.05, 0.2, 1e-2
    L = 2 * np.pi
    g = Grid(n, 4, 4, L, L * 4 / n, L * 4 / n)
    s = Solver(g, Rheology(mu_s=0.0, mu_p=0.0, lam=1e300, kappa=kappa))
    x = (np.arange(n) + 0.5) * g.dx
    B = _identity_B(g)
    B[0] = (-1.0 + eps * np.cos(x))[None, None, :]
    z = np.zeros(g.shape)
    s.write_fields(z, z, z, B)
    mu = -kappa * 4 * np.sin(g.dx / 2) ** 2 / g.dx ** 2
    a, old = eps, None
    for _ in range(50):
        f = mu * a
        a = a + dt * (f if old is None else 1.5 * f - 0.5 * old)
        old = f
    s.step(dt, 50, flags=Solver.FREEZE_VELOCITY)
    assert np.abs(s.B[0] - (-1.0 + a * np.cos(x))[None, None, :]).max() < 1e-13
    assert np.abs(s.B[3] - 1).max() == 0.0


def _lap_periodic(g, f):
    return ((np.roll(f, -1, 2) - 2 * f + np.roll(f, 1, 2)) / g.dx ** 2
            + (np.roll(f, -1, 1) - 2 * f + np.roll(f, 1, 1)) / g.dy ** 2
            + (np.roll(f, -1, 0) - 2 * f + np.roll(f, 1, 0)) / g.dz ** 2)


@pytest.mark.parametrize("model", [oracle.OLDROYD_B, oracle.FENE_P])
def test_artificial_diffusion_only_where_triggered(model):
    g = Grid(12, 8, 8, 2.0, 2.0, 2.0)
    rng = np.random.default_rng(9)
    u, v, w = (0.2 * rng.standard_normal(g.shape) for _ in range(3))
    B = _identity_B(g) + 0.02 * rng.standard_normal((6,) + g.shape)
    L2 = 50.0
    B[1, 2:4, 3, 5:8] = 3.0                      # det B < 0 here
    if model == oracle.FENE_P:
        B[0, 5, 5, 1:3] = 0.97 * L2 - 2.0        # tr B ~ 0.97 L^2 >= 0.95 L^2 here
        B[0, 6, 5, 1:3] = 0.93 * L2 - 2.0        # tr B ~ 0.93 L^2 and not here
    r0 = Rheology(model=model, mu_s=0.01, mu_p=0.02, lam=0.5, L2=L2)
    r1 = Rheology(model=model, mu_s=0.01, mu_p=0.02, lam=0.5, L2=L2, kappa=0.3)
    rt0 = oracle.terms(g, r0, u, v, w, B)[0]
    rt1 = oracle.terms(g, r1, u, v, w, B)[0]
    det = (B[0] * (B[3] * B[5] - B[4] ** 2) - B[1] * (B[1] * B[5] - B[4] * B[2])
           + B[2] * (B[1] * B[4] - B[3] * B[2]))
    on = det < 0
    if model == oracle.FENE_P:
        on |= (B[0] + B[3] + B[5]) >= 0.95 * L2
    expect_on = np.zeros(g.shape, bool)
    expect_on[2:4, 3, 5:8] = True
    if model == oracle.FENE_P:
        expect_on[5, 5, 1:3] = True
    assert np.array_equal(on, expect_on)
    for c in range(6):
        assert np.array_equal(rt1[c][~on], rt0[c][~on])
        d = rt1[c][on] - rt0[c][on]
        ref = 0.3 * _lap_periodic(g, B[c])[on]
        assert np.allclose(d, ref, rtol=1e-12, atol=1e-12)


# ---------------------------------------------------------------------------------------------
# steady plane Poiseuille flow (Oldroyd-B, FENE-P): exact discrete fixed point
# ---------------------------------------------------------------------------------------------

def _steady_B(model, lam, L2, Lxy):
    """Steady homogeneous shear at rate Lxy: (B_xx, B_xy, B_yy) of Eq. (SRM2) with only L_xy."""
    if model == oracle.OLDROYD_B:
        return 1 + 2 * lam ** 2 * Lxy ** 2, lam * Lxy, 1.0
    a = L2 / (L2 - 3)
    Wi = lam * Lxy
    if Wi == 0:
        return 1.0, 0.0, 1.0                                 # at rest F = a and B = I

    def h(F):
        return F - L2 / (L2 - (3 * a / F + 2 * Wi ** 2 * a / F ** 3))
    F = brentq(h, 1.0, 1e6, xtol=1e-16, rtol=1e-15)
    return a / F + 2 * Wi ** 2 * a / F ** 3, Wi * a / F ** 2, a / F


def _tau_xy(model, lam, mu_p, L2, b):
    G = mu_p / lam
    if model == oracle.OLDROYD_B:
        return G * b[1]
    tr = b[0] + 2 * b[2]
    return G * L2 / (L2 - tr) * b[1]


def _poiseuille_residual(u, g, model, mu_s, mu_p, lam, L2, f):
    ny, dy = g.ny, g.dy
    ue = np.concatenate([[-u[0]], u, [-u[-1]]])           # no-slip ghosts
    Lxy = (ue[2:] - ue[:-2]) / (2 * dy)
    Bs = np.array([_steady_B(model, lam, L2, L) for L in Lxy])    # rows 0..ny-1: (xx, xy, yy)
    Be = np.vstack([2 * Bs[0] - Bs[1], Bs, 2 * Bs[-1] - Bs[-2]])  # linear ghosts
    t = np.array([_tau_xy(model, lam, mu_p, L2, b) for b in Be])
    edge = 0.5 * (t[1:] + t[:-1])                          # edges j-1/2 .. ny-1/2
    lap = (ue[2:] - 2 * ue[1:-1] + ue[:-2]) / dy ** 2
    return mu_s * lap + (edge[1:] - edge[:-1]) / dy + f, Bs


@pytest.mark.parametrize("model", [oracle.OLDROYD_B, oracle.FENE_P])
def test_steady_poiseuille_is_a_fixed_point(model):
    g = Grid(4, 16, 4, 1.0, 2.0, 1.0, walls=True)
    mu_s, mu_p, lam, L2, f = 0.3, 0.7, 0.8, 30.0, 1.5
    y = g.yc()
    u0 = f / (2 * (mu_s + mu_p)) * (1 - y ** 2)
    u = fsolve(lambda x: _poiseuille_residual(x, g, model, mu_s, mu_p, lam, L2, f)[0], u0,
               xtol=1e-13)
    res, Bs = _poiseuille_residual(u, g, model, mu_s, mu_p, lam, L2, f)
    assert np.abs(res).max() < 1e-11
    B = _identity_B(g)
    B[0] = _yprofile(g, Bs[:, 0])
    B[1] = _yprofile(g, Bs[:, 1])
    B[3] = _yprofile(g, Bs[:, 2])
    B[5] = _yprofile(g, Bs[:, 2])
    s = Solver(g, Rheology(model=model, mu_s=mu_s, mu_p=mu_p, lam=lam, L2=L2),
               forcing=(oracle.FORCE_CONST_X, f, 0.0))
    uu = _yprofile(g, u)
    z = np.zeros(g.shape)
    s.write_fields(uu, z, z, B)
    s.step(1e-3, 20)
    assert np.abs(s.u - uu).max() < 1e-11 * np.abs(u).max()
    assert np.abs(s.B - B).max() < 1e-11 * np.abs(B).max()
    assert np.abs(s.v).max() < 1e-12 and np.abs(s.w).max() < 1e-12
    if model == oracle.OLDROYD_B:
        # the fixed point tends to the parabola of the total viscosity as dy -> 0
        assert np.abs(u - u0).max() < 0.05 * u0.max()


# ---------------------------------------------------------------------------------------------
# oscillatory simple shear of the Saramito model
# ---------------------------------------------------------------------------------------------

def _saramito_rhs(t, b, G, lam, ty, gd_of_t):
    B = np.array([[b[0], b[1], b[2]], [b[1], b[3], b[4]], [b[2], b[4], b[5]]])
    tau = G * (B - np.eye(3))
    dev = tau - np.trace(tau) / 3 * np.eye(3)
    nrm = np.sqrt(0.5 * np.sum(dev * dev))
    F = max(0.0, 1 - ty / nrm) if nrm > 0 else 0.0
    Lm = np.zeros((3, 3))
    Lm[0, 1] = gd_of_t(t)
    dB = (F * np.eye(3) - F * B) / lam + Lm @ B + B @ Lm.T
    return [dB[0, 0], dB[0, 1], dB[0, 2], dB[1, 1], dB[1, 2], dB[2, 2]]


def test_saramito_oscillatory_shear_second_order():
    """Large-amplitude oscillatory shear, gd(t) = gd0 cos(w t): the material yields and
    re-solidifies twice per period; AB2 with the velocity reset every step converges at second
    order to a tight ODE solution."""
    G, lam, ty, gd0, om, T = 1.0, 1.0, 0.6, 2.0, 2.0, 3.0
    gd = lambda t: gd0 * np.cos(om * t)
    ref = solve_ivp(_saramito_rhs, (0, T), [1, 0, 0, 1, 0, 1], args=(G, lam, ty, gd),
                    method="DOP853", rtol=1e-12, atol=1e-13).y[:, -1]
    errs, solid, yielded = [], 0, 0
    for dt in (0.01, 0.005, 0.0025):
        s = _shear_solver(Rheology(model=oracle.SARAMITO, mu_s=0.1, mu_p=G * lam, lam=lam,
                                   tau_y=ty), gd(0.0))
        y = s.g.yc()
        n = int(round(T / dt))
        for m in range(n):
            g_now = gd(m * dt)
            s.u = _yprofile(s.g, g_now * y)
            s.walls_uv = (-g_now, g_now, 0.0, 0.0)
            s.step(dt, 1, flags=Solver.FREEZE_VELOCITY)
            F = oracle.closure(s.g, s.r, s.B)[0]
            solid += int(F.max() == 0.0)
            yielded += int(F.min() > 0.0)
        b = s.B[:, 0, 3, 1]
        errs.append(np.abs(b - ref).max())
    assert solid > 0 and yielded > 0          # the switch acts both ways within the run
    assert errs[2] < 1e-3
    assert 3.0 < errs[0] / errs[1] < 5.0 and 3.0 < errs[1] / errs[2] < 5.0, errs
