"""Closed-form pins of the momentum and stress terms that the flows of test_oracle_flows.py leave
free: every face of the stress divergence in Eq. (ru), the velocity gradient of Eq. (SRM2) in every
orientation, the exchange symmetries of the step, and the start-up Poiseuille flow of Sec. 4.1.1
at the parameters of its figures.

* Fourier symbol of div(tau): with u = 0, mu_s = 0 and no force, one Euler predictor step gives
  RU = div_h(tau)/rho.  For tau built from single Fourier modes at the cell centres, every part of
  div_h has a closed form from trigonometric identities: the normal difference of tau_dd across a
  d-face multiplies the mode by -(2/h_d) sin(k_d h_d/2), the difference of the four-cell edge
  averages of tau_de multiplies it by -cos(k_d h_d/2) sin(k_e h_e)/h_e (both evaluated as
  sin(phase) at the face).  Oldroyd-B, Saramito and Neo-Hookean (tau = G (B - I) up to a
  constant) and FENE-P (tau = G (F B - a I), Table 1; with tr B = 3 everywhere F = a, so
  tau = G a (B - I)).  A wrong sign, spacing, index or average anywhere in div_h fails it.
* viscoelastic shear wave u_a = A sin(x_b) for all six ordered pairs a != b: the discrete problem
  is exactly linear (one 2x2 AB2 recurrence per mode for (A, B_ab), a driven scalar recurrence for
  B_aa - 1 through the upper-convected term), so each of the nine velocity-gradient entries and
  each off-diagonal stress face is pinned with its sign.
* exchange of x with y, and of y with z, on a periodic cube commutes with the step.
* start-up Poiseuille flow of an Oldroyd-B fluid (Sec. 4.1.1; Re, Wi and beta read from
  tests/golden/startup_poiseuille_params.json): the walls-and-ghosts discretisation converges at
  second order in (h, dt) to the continuum eigenfunction series of the start-up problem.
"""
import json
import os

import numpy as np
import pytest
import scipy.linalg

import oracle
from oracle import Grid, Rheology, Solver

HERE = os.path.dirname(os.path.abspath(__file__))
I6 = np.array([1.0, 0, 0, 1.0, 0, 1.0])
# component index of (a, b)
CIDX = {(0, 0): 0, (0, 1): 1, (1, 0): 1, (0, 2): 2, (2, 0): 2, (1, 1): 3, (1, 2): 4, (2, 1): 4,
        (2, 2): 5}


def _coords(g, face):
    """(x, y, z) of the points of a face family (-1: cell centres; 0, 1, 2: +x, +y, +z faces),
    broadcast to the grid shape (nz, ny, nx)."""
    h = (g.dx, g.dy, g.dz)
    n = (g.nx, g.ny, g.nz)
    out = []
    for d in range(3):
        c = (np.arange(n[d]) + (1.0 if d == face else 0.5)) * h[d]
        shp = [1, 1, 1]
        shp[2 - d] = n[d]
        out.append(np.broadcast_to(c.reshape(shp), g.shape))
    return out


def _modes():
    """Two Fourier modes per stress component (integer wave vectors, amplitude, phase)."""
    rng = np.random.default_rng(20180326)
    m = {}
    for c in range(6):
        m[c] = [(tuple(int(v) for v in rng.integers(-2, 3, size=3)), float(rng.uniform(0.5, 1.5)),
                 float(rng.uniform(0, 2 * np.pi))) for _ in range(2)]
    return m


def _eval_modes(modes, X, fn=np.cos):
    x, y, z = X
    return sum(a * fn(k[0] * x + k[1] * y + k[2] * z + ph) for k, a, ph in modes)


def _symbol_divergence(g, tmodes):
    """Expected div_h(tau) on the three face families for tau_c = sum a cos(k.x + phase)."""
    h = (g.dx, g.dy, g.dz)
    T = np.zeros((3,) + g.shape)
    for d in range(3):
        X = _coords(g, d)
        for e in range(3):
            for k, a, ph in tmodes[CIDX[(d, e)]]:
                s = np.sin(k[0] * X[0] + k[1] * X[1] + k[2] * X[2] + ph)
                if e == d:
                    fac = -(2.0 / h[d]) * np.sin(k[d] * h[d] / 2)
                else:
                    fac = -np.cos(k[d] * h[d] / 2) * np.sin(k[e] * h[e]) / h[e]
                T[d] += a * fac * s
    return T


@pytest.mark.parametrize("model", ["oldroyd_b", "saramito", "neo_hookean", "fene_p"])
def test_stress_divergence_fourier_symbol(model):
    # periodic box 2 pi in each direction, different cell counts: three different spacings
    g = Grid(16, 12, 10, 2 * np.pi, 2 * np.pi, 2 * np.pi)
    rho, mu_p, lam, L2 = 1.7, 0.3, 0.6, 12.0
    G = mu_p / lam
    kw = dict(rho=rho, mu_s=0.0, mu_p=mu_p, lam=lam)
    r = {"oldroyd_b": Rheology(model=oracle.OLDROYD_B, **kw),
         "saramito": Rheology(model=oracle.SARAMITO, tau_y=0.05, **kw),
         "neo_hookean": Rheology(model=oracle.NEO_HOOKEAN, **kw),
         "fene_p": Rheology(model=oracle.FENE_P, L2=L2, **kw)}[model]
    modes = _modes()
    eps = 0.01
    Xc = _coords(g, -1)
    Bm = np.stack([eps * _eval_modes(modes[c], Xc) for c in range(6)])
    if model == "fene_p":
        Bm[5] = -(Bm[0] + Bm[3])           # tr B = 3 in every cell: F = a
        modes[5] = [(k, -eps * a, ph) for k, a, ph in modes[0]] + \
                   [(k, -eps * a, ph) for k, a, ph in modes[3]]
        for c in (0, 1, 2, 3, 4):
            modes[c] = [(k, eps * a, ph) for k, a, ph in modes[c]]
        scale = G * L2 / (L2 - 3.0)
    else:
        modes = {c: [(k, eps * a, ph) for k, a, ph in modes[c]] for c in range(6)}
        scale = G
    tmodes = {c: [(k, scale * a, ph) for k, a, ph in modes[c]] for c in range(6)}
    B = Bm + I6[:, None, None, None]
    z = np.zeros(g.shape)
    s = Solver(g, r)
    s.write_fields(z, z, z, B)
    s.step(1e-3, 1, flags=Solver.STOP_AFTER_PREDICTOR)
    expect = _symbol_divergence(g, tmodes) / rho
    tol = 1e-13 * np.abs(expect).max()
    assert np.abs(s.RU - expect).max() < tol, np.abs(s.RU - expect).max() / np.abs(expect).max()
    # the stress right-hand side at rest is the relaxation of Table 1 alone
    if model == "oldroyd_b":
        assert np.abs(s.RT + Bm / lam).max() < 1e-15


PAIRS = [(a, b) for a in range(3) for b in range(3) if a != b]


@pytest.mark.parametrize("a,b", PAIRS)
def test_shear_wave_every_orientation(a, b):
    n = [4, 4, 4]
    n[b] = 32
    L = [1.0, 1.0, 1.0]
    L[b] = 2 * np.pi
    g = Grid(n[0], n[1], n[2], *L)
    mu_s, mu_p, lam, rho, eps, dt = 0.05, 0.2, 0.7, 1.3, 0.3, 2e-3
    s = Solver(g, Rheology(model=oracle.OLDROYD_B, rho=rho, mu_s=mu_s, mu_p=mu_p, lam=lam))
    xf = _coords(g, a)[b]            # x_b at the a-faces
    xc = _coords(g, -1)[b]           # x_b at the centres
    vel = [np.zeros(g.shape) for _ in range(3)]
    vel[a] = eps * np.sin(xf)
    B = np.broadcast_to(I6[:, None, None, None], (6,) + g.shape).copy()
    s.write_fields(*vel, B)
    h = (g.dx, g.dy, g.dz)[b]
    G = mu_p / lam
    kc2 = 4 * np.sin(h / 2) ** 2 / h ** 2
    sg = np.sin(h) / h

    def rhs(A, C, D):
        # u_a = A sin(x_b), B_ab = C cos(x_b), B_aa - 1 = D cos^2(x_b)
        return ((-mu_s * kc2 * A - G * sg * C) / rho, sg * A - C / lam, 2 * sg * A * C - D / lam)

    st = np.array([eps, 0.0, 0.0])
    old = None
    nsteps = 120
    for _ in range(nsteps):
        f = np.array(rhs(*st))
        st = st + dt * (f if old is None else 1.5 * f - 0.5 * old)
        old = f
    s.step(dt, nsteps)
    A, C, D = st
    got = (s.u, s.v, s.w)
    assert np.abs(got[a] - A * np.sin(xf)).max() < 1e-13
    for c in range(3):
        if c != a:
            assert np.abs(got[c]).max() < 1e-13
    assert np.abs(s.B[CIDX[(a, b)]] - C * np.cos(xc)).max() < 1e-13
    assert np.abs(s.B[CIDX[(a, a)]] - 1.0 - D * np.cos(xc) ** 2).max() < 1e-13
    for c in range(6):
        if c not in (CIDX[(a, b)], CIDX[(a, a)]):
            assert np.abs(s.B[c] - I6[c]).max() < 1e-13, c


def _random_solenoidal(g, rng, amp):
    u, v, w = (amp * rng.standard_normal(g.shape) for _ in range(3))
    u, v, w, _ = oracle.project(g, u, v, w, 1.0)
    return u, v, w


def _exchange(fields, p, q):
    """Exchange directions p and q (0 = x, 1 = y, 2 = z) of a state on a cube: array axes,
    velocity components and tensor indices."""
    u, v, w, B = fields
    ax = {0: -1, 1: -2, 2: -3}
    t = lambda x: np.ascontiguousarray(np.swapaxes(x, ax[p], ax[q]))
    vel = [t(u), t(v), t(w)]
    vel[p], vel[q] = vel[q], vel[p]
    perm = [0, 1, 2]
    perm[p], perm[q] = q, p
    Bs = np.empty_like(B)
    for (i, j), c in CIDX.items():
        Bs[CIDX[(perm[i], perm[j])]] = t(B[c])
    return vel[0], vel[1], vel[2], Bs


@pytest.mark.parametrize("p,q", [(0, 1), (1, 2)])
@pytest.mark.parametrize("model", [oracle.FENE_P, oracle.SARAMITO])
def test_exchange_equivariance(p, q, model):
    n = 10
    g = Grid(n, n, n, 2.0, 2.0, 2.0)
    rng = np.random.default_rng(17 + p + q)
    u, v, w = _random_solenoidal(g, rng, 0.5)
    B = np.broadcast_to(I6[:, None, None, None], (6,) + g.shape) \
        + 0.05 * rng.standard_normal((6,) + g.shape)
    r = Rheology(model=model, mu_s=0.01, mu_p=0.03, lam=0.5, L2=50.0, tau_y=0.004)
    a, b = Solver(g, r), Solver(g, r)
    a.write_fields(u, v, w, B)
    b.write_fields(*_exchange((u, v, w, B), p, q))
    for s in (a, b):
        s.step(2e-3, 4)
    su, sv, sw, sB = _exchange((a.u, a.v, a.w, a.B), p, q)
    for x, y in ((su, b.u), (sv, b.v), (sw, b.w), (sB, b.B)):
        assert np.abs(x - y).max() < 1e-12


def _poiseuille_continuum(y, t, f, mu_s, mu_p, lam, rho, nmodes=3000):
    """u and tau_xy of an Oldroyd-B fluid at rest between walls y = -1, +1, driven from t = 0 by a
    constant body force f: the steady profile plus the decaying modes cos(k y), sin(k y),
    k = (m + 1/2) pi, each a 2x2 linear ODE  rho a' = -mu_s k^2 a + k s,
    lam s' + s = -mu_p k a, started from minus the steady profile's coefficients."""
    mu0 = mu_s + mu_p
    u = f / (2 * mu0) * (1 - y ** 2)
    tau = -mu_p * f / mu0 * y
    for m in range(nmodes):
        k = (m + 0.5) * np.pi
        sgn = (-1.0) ** m
        a0 = -(f / (2 * mu0)) * 4 * sgn / k ** 3
        s0 = (mu_p * f / mu0) * 2 * sgn / k ** 2
        M = np.array([[-mu_s * k * k / rho, k / rho], [-mu_p * k / lam, -1.0 / lam]])
        am, sm = scipy.linalg.expm(M * t) @ np.array([a0, s0])
        u += am * np.cos(k * y)
        tau += sm * np.sin(k * y)
    return u, tau


def test_startup_poiseuille_oldroyd_b_paper_parameters():
    """Sec. 4.1.1, Eq. (PRESS): h = 2 (walls at y = -1, +1), u0 = 1, rho = 1 give
    mu_s + mu_p = rho u0 h / Re, lambda = Wi h / u0 and -dp/dx = 8 (mu_s + mu_p) u0 / h^2 (applied
    as the body force).  Compared at T = t (mu_s + mu_p)/(rho h^2) = 1, in the middle of the
    overshoots of the start-up."""
    prm = json.load(open(os.path.join(HERE, "golden", "startup_poiseuille_params.json")))
    Re, Wi, beta = prm["Re"], prm["Wi"], prm["beta"]
    h, u0, rho = 2.0, 1.0, 1.0
    mu0 = rho * u0 * h / Re
    mu_s, mu_p, lam = beta * mu0, (1 - beta) * mu0, Wi * h / u0
    f = 8 * mu0 * u0 / h ** 2
    t_end = 1.0 * rho * h ** 2 / mu0
    errs = []
    for ny, dt in ((16, 5e-4), (32, 1.25e-4)):
        g = Grid(4, ny, 4, 1.0, h, 1.0, walls=True)
        r = Rheology(model=oracle.OLDROYD_B, rho=rho, mu_s=mu_s, mu_p=mu_p, lam=lam)
        s = Solver(g, r, forcing=(oracle.FORCE_CONST_X, f, 0.0))
        z = np.zeros(g.shape)
        s.write_fields(z, z, z, np.broadcast_to(I6[:, None, None, None], (6,) + g.shape))
        s.step(dt, int(round(t_end / dt)))
        y = g.yc()
        u_ex, tau_ex = _poiseuille_continuum(y, t_end, f, mu_s, mu_p, lam, rho)
        tau = oracle.stress(g, r, s.B)[1]
        errs.append(max(np.abs(s.u[0, :, 0] - u_ex).max() / u0,
                        np.abs(tau[0, :, 0] - tau_ex).max() / (mu0 * u0 / h)))
        assert np.abs(s.u - s.u[:1, :, :1]).max() < 1e-13
        assert np.abs(s.v).max() < 1e-13 and np.abs(s.w).max() < 1e-13
    # the centreline velocity is of order u0: the start-up has been resolved, not damped out
    assert errs[1] < 1e-2 and 3.3 < errs[0] / errs[1] < 4.7, errs
