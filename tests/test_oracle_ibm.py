"""Pins of the oracle's volume-penalisation immersed boundary (Sec. 3.3.2, Eqs. (Vol) and
(forceAdded)) with both integrators.

References: bitwise no-op at zero solid fraction; exact discrete steady channel flows between
penalised slabs (the fixed point of the one-step map solved directly as a linear system, fractional
interface rows included; a viscoelastic version solved with a nonlinear solver from the 1D
staggered definitions); the discrete parabola between fully solid rows under RK3.
"""
import numpy as np
import pytest

import oracle
from oracle import Grid, Rheology, Solver
from paper_1803_09563_amd import inputs


def _identity_B(g):
    B = np.zeros((6,) + g.shape)
    B[0] = B[3] = B[5] = 1.0
    return B


def _rows(g, prof):
    return np.broadcast_to(np.asarray(prof, dtype=float)[None, :, None], g.shape).copy()


@pytest.mark.parametrize("rk3", [False, True])
def test_zero_fraction_is_a_no_op(rk3):
    g = Grid(12, 10, 8, 2 * np.pi, 2.0, np.pi, walls=True)
    u, v, w, B = inputs.random_state(g.shape, 5, walls=True)
    out = []
    for solid in (False, True):
        s = Solver(g, Rheology(model=oracle.FENE_P, mu_s=0.01, mu_p=0.02, lam=0.5, L2=40.0),
                   walls_uv=(0.1, -0.2, 0.0, 0.05))
        s.write_fields(u, v, w, B)
        if solid:
            s.set_solid([np.zeros(g.shape)] * 3)
        (s.step_rk3 if rk3 else s.step)(1e-3, 3)
        out.append(s)
    for k in ("u", "v", "w", "p", "B"):
        assert np.array_equal(getattr(out[0], k), getattr(out[1], k)), k


def _slab_alpha(g, frac):
    """Rows 0, 1 solid, rows 2 and ny-1 partly solid (frac), the rest fluid; u- and w-points."""
    a = np.zeros(g.ny)
    a[:2] = 1.0
    a[2] = a[-1] = frac
    return a


@pytest.mark.parametrize("frac", [0.0, 0.4])
def test_newtonian_slab_channel_fixed_point(frac):
    """Periodic box with penalised slabs, constant f_x, Newtonian: the steady state satisfies
    u_j = (1 - alpha_j)(u_j + dt (nu D2 u + f)_j) row by row -- a linear system."""
    g = Grid(4, 16, 4, 1.0, 2.0, 1.0)
    nu, f, dt = 0.5, 2.0, 2e-3
    a = _slab_alpha(g, frac)
    n = g.ny
    D2 = (np.roll(np.eye(n), 1, 1) - 2 * np.eye(n) + np.roll(np.eye(n), -1, 1)) / g.dy ** 2
    M = np.eye(n) - np.diag(1 - a) @ (np.eye(n) + dt * nu * D2)
    u = np.linalg.solve(M, (1 - a) * dt * f)
    s = Solver(g, Rheology(mu_s=nu, mu_p=0.0), forcing=(oracle.FORCE_CONST_X, f, 0.0))
    z = np.zeros(g.shape)
    s.write_fields(_rows(g, u), z, z, _identity_B(g))
    s.set_solid([_rows(g, a), np.zeros(g.shape), _rows(g, a)])
    s.step(dt, 30)
    assert np.abs(s.u - _rows(g, u)).max() < 1e-13 * np.abs(u).max()
    assert np.abs(s.v).max() < 1e-14 and np.abs(s.w).max() < 1e-14
    assert (u[:2] == 0).all() and u[5] > 0


def test_rk3_keeps_the_parabola_between_solid_rows():
    g = Grid(4, 16, 4, 1.0, 2.0, 1.0)
    nu, f = 0.5, 2.0
    a = np.zeros(g.ny)
    a[:3] = 1.0
    j = np.arange(g.ny)
    u = np.where(a > 0, 0.0, f / (2 * nu) * (j - 2) * (g.ny - j) * g.dy ** 2)
    for rk3 in (False, True):
        s = Solver(g, Rheology(mu_s=nu, mu_p=0.0), forcing=(oracle.FORCE_CONST_X, f, 0.0))
        z = np.zeros(g.shape)
        s.write_fields(_rows(g, u), z, z, _identity_B(g))
        s.set_solid([_rows(g, a), np.zeros(g.shape), _rows(g, a)])
        (s.step_rk3 if rk3 else s.step)(2e-3, 20)
        assert np.abs(s.u - _rows(g, u)).max() < 1e-13 * u.max()


def test_oldroyd_b_slab_channel_fixed_point():
    """Viscoelastic channel between fully solid slabs: unknown u at fluid rows; B from the
    steady homogeneous-shear relation at every row (solid rows included, their L_xy comes from
    the neighbouring fluid); tau_xy edge averages; the 1D system solved directly."""
    g = Grid(4, 16, 4, 1.0, 2.0, 1.0)
    mu_s, mu_p, lam, f = 0.3, 0.7, 0.8, 1.5
    solid = np.zeros(g.ny, bool)
    solid[:3] = True
    fl = ~solid
    dy = g.dy

    def full(x):
        u = np.zeros(g.ny)
        u[fl] = x
        return u

    def state(u):
        Lxy = (np.roll(u, -1) - np.roll(u, 1)) / (2 * dy)
        bxx, bxy = 1 + 2 * lam ** 2 * Lxy ** 2, lam * Lxy
        return bxx, bxy

    def resid(x):
        u = full(x)
        _, bxy = state(u)
        t = mu_p / lam * bxy
        edge = 0.5 * (t + np.roll(t, -1))                      # edge j+1/2
        lap = (np.roll(u, -1) - 2 * u + np.roll(u, 1)) / dy ** 2
        return (mu_s * lap + (edge - np.roll(edge, 1)) / dy + f)[fl]

    # Oldroyd-B: tau_xy = mu_p L_xy, the residual is affine in u -- assemble it column by column
    m = int(fl.sum())
    r0 = resid(np.zeros(m))
    A = np.stack([resid(e) - r0 for e in np.eye(m)], axis=1)
    x = np.linalg.solve(A, -r0)
    assert np.abs(resid(x)).max() < 1e-10
    u = full(x)
    bxx, bxy = state(u)
    B = _identity_B(g)
    B[0], B[1] = _rows(g, bxx), _rows(g, bxy)
    s = Solver(g, Rheology(model=oracle.OLDROYD_B, mu_s=mu_s, mu_p=mu_p, lam=lam),
               forcing=(oracle.FORCE_CONST_X, f, 0.0))
    z = np.zeros(g.shape)
    s.write_fields(_rows(g, u), z, z, B)
    a = solid.astype(float)
    s.set_solid([_rows(g, a), np.zeros(g.shape), _rows(g, a)])
    s.step(1e-3, 20)
    assert np.abs(s.u - _rows(g, u)).max() < 1e-10 * u.max()
    assert np.abs(s.B - B).max() < 1e-10 * np.abs(B).max()


def test_sphere_fractions_volume():
    """The input generator's fractions integrate to the sphere volume (to sampling accuracy)."""
    wl = inputs.kolmogorov_saramito(32)
    R = 1.0
    au, av, aw = inputs.solid_fractions(wl, inputs.sphere((np.pi, np.pi, np.pi), R), sub=4)
    vol = 4 / 3 * np.pi * R ** 3
    for a in (au, av, aw):
        assert a.min() >= 0 and a.max() <= 1
        assert abs(a.sum() * wl.dx * wl.dy * wl.dz - vol) < 0.02 * vol
