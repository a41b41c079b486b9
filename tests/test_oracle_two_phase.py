"""Pins of the oracle's two-phase (bubbly-flow) path, Sec. 3.2.

References: the single-phase oracle (C WENO5 lines, the plain projection, the single-phase step,
which the two-phase path must reproduce when both phases are equal), closed forms of a sphere
(volume, area, curvature), Laplace's law for a static drop, the exact discrete steady state of a
two-layer Couette flow solved as a linear system, convergence of level-set transport, and the
signed-distance property restored by reinitialisation.
"""
import numpy as np
import pytest

import oracle
from oracle import Grid, Rheology, Solver
from oracle import two_phase as tp


def _identity_B(g):
    B = np.zeros((6,) + g.shape)
    B[0] = B[3] = B[5] = 1.0
    return B


def _centres(g):
    x = (np.arange(g.nx) + 0.5) * g.dx
    y = g.y0 + (np.arange(g.ny) + 0.5) * g.dy
    z = (np.arange(g.nz) + 0.5) * g.dz
    return np.meshgrid(z, y, x, indexing="ij")[::-1]          # X, Y, Z of shape (nz, ny, nx)


def _sphere_distance(g, c, R):
    X, Y, Z = _centres(g)
    return np.sqrt((X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2) - R


def test_numpy_weno_matches_c_lines():
    g = Grid(32, 4, 4, 2 * np.pi, 1.0, 1.0)
    X, _, _ = _centres(g)
    f = np.sin(X) + 0.3 * np.cos(3 * X) + 0.1 * np.sign(np.sin(2 * X))
    m, p = tp.one_sided(g, f, 2)
    line = f[0, 0]
    assert np.allclose(m[0, 0], oracle.upwind_line(line, g.dx, 1.0), rtol=1e-13, atol=1e-13)
    assert np.allclose(p[0, 0], oracle.upwind_line(line, g.dx, -1.0), rtol=1e-13, atol=1e-13)


def test_level_set_transport_converges():
    """Smooth phi carried once around a periodic box by a uniform velocity (u, v) = (1, 0.5)."""
    errs = []
    for n in (32, 64):
        g = Grid(n, n, 4, 2 * np.pi, 2 * np.pi, 2 * np.pi * 4 / n)
        X, Y, _ = _centres(g)
        phi0 = np.cos(X) + 0.5 * np.sin(Y)
        dt = 0.5 * g.dx
        nsteps = int(round(2 * np.pi / dt))
        dt = 2 * np.pi / nsteps
        u = np.ones(g.shape)
        v = np.full(g.shape, 0.5)
        w = np.zeros(g.shape)
        phi = phi0
        for _ in range(nsteps):
            phi = tp.advect(g, phi, u, v, w, dt)
        exact = np.cos(X - 2 * np.pi) + 0.5 * np.sin(Y - np.pi)
        errs.append(np.abs(phi - exact).max())
    assert errs[1] < 2e-3 and errs[0] / errs[1] > 8, errs


def test_heaviside_and_delta_integrals():
    """Volume inside and area of a sphere from H and delta: within 2 % and second order in h."""
    ev, ea = [], []
    for n in (32, 64):
        g = Grid(n, n, n, 2 * np.pi, 2 * np.pi, 2 * np.pi)
        R = 1.2
        phi = _sphere_distance(g, (np.pi, np.pi, np.pi), R)
        vol = g.dx * g.dy * g.dz
        inside = np.sum(1.0 - tp.heaviside(g, phi)) * vol
        area = np.sum(tp.delta(g, phi)) * vol               # |grad phi| = 1 for a distance
        ev.append(abs(inside / (4 / 3 * np.pi * R ** 3) - 1))
        ea.append(abs(area / (4 * np.pi * R ** 2) - 1))
    assert ev[0] < 0.03 and ea[0] < 0.03, (ev, ea)
    assert ev[0] / ev[1] > 3 and ea[0] / ea[1] > 3, (ev, ea)


def test_curvature_of_a_sphere_second_order():
    errs = []
    for n in (32, 64):
        g = Grid(n, n, n, 2 * np.pi, 2 * np.pi, 2 * np.pi)
        R = 1.5
        phi = _sphere_distance(g, (np.pi + 0.1, np.pi - 0.2, np.pi + 0.05), R)
        kap = tp.curvature(g, phi)
        band = np.abs(phi) < g.dx
        ref = -2.0 / (R + phi[band])
        errs.append(np.abs(kap[band] - ref).max() / (2 / R))
    assert errs[0] < 0.05 and errs[0] / errs[1] > 3.0, errs


def test_surface_force_has_zero_resultant():
    g = Grid(32, 32, 32, 2 * np.pi, 2 * np.pi, 2 * np.pi)
    phi = _sphere_distance(g, (np.pi, np.pi, np.pi), 1.3)
    f = tp.surface_force(g, phi, 0.7)
    for c in range(3):
        assert abs(f[c].sum()) < 1e-12 * np.abs(f[c]).sum()


def test_reinitialisation_restores_distance_and_keeps_interface():
    g = Grid(48, 48, 4, 2 * np.pi, 2 * np.pi, 2 * np.pi * 4 / 48)
    X, Y, _ = _centres(g)
    r = np.sqrt((X - np.pi) ** 2 + (Y - np.pi) ** 2)
    phi0 = (r - 1.5) * (1.0 + 0.4 * np.cos(X))                 # right zero set, wrong slope
    phi = tp.reinitialise(g, phi0, 40)
    band = np.abs(r - 1.5) < 2 * g.dx
    gx = (np.roll(phi, -1, 2) - np.roll(phi, 1, 2)) / (2 * g.dx)
    gy = (np.roll(phi, -1, 1) - np.roll(phi, 1, 1)) / (2 * g.dy)
    slope = np.sqrt(gx ** 2 + gy ** 2)
    assert np.abs(slope[band] - 1).mean() < 0.03
    assert np.abs(phi[band] - (r[band] - 1.5)).max() < 0.15 * g.dx


def test_dong_shen_with_equal_densities_is_the_plain_projection():
    g = Grid(16, 12, 8, 2 * np.pi, 2.0, np.pi, walls=True)
    rng = np.random.default_rng(2)
    us, vs, ws, pn, pm = (rng.standard_normal(g.shape) for _ in range(5))
    vs[:, -1, :] = 0.0
    rho = np.full(g.shape, 1.3)
    a = tp.project_split(g, us, vs, ws, rho, 1.3, pn, pm, 1e-2)
    b = oracle.project(g, us, vs, ws, 1e-2, 1.3)
    for x, y in zip(a[:3], b[:3]):
        assert np.abs(x - y).max() < 1e-11 * np.abs(y).max()


def test_equal_phases_reduce_to_the_single_phase_step():
    g = Grid(16, 12, 8, 2 * np.pi, 2.0, np.pi, walls=True)
    rng = np.random.default_rng(3)
    u, v, w = (0.3 * rng.standard_normal(g.shape) for _ in range(3))
    v[:, -1, :] = 0.0
    u, v, w, _ = oracle.project(g, u, v, w, 1.0)
    B = _identity_B(g) + 0.05 * rng.standard_normal((6,) + g.shape)
    r = Rheology(model=oracle.SARAMITO, rho=1.2, mu_s=0.02, mu_p=0.05, lam=0.7, tau_y=0.01)
    walls = (0.1, -0.2, 0.0, 0.3)
    one = Solver(g, r, walls_uv=walls)
    one.write_fields(u, v, w, B)
    two = tp.TwoPhaseSolver(g, r, tp.TwoPhase(rho1=1.2, rho2=1.2, mu_s1=0.02, mu_s2=0.02,
                                              mu_p1=0.05, mu_p2=0.05, lam1=0.7, lam2=0.7),
                            walls_uv=walls)
    two.write_fields(u, v, w, B)
    two.write_level_set(_centres(g)[1] - 0.1)                    # a flat interface
    one.step(1e-3, 5)
    two.step(1e-3, 5)
    for k in ("u", "v", "w", "B"):
        a, b = getattr(one, k), getattr(two, k)
        assert np.abs(a - b).max() < 1e-11 * np.abs(a).max(), k


def test_static_drop_laplace_pressure():
    g = Grid(32, 32, 32, 2 * np.pi, 2 * np.pi, 2 * np.pi)
    R, sigma = 1.2, 0.5
    r = Rheology(model=oracle.OLDROYD_B, rho=1.0, mu_s=0.1, mu_p=0.0, lam=1.0)
    for rho2 in (1.0, 0.2):
        s = tp.TwoPhaseSolver(g, r, tp.TwoPhase(rho1=1.0, rho2=rho2, mu_s1=0.1, mu_s2=0.1,
                                                sigma=sigma, reinit_every=0))
        z = np.zeros(g.shape)
        s.write_fields(z, z, z, _identity_B(g))
        s.write_level_set(_sphere_distance(g, (np.pi, np.pi, np.pi), R))
        s.step(2e-3, 20)
        inside = s.phi < -0.5 * R
        outside = s.phi > 1.0
        jump = s.p[inside].mean() - s.p[outside].mean()
        assert abs(jump / (2 * sigma / R) - 1) < 0.08, (rho2, jump)
        assert max(np.abs(s.u).max(), np.abs(s.v).max(), np.abs(s.w).max()) < 0.02


def test_two_layer_couette_fixed_point():
    """Walls at y = -1, +1 moving at -1 and +1, fluid 1 above the flat interface y = 0.2 and
    fluid 2 below, viscosities 0.2 and 1.0 blended by H: the steady u(y) solves the 1D system of
    edge fluxes mu_e (u_{j+1} - u_j)/dy (mu_e the mean of the two rows, wall ghosts reflected)."""
    g = Grid(4, 24, 4, 1.0, 2.0, 1.0, walls=True)
    yc = g.yc()
    phi_y = yc - 0.2
    mu = 0.2 * tp.heaviside(g, phi_y) + 1.0 * (1 - tp.heaviside(g, phi_y))
    n, dy = g.ny, g.dy
    me = 0.5 * (mu[:-1] + mu[1:])                               # edges j+1/2, j = 0..n-2
    A = np.zeros((n, n))
    b = np.zeros(n)
    for j in range(n):
        if j < n - 1:
            A[j, j + 1] += me[j]; A[j, j] -= me[j]
        else:                                                   # top wall: ghost 2*1 - u
            A[j, j] -= 2 * mu[j]; b[j] -= mu[j] * 2 * 1.0
        if j > 0:
            A[j, j - 1] += me[j - 1]; A[j, j] -= me[j - 1]
        else:                                                   # bottom wall: ghost 2*(-1) - u
            A[j, j] -= 2 * mu[j]; b[j] -= mu[j] * 2 * (-1.0)
    u = np.linalg.solve(A, b)
    r = Rheology(model=oracle.OLDROYD_B, rho=1.0, mu_s=0.2, mu_p=0.0, lam=1.0)
    s = tp.TwoPhaseSolver(g, r, tp.TwoPhase(mu_s1=0.2, mu_s2=1.0, reinit_every=1,
                                            reinit_iters=1),
                          walls_uv=(-1.0, 1.0, 0.0, 0.0))
    z = np.zeros(g.shape)
    U = np.broadcast_to(u[None, :, None], g.shape).copy()
    s.write_fields(U, z, z, _identity_B(g))
    s.write_level_set(np.broadcast_to(phi_y[None, :, None], g.shape).copy())
    s.step(2e-3, 10)
    assert np.abs(s.u - U).max() < 1e-12
    assert np.abs(s.phi - phi_y[None, :, None]).max() < 1e-12


def test_translating_drop_keeps_its_volume():
    g = Grid(32, 32, 32, 2 * np.pi, 2 * np.pi, 2 * np.pi)
    R = 1.0
    r = Rheology(model=oracle.OLDROYD_B, rho=1.0, mu_s=0.05, mu_p=0.0, lam=1.0)
    s = tp.TwoPhaseSolver(g, r, tp.TwoPhase(mu_s1=0.05, mu_s2=0.05, sigma=0.0, reinit_every=5))
    one = np.ones(g.shape)
    z = np.zeros(g.shape)
    s.write_fields(one, z, z, _identity_B(g))
    s.write_level_set(_sphere_distance(g, (np.pi, np.pi, np.pi), R))
    vol0 = np.sum(1 - tp.heaviside(g, s.phi))
    s.step(0.02, 50)                                            # moves by one radius
    vol1 = np.sum(1 - tp.heaviside(g, s.phi))
    assert abs(vol1 / vol0 - 1) < 0.02
    assert np.abs(s.u - 1).max() < 1e-12
