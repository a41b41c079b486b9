"""Pins of the oracle's stress advection: fifth-order WENO (Sec. 3.1) and its use in u.grad(B)
of Eq. (rt).

Checked against facts the scheme must satisfy: every candidate stencil is exact for cubics, so the
WENO derivative is exact for cubics whatever the weights; the error on smooth data falls as h^5;
upwinding picks the side the velocity comes from; and in 3D, pure transport by a uniform velocity
translates the pattern (exact solution B(x - U t)).
"""
import numpy as np
import pytest

import oracle
from oracle import Grid, Rheology, Solver


@pytest.mark.parametrize("vel", [1.0, -1.0])
def test_weno_exact_for_cubics(vel):
    n, h = 40, 0.1
    x = np.arange(n) * h
    f = 0.3 * x ** 3 - x ** 2 + 2 * x + 1
    d = oracle.weno5_line(f, h, vel)
    exact = 0.9 * x ** 2 - 2 * x + 2
    interior = slice(4, n - 4)          # away from the periodic seam
    assert np.abs(d - exact)[interior].max() < 1e-12 * np.abs(exact).max()


@pytest.mark.parametrize("vel", [1.0, -1.0])
def test_weno_fifth_order_on_smooth_data(vel):
    errs = []
    for n in (32, 64, 128):
        h = 2 * np.pi / n
        x = np.arange(n) * h
        errs.append(np.abs(oracle.weno5_line(np.sin(x), h, vel) - np.cos(x)).max())
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 26.0 < r1 < 40.0 and 26.0 < r2 < 40.0, errs


def test_weno_upwind_side():
    """At a step, the stencil on the upwind side sees nothing of the jump."""
    n, h, m = 24, 1.0, 12
    f = np.where(np.arange(n) >= m, 1.0, 0.0)
    left = oracle.weno5_line(f, h, +1.0)
    right = oracle.weno5_line(f, h, -1.0)
    assert left[m - 3] == 0.0 and right[m - 3] != 0.0
    assert right[m + 2] == 0.0 and left[m + 2] != 0.0
    # no overshoot of the jump size (essentially non-oscillatory)
    assert np.all(np.abs(left) <= 1.0 / h + 1e-12) and np.all(np.abs(right) <= 1.0 / h + 1e-12)


def test_weno_linear_weights_on_quadratic_data():
    """Quadratic data make the three smoothness indicators equal, so the weights are the linear
    ones (0.1, 0.6, 0.3) and the result is the fifth-order upwind combination of v1..v5."""
    n, h = 30, 0.2
    x = np.arange(n) * h
    f = 1.7 * x ** 2 - 0.4 * x
    d = oracle.weno5_line(f, h, 1.0)
    v = np.diff(f) / h                  # v[m] = D-f at m+1
    i = 12
    v1, v2, v3, v4, v5 = v[i - 3], v[i - 2], v[i - 1], v[i], v[i + 1]
    lin = v1 / 30 - 13 * v2 / 60 + 47 * v3 / 60 + 27 * v4 / 60 - v5 / 20
    assert abs(d[i] - lin) < 1e-12 * abs(lin)


def _advect(axis, vel, n=32, t_end=0.25, dt=2.5e-3):
    """Transport of a smooth B pattern by a uniform velocity along one axis (velocity frozen,
    relaxation switched off by lambda -> infinity)."""
    L = 2 * np.pi
    shape = [4, 4, 4]
    shape[2 - axis] = n
    nz, ny, nx = shape
    g = Grid(nx, ny, nz, L * nx / n, L * ny / n, L * nz / n)
    r = Rheology(model=oracle.OLDROYD_B, mu_s=0.0, mu_p=0.0, lam=1e30)
    s = Solver(g, r)
    h = L / n
    c = (np.arange(n) + 0.5) * h
    prof = lambda xx: np.sin(xx) + 0.3 * np.cos(2 * xx)
    B = np.zeros((6, nz, ny, nx))
    sl = [None, None, None]
    sl[2 - axis] = slice(None)
    base = prof(c)[tuple(sl)]
    for comp in range(6):
        B[comp] = (1.0 if comp in (0, 3, 5) else 0.0) + (0.1 * (comp + 1)) * base
    vel_f = [np.zeros(g.shape) for _ in range(3)]
    vel_f[axis][:] = vel
    s.write_fields(*vel_f, B)
    nsteps = int(round(t_end / dt))
    s.step(dt, nsteps, flags=Solver.FREEZE_VELOCITY)
    exact = prof(c - vel * nsteps * dt)[tuple(sl)]
    err = 0.0
    for comp in range(6):
        ref = (1.0 if comp in (0, 3, 5) else 0.0) + (0.1 * (comp + 1)) * exact
        err = max(err, np.abs(s.B[comp] - ref).max())
    return err


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("vel", [1.0, -1.0])
def test_uniform_transport_translates_pattern(axis, vel):
    e32 = _advect(axis, vel, n=32, dt=1e-3)
    e64 = _advect(axis, vel, n=64, dt=1e-3)
    # WENO5 converges at fifth order on smooth data (slower at n = 32, where the nonlinear
    # weights still act at the extrema); a wrong spacing, axis or upwind side gives O(h) errors
    assert e64 < 2e-5 and e32 / e64 > 16.0, (e32, e64)


def test_transport_is_axis_and_direction_symmetric():
    """The same pattern moved along x, y or z, forwards or backwards, gives the same error."""
    errs = [_advect(ax, v, n=16, dt=2e-3) for ax in (0, 1, 2) for v in (1.0, -1.0)]
    assert max(errs) - min(errs) <= 1e-12 * max(errs)
