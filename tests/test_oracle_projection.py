"""Pins of the oracle's projection (Sec. 3.2.2, Eqs. (var poisson), (projection)).

The oracle solves L_h p = r with the discrete Fourier transform (periodic directions) and a
Thomas sweep (wall-normal direction).  Here it is checked against things it does not use:
closed-form eigenpairs of the 7-point Laplacian, a sparse matrix assembled cell by cell and solved
with scipy's direct solver, scipy's banded solver, and the properties a projection must have.
"""
import numpy as np
import pytest
import scipy.linalg
import scipy.sparse
import scipy.sparse.linalg

import oracle
from oracle import Grid


def _centres(n, h, x0=0.0):
    return x0 + (np.arange(n) + 0.5) * h


def _sparse_laplacian(g: Grid):
    """7-point Laplacian of cell values, assembled cell by cell: periodic in x and z, periodic or
    homogeneous-Neumann (wall) in y."""
    nx, ny, nz = g.nx, g.ny, g.nz
    idx = lambda i, j, k: (k * ny + j) * nx + i
    rows, cols, vals = [], [], []
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                q = idx(i, j, k)
                diag = 0.0
                for (di, dj, dk, h) in ((1, 0, 0, g.dx), (-1, 0, 0, g.dx), (0, 1, 0, g.dy),
                                        (0, -1, 0, g.dy), (0, 0, 1, g.dz), (0, 0, -1, g.dz)):
                    jj = j + dj
                    if g.walls and (jj < 0 or jj >= ny):
                        continue        # no flux through a wall
                    jj %= ny
                    rows.append(q); cols.append(idx((i + di) % nx, jj, (k + dk) % nz))
                    vals.append(1.0 / h ** 2)
                    diag -= 1.0 / h ** 2
                rows.append(q); cols.append(q); vals.append(diag)
    n = nx * ny * nz
    return scipy.sparse.csr_matrix((vals, (rows, cols)), shape=(n, n))


def _brute_solve(g: Grid, r):
    """Zero-mean solution by a direct sparse solve with one node pinned."""
    A = _sparse_laplacian(g).tolil()
    b = r.ravel().copy()
    A[0, :] = 0.0
    A[0, 0] = 1.0
    b[0] = 0.0
    p = scipy.sparse.linalg.spsolve(A.tocsr(), b).reshape(g.shape)
    return p - p.mean()


@pytest.mark.parametrize("walls", [False, True])
@pytest.mark.parametrize("shape", [(8, 8, 8), (8, 6, 4), (6, 10, 4)])
def test_poisson_matches_sparse_direct_solve(walls, shape):
    nx, ny, nz = shape
    g = Grid(nx, ny, nz, 1.3, 2.0, 0.7, walls=walls)
    rng = np.random.default_rng(11)
    p_ex = rng.standard_normal(g.shape)
    p_ex -= p_ex.mean()
    r = (_sparse_laplacian(g) @ p_ex.ravel()).reshape(g.shape)
    p = oracle.solve_poisson(g, r)
    assert np.abs(p - p_ex).max() <= 1e-12 * np.abs(p_ex).max() * 10
    pb = _brute_solve(g, r)
    assert np.abs(p - pb).max() <= 1e-11 * np.abs(pb).max()


def test_sparse_laplacian_equals_div_grad():
    """The assembled matrix is D_h G_h of the oracle (both walls and periodic)."""
    for walls in (False, True):
        g = Grid(6, 5, 4, 1.0, 1.5, 2.0, walls=walls)
        p = np.random.default_rng(3).standard_normal(g.shape)
        gx, gy, gz = oracle.gradient(g, p)
        lap = oracle.divergence(g, gx, gy, gz)
        ref = (_sparse_laplacian(g) @ p.ravel()).reshape(g.shape)
        assert np.abs(lap - ref).max() < 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("n", [16, 24, 32])
def test_poisson_periodic_eigenfunction(n):
    """cos/sin modes on cell centres are eigenvectors with eigenvalue -(4/h^2) sin^2(pi m/N)."""
    g = Grid(n, n // 2 * 2, n // 2, 2.0, 3.0, 1.0)
    mx, my, mz = 3, 2, 1
    xc = _centres(g.nx, g.dx)[None, None, :]
    yc = _centres(g.ny, g.dy)[None, :, None]
    zc = _centres(g.nz, g.dz)[:, None, None]
    p = np.cos(2 * np.pi * mx * xc / g.lx) * np.cos(2 * np.pi * my * yc / g.ly) \
        * np.sin(2 * np.pi * mz * zc / g.lz)
    lam = -(4 / g.dx ** 2) * np.sin(np.pi * mx / g.nx) ** 2 \
          - (4 / g.dy ** 2) * np.sin(np.pi * my / g.ny) ** 2 \
          - (4 / g.dz ** 2) * np.sin(np.pi * mz / g.nz) ** 2
    out = oracle.solve_poisson(g, lam * p)
    assert np.abs(out - p).max() < 1e-12


@pytest.mark.parametrize("ny", [8, 13, 32])
def test_poisson_wall_eigenfunction(ny):
    """Neumann eigenvectors cos(pi m (j+1/2)/Ny) in y with eigenvalue -(4/dy^2) sin^2(pi m/(2Ny))."""
    g = Grid(8, ny, 4, 2.0, 2.0, 1.0, walls=True)
    for (mx, my, mz) in ((0, 1, 0), (1, 3, 1), (2, ny - 1, 0)):
        xc = _centres(g.nx, g.dx)[None, None, :]
        zc = _centres(g.nz, g.dz)[:, None, None]
        jj = np.arange(g.ny)[None, :, None]
        p = np.cos(2 * np.pi * mx * xc / g.lx) * np.cos(np.pi * my * (jj + 0.5) / g.ny) \
            * np.cos(2 * np.pi * mz * zc / g.lz)
        lam = -(4 / g.dx ** 2) * np.sin(np.pi * mx / g.nx) ** 2 \
              - (4 / g.dy ** 2) * np.sin(np.pi * my / (2 * g.ny)) ** 2 \
              - (4 / g.dz ** 2) * np.sin(np.pi * mz / g.nz) ** 2
        out = oracle.solve_poisson(g, lam * p)
        assert np.abs(out - p).max() < 1e-12


def test_thomas_matches_solve_banded():
    rng = np.random.default_rng(5)
    for n in (2, 3, 17, 256):
        a = rng.uniform(0.5, 1.0, n)
        c = rng.uniform(0.5, 1.0, n)
        b = -(a + c) - rng.uniform(0.1, 1.0, n)      # diagonally dominant
        d = rng.standard_normal((n, 4)) + 1j * rng.standard_normal((n, 4))
        x = oracle.thomas(a[:, None], b[:, None], c[:, None], d)
        ab = np.zeros((3, n))
        ab[0, 1:] = c[:-1]
        ab[1] = b
        ab[2, :-1] = a[1:]
        ref = scipy.linalg.solve_banded((1, 1), ab, d)
        assert np.abs(x - ref).max() < 1e-13 * max(1.0, np.abs(ref).max())


def _random_velocity(g, rng, amp=1.0):
    u = amp * rng.standard_normal(g.shape)
    v = amp * rng.standard_normal(g.shape)
    w = amp * rng.standard_normal(g.shape)
    if g.walls:
        v[:, -1, :] = 0.0
    return u, v, w


@pytest.mark.parametrize("walls", [False, True])
def test_projection_is_solenoidal_and_idempotent(walls):
    g = Grid(16, 12, 8, 2 * np.pi, 2.0, np.pi, walls=walls)
    rng = np.random.default_rng(1803)
    u, v, w = _random_velocity(g, rng)
    dt = 1e-3
    u1, v1, w1, _ = oracle.project(g, u, v, w, dt)
    umax = max(np.abs(u1).max(), np.abs(v1).max(), np.abs(w1).max())
    div = np.abs(oracle.divergence(g, u1, v1, w1)).max()
    assert div * min(g.dx, g.dy, g.dz) / umax <= 1e-12
    if walls:
        assert np.all(v1[:, -1, :] == 0.0)
    u2, v2, w2, _ = oracle.project(g, u1, v1, w1, dt)
    for a, b in ((u1, u2), (v1, v2), (w1, w2)):
        assert np.abs(a - b).max() <= 1e-13 * umax


@pytest.mark.parametrize("walls", [False, True])
def test_projection_removes_gradient_fields(walls):
    g = Grid(12, 10, 6, 1.0, 2.0, 1.5, walls=walls)
    phi = np.random.default_rng(9).standard_normal(g.shape)
    gx, gy, gz = oracle.gradient(g, phi)
    u, v, w, p = oracle.project(g, gx, gy, gz, dt=0.5)
    scale = max(np.abs(gx).max(), np.abs(gy).max())
    for a in (u, v, w):
        assert np.abs(a).max() <= 1e-12 * scale
    # and the pressure recovers phi (up to the constant) since u = u* - dt G p
    ref = (phi - phi.mean()) / 0.5
    assert np.abs(p - ref).max() <= 1e-11 * np.abs(ref).max()
