"""ORACLE -- test infrastructure only.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may import
this package.  It shares no code with the HIP path (``paper_1803_09563_amd``) and never imports it.

A plain, slow FP64 CPU implementation of one time step of the paper's single-phase Eulerian
solver (Izbassarov et al., Sec. 3.2.2 "Time integration: Adams-Bashforth scheme", and the
Runge-Kutta alternative of Sec. 3.3.1, ``Solver.step_rk3``):

* predictor -- Eqs. (ab2tau), (ab2), (rt), (ru) with the closures of Table 1 -- in plain C loops
  (``evp_oracle.c``), loaded through ctypes;
* projection -- Eqs. (var poisson) and (projection) with rho constant -- written here from its plain
  definition: p is the zero-mean solution of L_h p = rho * D_h u* / dt, where D_h is the
  cell-centred divergence of face values and L_h = D_h G_h the 7-point Laplacian (G_h the face
  gradient, zero on wall faces); u^{n+1} = u* - (dt/rho) G_h p.  Periodic directions use the
  discrete Fourier transform (numpy.fft as the library primitive); the wall-normal direction of a
  channel is a tridiagonal solve (Thomas algorithm written out below).

Fields are numpy arrays of shape (nz, ny, nx), x fastest; u[k, j, i] is on the +x face of cell
(i, j, k), v on its +y face, w on its +z face; B has shape (6, nz, ny, nx), order xx xy xz yy yz zz.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# EVP_ORACLE_LIB selects another build of evp_oracle.c (the sanitizer test loads the ASan/UBSan
# build made by build_sanitized in a child process)
_LIB_PATH = os.environ.get("EVP_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")

OLDROYD_B, FENE_P, SARAMITO, NEO_HOOKEAN = 0, 1, 2, 3
WENO5, HOUC5 = 0, 1
FORCE_NONE, FORCE_CONST_X, FORCE_SIN_X_OF_Y = 0, 1, 2


def build(verbose: bool = False) -> str:
    """Compile ``evp_oracle.c`` with gcc (plain -O2, OpenMP, no fast-math)."""
    import subprocess
    src = os.path.join(_HERE, "evp_oracle.c")
    tmp = _LIB_PATH + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-fno-fast-math",
           "-ffp-contract=off", src, "-o", tmp, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def build_sanitized(out: str) -> str:
    """Compile ``evp_oracle.c`` with AddressSanitizer and UndefinedBehaviorSanitizer (every
    finding fatal) into ``out``; a process loads it through EVP_ORACLE_LIB with gcc's libasan
    preloaded."""
    import subprocess
    src = os.path.join(_HERE, "evp_oracle.c")
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-fno-fast-math",
           "-ffp-contract=off", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", src, "-o", out, "-lm"]
    subprocess.run(cmd, check=True)
    return out


class _Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
        ("walls", ctypes.c_int),
        ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("dz", ctypes.c_double),
        ("y0", ctypes.c_double),
        ("model", ctypes.c_int),
        ("rho", ctypes.c_double), ("mu_s", ctypes.c_double), ("mu_p", ctypes.c_double),
        ("lam", ctypes.c_double), ("tau_y", ctypes.c_double), ("L2", ctypes.c_double),
        ("force_kind", ctypes.c_int),
        ("force_amp", ctypes.c_double), ("force_ky", ctypes.c_double),
        ("u_bot", ctypes.c_double), ("u_top", ctypes.c_double),
        ("w_bot", ctypes.c_double), ("w_top", ctypes.c_double),
        ("adv_scheme", ctypes.c_int), ("kappa", ctypes.c_double),
        ("lam_c", ctypes.c_void_p), ("mup_c", ctypes.c_void_p), ("mus_c", ctypes.c_void_p),
        ("rho_c", ctypes.c_void_p), ("fs", ctypes.c_void_p),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        pp = ctypes.POINTER(_Params)
        lib.oracle_predictor.argtypes = [pp, dp, dp, dp, dp, dp, dp, ctypes.c_int, ctypes.c_int,
                                         ctypes.c_double, dp, dp, dp, dp, dp, dp]
        lib.oracle_predictor.restype = None
        lib.oracle_weno5_line.argtypes = [dp, ctypes.c_int, ctypes.c_double, ctypes.c_double, dp]
        lib.oracle_weno5_line.restype = None
        lib.oracle_upwind_line.argtypes = [dp, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                           ctypes.c_int, dp]
        lib.oracle_upwind_line.restype = None
        lib.oracle_stress.argtypes = [pp, dp, dp]
        lib.oracle_stress.restype = None
        lib.oracle_closure.argtypes = [pp, dp, dp, dp]
        lib.oracle_closure.restype = None
        lib.oracle_terms.argtypes = [pp, dp, dp, dp, dp, dp, dp, dp, dp]
        lib.oracle_terms.restype = None
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


@dataclass
class Grid:
    """Uniform staggered grid.  walls=True puts no-slip walls at y = -ly/2 and y = +ly/2."""
    nx: int
    ny: int
    nz: int
    lx: float
    ly: float
    lz: float
    walls: bool = False

    @property
    def dx(self): return self.lx / self.nx

    @property
    def dy(self): return self.ly / self.ny

    @property
    def dz(self): return self.lz / self.nz

    @property
    def y0(self): return -0.5 * self.ly if self.walls else 0.0

    @property
    def shape(self): return (self.nz, self.ny, self.nx)

    def yc(self):
        """y of cell centres (and of u, w faces)."""
        return self.y0 + (np.arange(self.ny) + 0.5) * self.dy


@dataclass
class Rheology:
    """Coefficients of Eq. (NS) and Table 1 (rho, mu_s, mu_p, lambda, tau_y, L^2), the stress
    advection scheme (WENO5 or HOUC5, Sec. 3) and the artificial diffusion coefficient kappa of
    Sec. 3.1 (0: off).  Neo-Hookean: G = mu_p / lambda."""
    model: int = OLDROYD_B
    rho: float = 1.0
    mu_s: float = 0.0
    mu_p: float = 0.0
    lam: float = 1.0
    tau_y: float = 0.0
    L2: float = 1.0e4
    adv: int = WENO5
    kappa: float = 0.0


def _params(g: Grid, r: Rheology, forcing=(FORCE_NONE, 0.0, 0.0), walls_uv=(0.0, 0.0, 0.0, 0.0)):
    return _Params(g.nx, g.ny, g.nz, int(g.walls), g.dx, g.dy, g.dz, g.y0, r.model, r.rho, r.mu_s,
                   r.mu_p, r.lam, r.tau_y, r.L2, int(forcing[0]), float(forcing[1]),
                   float(forcing[2]), *map(float, walls_uv), int(r.adv), float(r.kappa))


def upwind_line(f: np.ndarray, h: float, vel: float, scheme: int = WENO5) -> np.ndarray:
    """Periodic upwind derivative of a 1D array with the oracle's WENO5 or HOUC5 stencil."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = np.empty_like(f)
    _load().oracle_upwind_line(_ptr(f), f.size, float(h), float(vel), int(scheme), _ptr(out))
    return out


def weno5_line(f: np.ndarray, h: float, vel: float) -> np.ndarray:
    """Periodic upwind WENO5 derivative of a 1D array (the oracle's own scheme)."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = np.empty_like(f)
    _load().oracle_weno5_line(_ptr(f), f.size, float(h), float(vel), _ptr(out))
    return out


def stress(g: Grid, r: Rheology, B: np.ndarray) -> np.ndarray:
    """Extra stress tau from B (Table 1 inverted), shape (6, nz, ny, nx)."""
    B = np.ascontiguousarray(B, dtype=np.float64)
    out = np.empty_like(B)
    p = _params(g, r)
    _load().oracle_stress(ctypes.byref(p), _ptr(B), _ptr(out))
    return out


def closure(g: Grid, r: Rheology, B: np.ndarray):
    """(F, a) of Table 1 on every cell."""
    B = np.ascontiguousarray(B, dtype=np.float64)
    F = np.empty(g.shape)
    a = np.empty(g.shape)
    p = _params(g, r)
    _load().oracle_closure(ctypes.byref(p), _ptr(B), _ptr(F), _ptr(a))
    return F, a


# ----------------------------------------------------------------------------------------------
# Projection: Eqs. (var poisson) and (projection) with constant rho.
# ----------------------------------------------------------------------------------------------

def divergence(g: Grid, u, v, w):
    """D_h u: cell-centred divergence of face velocities (wall faces carry v = 0)."""
    d = (u - np.roll(u, 1, axis=2)) / g.dx + (w - np.roll(w, 1, axis=0)) / g.dz
    if g.walls:
        vb = np.concatenate([np.zeros_like(v[:, :1, :]), v[:, :-1, :]], axis=1)
        d += (v - vb) / g.dy
    else:
        d += (v - np.roll(v, 1, axis=1)) / g.dy
    return d


def gradient(g: Grid, p):
    """G_h p on faces; the y-gradient on wall faces is zero (no-penetration)."""
    gx = (np.roll(p, -1, axis=2) - p) / g.dx
    gz = (np.roll(p, -1, axis=0) - p) / g.dz
    if g.walls:
        gy = np.zeros_like(p)
        gy[:, :-1, :] = (p[:, 1:, :] - p[:, :-1, :]) / g.dy
    else:
        gy = (np.roll(p, -1, axis=1) - p) / g.dy
    return gx, gy, gz


def _eig(n, h):
    """Eigenvalues of the periodic second difference: -(4/h^2) sin^2(pi k / n)."""
    k = np.arange(n)
    return -(4.0 / h ** 2) * np.sin(np.pi * k / n) ** 2


def thomas(a, b, c, d):
    """Thomas algorithm for tridiagonal systems a_j x_{j-1} + b_j x_j + c_j x_{j+1} = d_j,
    j = 0..n-1 (a_0, c_{n-1} unused).  Arrays have the system index first; further axes are
    independent systems (broadcast)."""
    n = d.shape[0]
    cp = np.empty(np.broadcast(b, d).shape, dtype=np.result_type(b, c))
    dp = np.empty(np.broadcast(b, d).shape, dtype=np.result_type(b, d))
    cp[0] = c[0] / b[0]
    dp[0] = d[0] / b[0]
    for j in range(1, n):
        den = b[j] - a[j] * cp[j - 1]
        cp[j] = c[j] / den if j < n - 1 else 0.0
        dp[j] = (d[j] - a[j] * dp[j - 1]) / den
    x = np.empty_like(dp)
    x[n - 1] = dp[n - 1]
    for j in range(n - 2, -1, -1):
        x[j] = dp[j] - cp[j] * x[j + 1]
    return x


def solve_poisson(g: Grid, r):
    """Zero-mean p with L_h p = r (r must have zero sum for solvability)."""
    lx = _eig(g.nx, g.dx)[None, None, :]
    lz = _eig(g.nz, g.dz)[:, None, None]
    if not g.walls:
        ly = _eig(g.ny, g.dy)[None, :, None]
        rh = np.fft.fftn(r)
        den = lx + ly + lz
        den[0, 0, 0] = 1.0
        ph = rh / den
        ph[0, 0, 0] = 0.0
        return np.real(np.fft.ifftn(ph))
    # walls: DFT in x and z, tridiagonal (Neumann rows at both walls) in y for every (kz, kx)
    rh = np.fft.fft2(r, axes=(0, 2))                    # (nz, ny, nx) complex
    ny, h2 = g.ny, g.dy ** 2
    mu = (lx + lz)[:, 0, :]                               # (nz, nx)
    d = np.moveaxis(rh, 1, 0)                             # (ny, nz, nx)
    a = np.full(ny, 1.0 / h2)
    c = np.full(ny, 1.0 / h2)
    bdiag = np.full(ny, -2.0 / h2)
    bdiag[0] += 1.0 / h2
    bdiag[-1] += 1.0 / h2
    b = bdiag[:, None, None] + mu[None, :, :]
    ph = np.empty_like(d)
    # every mode but (0, 0) is non-singular
    mask = np.ones(mu.shape, dtype=bool)
    mask[0, 0] = False
    ph[:, mask] = thomas(a[:, None], b[:, mask], c[:, None], d[:, mask])
    # mode (0, 0): rows sum to zero; fix p_{ny-1} = 0 and solve the leading (ny-1) block
    ph[:, 0, 0] = 0.0
    if ny > 1:
        ph[:-1, 0, 0] = thomas(a[:-1], b[:-1, 0, 0], c[:-1], d[:-1, 0, 0])
    p = np.real(np.fft.ifft2(np.moveaxis(ph, 0, 1), axes=(0, 2)))
    return p - p.mean()


def project(g: Grid, us, vs, ws, dt: float, rho: float = 1.0):
    """Chorin projection, Eqs. (var poisson) and (projection): returns (u, v, w, p)."""
    r = rho * divergence(g, us, vs, ws) / dt
    p = solve_poisson(g, r)
    gx, gy, gz = gradient(g, p)
    u = us - (dt / rho) * gx
    v = vs - (dt / rho) * gy
    w = ws - (dt / rho) * gz
    if g.walls:
        v[:, -1, :] = 0.0
    return u, v, w, p


# ----------------------------------------------------------------------------------------------
# Terms of the Runge-Kutta integrator (Sec. 3.3.1)
# ----------------------------------------------------------------------------------------------

# Eq. (eq:RK): alpha, zeta, xi of the three substeps
RK3_ALPHA = (4.0 / 15.0, 1.0 / 15.0, 1.0 / 6.0)
RK3_ZETA = (8.0 / 15.0, 5.0 / 12.0, 3.0 / 4.0)
RK3_XI = (0.0, -17.0 / 60.0, -5.0 / 12.0)


def terms(g: Grid, r: Rheology, u, v, w, B, forcing=(FORCE_NONE, 0.0, 0.0),
          walls_uv=(0.0, 0.0, 0.0, 0.0)):
    """At one state: RT (bracket of Eq. RK-rt, 6 planes), and on the faces A = div(uu),
    V = mu_s lap u, T = div(tau) (3 planes each)."""
    shp = g.shape
    RT = np.empty((6,) + shp); A = np.empty((3,) + shp)
    V = np.empty((3,) + shp); T = np.empty((3,) + shp)
    p = _params(g, r, forcing, walls_uv)
    arrs = [np.ascontiguousarray(x, dtype=np.float64) for x in (u, v, w, B)]
    _load().oracle_terms(ctypes.byref(p), *[_ptr(x) for x in arrs], _ptr(RT), _ptr(A), _ptr(V),
                         _ptr(T))
    return RT, A, V, T


def body_force(g: Grid, forcing):
    """f on the faces (3 planes): f_x = amp or amp sin(ky y) on the x-faces, zero elsewhere."""
    f = np.zeros((3,) + g.shape)
    kind, amp, ky = forcing
    if kind == FORCE_CONST_X:
        f[0] = amp
    elif kind == FORCE_SIN_X_OF_Y:
        f[0] = (amp * np.sin(ky * g.yc()))[None, :, None]
    return f


# ----------------------------------------------------------------------------------------------
# The whole step
# ----------------------------------------------------------------------------------------------

class Solver:
    """State (u, v, w, B, p, AB2 history) plus the step of Sec. 3.2.2."""

    FREEZE_VELOCITY = 1
    STOP_AFTER_PREDICTOR = 2

    def __init__(self, grid: Grid, rheology: Rheology, forcing=(FORCE_NONE, 0.0, 0.0),
                 walls_uv=(0.0, 0.0, 0.0, 0.0)):
        self.g = grid
        self.r = rheology
        self.forcing = forcing
        self.walls_uv = walls_uv
        shp = grid.shape
        self.u = np.zeros(shp); self.v = np.zeros(shp); self.w = np.zeros(shp)
        self.B = np.zeros((6,) + shp)
        self.B[0] = self.B[3] = self.B[5] = 1.0
        self.p = np.zeros(shp)
        self.RT = np.zeros((6,) + shp)
        self.RU = np.zeros((3,) + shp)
        self.have_hist = False
        self.nstep = 0
        self.alpha = None

    def _p(self):
        return _params(self.g, self.r, self.forcing, self.walls_uv)

    def write_fields(self, u, v, w, B, hist=None):
        self.u = np.array(u, dtype=np.float64, copy=True)
        self.v = np.array(v, dtype=np.float64, copy=True)
        self.w = np.array(w, dtype=np.float64, copy=True)
        self.B = np.array(B, dtype=np.float64, copy=True)
        if self.g.walls:
            self.v[:, -1, :] = 0.0
        if hist is None:
            self.RT[:] = 0.0
            self.RU[:] = 0.0
            self.have_hist = False
        else:
            self.RT = np.array(hist[:6], dtype=np.float64, copy=True)
            self.RU = np.array(hist[6:9], dtype=np.float64, copy=True)
            self.have_hist = True

    def set_solid(self, alpha=None):
        """Solid volume fractions (alpha_u, alpha_v, alpha_w) around the u-, v- and w-points of
        the volume-penalisation immersed boundary method, Sec. 3.3.2, Eqs. (Vol) and
        (forceAdded), for non-moving solids (u_s = 0).  None removes the solid."""
        self.alpha = None if alpha is None else [np.array(a, dtype=np.float64, copy=True)
                                                 for a in alpha]

    def _penalise(self, dt, us, vs, ws):
        """Eq. (Vol) with u_s = 0: f = rho alpha (u_s - u*) / dt, u** = u* + dt f / rho."""
        if self.alpha is None:
            return us, vs, ws
        rho = self.r.rho
        out = []
        for a, x in zip(self.alpha, (us, vs, ws)):
            f = rho * a * (0.0 - x) / dt
            out.append(x + dt * f / rho)
        return out

    def project(self, dt: float = 1.0):
        """Make u discretely solenoidal (used once on initial data)."""
        self.u, self.v, self.w, _ = project(self.g, self.u, self.v, self.w, dt, self.r.rho)

    def predictor(self, dt: float, flags: int = 0):
        shp = self.g.shape
        Bn = np.empty((6,) + shp); RT = np.empty((6,) + shp); RU = np.empty((3,) + shp)
        us = np.empty(shp); vs = np.empty(shp); ws = np.empty(shp)
        p = self._p()
        u = np.ascontiguousarray(self.u); v = np.ascontiguousarray(self.v)
        w = np.ascontiguousarray(self.w); B = np.ascontiguousarray(self.B)
        _load().oracle_predictor(ctypes.byref(p), _ptr(u), _ptr(v), _ptr(w), _ptr(B),
                                 _ptr(self.RT), _ptr(self.RU), int(not self.have_hist),
                                 int(bool(flags & self.FREEZE_VELOCITY)), float(dt),
                                 _ptr(Bn), _ptr(RT), _ptr(us), _ptr(vs), _ptr(ws), _ptr(RU))
        return Bn, RT, us, vs, ws, RU

    def step(self, dt: float, nsteps: int = 1, flags: int = 0):
        for _ in range(nsteps):
            Bn, RT, us, vs, ws, RU = self.predictor(dt, flags)
            self.B, self.RT, self.RU = Bn, RT, RU
            self.have_hist = True
            self.nstep += 1
            if not flags & self.FREEZE_VELOCITY:
                us, vs, ws = self._penalise(dt, us, vs, ws)
            if flags & self.STOP_AFTER_PREDICTOR:
                self.u, self.v, self.w = us, vs, ws
                continue
            if flags & self.FREEZE_VELOCITY:
                continue
            self.u, self.v, self.w, self.p = project(self.g, us, vs, ws, dt, self.r.rho)

    def step_rk3(self, dt: float, nsteps: int = 1, flags: int = 0):
        """Low-storage three-substep Runge-Kutta step of Sec. 3.3.1.  Per substep k:
        B^k = B^{k-1} + dt (zeta RT^{k-1} + xi RT^{k-2})                         (Eqs. RK-rt, rk3tau)
        u*  = u^{k-1} + dt [-zeta A^{k-1} - xi A^{k-2} - 2 alpha grad p^{k-1} / rho
                            + (2 alpha V^{k-1} + alpha (T^k + T^{k-1}) + 2 alpha f) / rho]
                                                                              (Eqs. NS-num1, rk3)
        L psi = rho div(u*) / (2 alpha dt);  p^k = p^{k-1} + psi;
        u^k = u* - 2 alpha dt grad(psi) / rho                                  (Eqs. NS-num2, NS-num3)
        The viscous term is taken explicitly at k-1 with weight 2 alpha (the paper's superscript k
        on it would need an implicit solve it does not describe); the stress divergence uses
        B^k, known from the stress update of the same substep.  With a solid (``set_solid``) the
        penalisation of Eq. (Vol) acts on the prediction from the momentum terms, before the old
        pressure gradient -2 alpha dt grad p^{k-1} / rho is added."""
        g, rh = self.g, self.r
        rho = rh.rho
        f = body_force(g, self.forcing)
        for _ in range(nsteps):
            RT2 = A2 = None
            for kk in range(3):
                al, ze, xi = RK3_ALPHA[kk], RK3_ZETA[kk], RK3_XI[kk]
                RT1, A1, V1, T1 = terms(g, rh, self.u, self.v, self.w, self.B, self.forcing,
                                        self.walls_uv)
                Bk = self.B + dt * (ze * RT1 + (xi * RT2 if RT2 is not None else 0.0))
                if flags & self.FREEZE_VELOCITY:
                    self.B = Bk
                    RT2 = RT1
                    continue
                _, _, _, Tk = terms(g, rh, self.u, self.v, self.w, Bk, self.forcing, self.walls_uv)
                gx, gy, gz = gradient(g, self.p)
                G = np.stack([gx, gy, gz])
                # RU of Eq. (NS-num1) in two parts: the momentum terms RM and the old pressure
                # gradient; u* = (u + dt RM) - dt 2 alpha grad p^{k-1} / rho, the solid
                # penalisation (if any) acting on the first part
                RM = -ze * A1 - (xi * A2 if A2 is not None else 0.0) \
                    + (2 * al * V1 + al * (Tk + T1) + 2 * al * f) / rho
                us, vs, ws = self._penalise(dt, self.u + dt * RM[0], self.v + dt * RM[1],
                                            self.w + dt * RM[2])
                us = us - dt * (2 * al * G[0] / rho)
                vs = vs - dt * (2 * al * G[1] / rho)
                ws = ws - dt * (2 * al * G[2] / rho)
                if g.walls:
                    vs[:, -1, :] = 0.0
                dte = 2 * al * dt
                u, v, w, psi = project(g, us, vs, ws, dte, rho)
                self.u, self.v, self.w = u, v, w
                self.p = self.p + psi
                self.B = Bk
                RT2, A2 = RT1, A1
            self.have_hist = False       # no AB2 history: a later AB2 step starts with Euler
            self.nstep += 1

    def stress(self):
        return stress(self.g, self.r, self.B)

    def health(self):
        """Counts the paper's trigger conditions for local artificial diffusion (Sec. 3.1:
        det B < 0, tr B >= 0.95 L^2) plus non-finite cells, max |D_h u| and kinetic energy."""
        B = self.B
        bxx, bxy, bxz, byy, byz, bzz = B
        det = (bxx * (byy * bzz - byz * byz) - bxy * (bxy * bzz - byz * bxz)
               + bxz * (bxy * byz - byy * bxz))
        tr = bxx + byy + bzz
        finite = np.isfinite(B).all(axis=0) & np.isfinite(self.u) & np.isfinite(self.v) \
            & np.isfinite(self.w)
        n95 = int(np.sum(tr >= 0.95 * self.r.L2)) if self.r.model == FENE_P else 0
        vol = self.g.dx * self.g.dy * self.g.dz
        return {
            "nonfinite": int(np.sum(~finite)),
            "det_le0": int(np.sum(det <= 0.0)),
            "trace_ge95": n95,
            "max_div": float(np.max(np.abs(divergence(self.g, self.u, self.v, self.w)))),
            "energy": float(0.5 * vol * np.sum(self.u ** 2 + self.v ** 2 + self.w ** 2)),
        }
