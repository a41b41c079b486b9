"""Pins of the oracle's constitutive part (Eq. (SRM2), Table 1, the |tau^d| norm of Sec. 2) in
homogeneous simple shear with the velocity frozen -- the paper's "uncoupled" test of Sec. 4.1.3.

Channel 4 x 8 x 4 with walls at y = -1, +1 moving at -gd and +gd and u = gd*y: every cell then
sees exactly L_xy = gd and no advection, so each cell integrates the same ODE with AB2.

Independent references: closed forms (Oldroyd-B start-up; Saramito below yield), the yield time
from the von Mises condition (with the value the paper prints, T ~ 1, from tests/golden), and the
steady states of the Saramito and FENE-P models, each the root of one scalar equation derived
from the steady constitutive law.
"""
import json
import os

import numpy as np
import pytest
from scipy.optimize import brentq

import oracle
from oracle import Grid, Rheology, Solver

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _shear_solver(rheo: Rheology, gd: float):
    g = Grid(4, 8, 4, 1.0, 2.0, 1.0, walls=True)
    s = Solver(g, rheo, walls_uv=(-gd, gd, 0.0, 0.0))
    u = np.broadcast_to((gd * g.yc())[None, :, None], g.shape).copy()
    B = np.zeros((6,) + g.shape)
    B[0] = B[3] = B[5] = 1.0
    s.write_fields(u, np.zeros(g.shape), np.zeros(g.shape), B)
    return s


def _uniform(s):
    """All cells carry the same B; return it (6,)."""
    B = s.B.reshape(6, -1)
    assert np.abs(B - B[:, :1]).max() <= 1e-13 * max(1.0, np.abs(B).max())
    return B[:, 0]


def _ob_closed_form(t, lam, gd):
    e = np.exp(-t / lam)
    bxy = lam * gd * (1 - e)
    bxx = 1 + 2 * lam ** 2 * gd ** 2 * (1 - e) - 2 * lam * gd ** 2 * t * e
    return bxx, bxy


def test_oldroyd_b_startup_second_order():
    lam, gd, T = 0.5, 1.3, 1.0
    errs = []
    for dt in (0.02, 0.01, 0.005):
        s = _shear_solver(Rheology(model=oracle.OLDROYD_B, mu_s=0.1, mu_p=0.4, lam=lam), gd)
        n = int(round(T / dt))
        s.step(dt, n, flags=Solver.FREEZE_VELOCITY)
        b = _uniform(s)
        bxx, bxy = _ob_closed_form(n * dt, lam, gd)
        assert abs(b[3] - 1) < 1e-13 and abs(b[5] - 1) < 1e-13     # yy, zz stay 1
        assert abs(b[2]) < 1e-13 and abs(b[4]) < 1e-13              # xz, yz stay 0
        errs.append(max(abs(b[0] - bxx), abs(b[1] - bxy)))
    assert errs[2] < 1e-3
    assert 3.5 < errs[0] / errs[1] < 4.5 and 3.5 < errs[1] / errs[2] < 4.5, errs


def test_saramito_below_yield_is_exact_elastic_solid():
    """F = 0 below yield: dB_xy/dt = gd, dB_xx/dt = 2 gd B_xy.  Euler-started AB2 then gives
    B_xy = gd t and B_xx = 1 + gd^2 (t^2 - dt^2) exactly (t = n dt, n >= 1)."""
    gd, dt = 1.0, 0.01
    s = _shear_solver(Rheology(model=oracle.SARAMITO, mu_s=1 / 9, mu_p=8 / 9, lam=1.0,
                               tau_y=1.0), gd)
    for n in range(1, 60):
        s.step(dt, 1, flags=Solver.FREEZE_VELOCITY)
        b = _uniform(s)
        t = n * dt
        assert abs(b[1] - gd * t) < 1e-13
        assert abs(b[0] - (1 + gd ** 2 * (t * t - dt * dt))) < 1e-13


def _yield_time_closed_form(G, gd, tau_y):
    """Below yield tau_xy = G gd t, tau_xx = G gd^2 t^2; |tau^d|^2 = G^2 gd^4 t^4/3 + G^2 gd^2 t^2."""
    c4, c2 = G ** 2 * gd ** 4 / 3.0, G ** 2 * gd ** 2
    t2 = (-c2 + np.sqrt(c2 ** 2 + 4 * c4 * tau_y ** 2)) / (2 * c4)
    return np.sqrt(t2)


def test_saramito_yield_time_matches_paper():
    gold = json.load(open(os.path.join(GOLDEN, "saramito_simple_shear.json")))
    Wi, Bi, beta = gold["Wi"], gold["Bi"], gold["beta"]
    # gd = 1, lambda = Wi, mu_0 = mu_s + mu_p = 1, tau_y = Bi * mu_0 * gd
    gd, lam, mu_s, mu_p, tau_y = 1.0, Wi, beta, 1 - beta, Bi
    G = mu_p / lam
    ty = _yield_time_closed_form(G, gd, tau_y)
    assert abs(ty - gold["printed_yield_time"]) < gold["tolerance_used"]
    dt = 1e-3
    s = _shear_solver(Rheology(model=oracle.SARAMITO, mu_s=mu_s, mu_p=mu_p, lam=lam,
                               tau_y=tau_y), gd)
    n_yield = None
    for n in range(1, 1200):
        s.step(dt, 1, flags=Solver.FREEZE_VELOCITY)
        F, _ = oracle.closure(s.g, s.r, s.B)
        if F.max() > 0.0:
            n_yield = n
            break
    assert n_yield is not None
    # the discrete state lags the continuum one by dt^2 in B_xx; yield within one step of t_y
    assert abs(n_yield * dt - ty) <= 1.5 * dt, (n_yield * dt, ty)


def _saramito_steady_F(G, Wi, tau_y):
    """Steady simple shear (B_yy = 1): B_xy = Wi/F, B_xx - 1 = 2 Wi^2/F^2, and
    F = 1 - tau_y/|tau^d| with |tau^d|^2 = G^2 ((B_xx-1)^2/3 + B_xy^2)."""
    def h(F):
        norm = G * np.sqrt((2 * Wi ** 2 / F ** 2) ** 2 / 3 + (Wi / F) ** 2)
        return F - (1 - tau_y / norm)
    return brentq(h, 1e-6, 1 - 1e-12, xtol=1e-15)


def test_saramito_steady_state_above_yield():
    gd, lam, mu_s, mu_p, tau_y = 1.0, 1.0, 1 / 9, 8 / 9, 1.0
    G, Wi = mu_p / lam, lam * gd
    F = _saramito_steady_F(G, Wi, tau_y)
    s = _shear_solver(Rheology(model=oracle.SARAMITO, mu_s=mu_s, mu_p=mu_p, lam=lam,
                               tau_y=tau_y), gd)
    s.step(0.01, 5000, flags=Solver.FREEZE_VELOCITY)
    b = _uniform(s)
    assert abs(b[1] - Wi / F) < 1e-9
    assert abs(b[0] - (1 + 2 * Wi ** 2 / F ** 2)) < 1e-9
    assert abs(b[3] - 1) < 1e-12 and abs(b[5] - 1) < 1e-12


def _fene_steady(L2, Wi):
    """Steady FENE-P simple shear: B_yy = B_zz = a/F, B_xy = Wi a/F^2, B_xx = a/F + 2 Wi^2 a/F^3
    with a = L2/(L2-3) and F = L2/(L2 - tr B)."""
    a = L2 / (L2 - 3)
    def h(F):
        tr = 3 * a / F + 2 * Wi ** 2 * a / F ** 3
        return F - L2 / (L2 - tr)
    F = brentq(h, 1.0 + 1e-12, 1e6, xtol=1e-15)
    return F, a


def test_fene_p_steady_state():
    gd, lam, L2 = 2.0, 1.0, 100.0
    Wi = lam * gd
    F, a = _fene_steady(L2, Wi)
    s = _shear_solver(Rheology(model=oracle.FENE_P, mu_s=0.1, mu_p=0.9, lam=lam, L2=L2), gd)
    s.step(0.005, 8000, flags=Solver.FREEZE_VELOCITY)
    b = _uniform(s)
    assert abs(b[3] - a / F) < 1e-9 and abs(b[5] - a / F) < 1e-9
    assert abs(b[1] - Wi * a / F ** 2) < 1e-9
    assert abs(b[0] - (a / F + 2 * Wi ** 2 * a / F ** 3)) < 1e-9
