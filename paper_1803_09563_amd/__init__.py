"""MI355X-native solver step for viscoelastic / elastoviscoplastic flow (Oldroyd-B, FENE-P,
Saramito) on a uniform staggered grid: the single-phase Eulerian path of Izbassarov et al.,
Sec. 3.2.2 (AB2 predictor + FFT/Thomas pressure projection), or the low-storage RK3 step of
Sec. 3.3.1.

This module is a thin ctypes binding of ``libevp.so`` (C-ABI in ``include/evp.h``).  It only
marshals arguments: PyTorch provides device memory and the stream; every step of the method runs
in the library's HIP kernels.  There is no CPU fallback: if the library is missing, importing this
package raises.
"""
from __future__ import annotations

import ctypes
import os

__all__ = ["Grid", "step_batch", "EvpError", "lib", "workspace_bytes", "symbols", "TwoPhaseParams",
           "OLDROYD_B", "FENE_P", "SARAMITO", "FP64", "MIXED", "PERIODIC", "WALLS",
           "FORCE_NONE", "FORCE_CONST_X", "FORCE_SIN_X_OF_Y", "FREEZE_VELOCITY",
           "STOP_AFTER_PREDICTOR", "MAX_BATCH", "KERNEL_NAMES", "AB2", "RK3", "NEO_HOOKEAN",
           "WENO5", "HOUC5", "STATIC_WORKSPACE_BYTES"]

_HERE = os.path.dirname(os.path.abspath(__file__))
# EVP_LIB selects another build of the same library (the host-sanitizer test loads one)
LIB_PATH = os.environ.get("EVP_LIB") or os.path.join(_HERE, "libevp.so")

PERIODIC, WALLS = 0, 1
FP64, MIXED = 0, 1
OLDROYD_B, FENE_P, SARAMITO, NEO_HOOKEAN = 0, 1, 2, 3
WENO5, HOUC5 = 0, 1
FORCE_NONE, FORCE_CONST_X, FORCE_SIN_X_OF_Y = 0, 1, 2
AB2, RK3 = 0, 1
FREEZE_VELOCITY, STOP_AFTER_PREDICTOR = 1, 2
READ_U, READ_V, READ_W, READ_P, READ_B, READ_HIST = 1, 2, 4, 8, 16, 32
MAX_BATCH = 32
STATIC_WORKSPACE_BYTES = 64 << 20
KERNEL_NAMES = ("predictor", "div_fftx", "fft_fwd", "solve", "fft_inv", "ifftx", "correct",
                "stress_div", "penalise", "level_set", "reinit", "curvature", "momentum2", "split")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python paper_1803_09563_amd/build.py` "
                      "(there is no CPU fallback)")

# PyTorch ships its own HIP runtime (soname libamdhip64.so.7).  Load it first so that libevp.so
# binds to the same runtime instance as the tensors and streams it is handed.
import torch as _torch_rt  # noqa: E402,F401

lib = ctypes.CDLL(LIB_PATH)

_vp = ctypes.c_void_p
_i = ctypes.c_int
_d = ctypes.c_double


class _Health(ctypes.Structure):
    _fields_ = [("nonfinite", ctypes.c_longlong), ("det_le0", ctypes.c_longlong),
                ("trace_ge95", ctypes.c_longlong), ("max_div", _d), ("energy", _d),
                ("guard_bad", ctypes.c_longlong)]


class TwoPhaseParams(ctypes.Structure):
    """evp_two_phase_t: fluid 1 (phi > 0) and fluid 2 (phi < 0) properties, surface tension and the
    reinitialisation schedule (Sec. 3.2)."""
    _fields_ = [("rho1", _d), ("rho2", _d), ("mu_s1", _d), ("mu_s2", _d), ("mu_p1", _d),
                ("mu_p2", _d), ("lam1", _d), ("lam2", _d), ("sigma", _d),
                ("reinit_every", _i), ("reinit_iters", _i)]


class _Profile(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_longlong * len(KERNEL_NAMES)), ("ms", _d * len(KERNEL_NAMES))]


symbols = {
    "evp_error_string": (ctypes.c_char_p, [_i]),
    "evp_last_error": (ctypes.c_char_p, []),
    "evp_workspace_bytes": (ctypes.c_size_t, [_i, _i, _i, _i, _i]),
    "evp_guard_regions": (_i, [_i, _i, _i, _i, _i, ctypes.POINTER(ctypes.c_longlong),
                               ctypes.POINTER(ctypes.c_longlong), _i]),
    "evp_create_grid": (_i, [_i, _i, _i, _d, _d, _d, _i, _i, _vp, ctypes.c_size_t, _vp,
                             ctypes.POINTER(_vp)]),
    "evp_create_grid_static": (_i, [_i, _i, _i, _d, _d, _d, _i, _i, _vp, ctypes.POINTER(_vp)]),
    "evp_set_stream": (_i, [_vp, _vp]),
    "evp_set_rheology": (_i, [_vp, _i, _d, _d, _d, _d, _d, _d]),
    "evp_set_forcing": (_i, [_vp, _i, _d, _d]),
    "evp_set_transport": (_i, [_vp, _i, _d]),
    "evp_set_solid": (_i, [_vp, _vp, _vp, _vp]),
    "evp_two_phase_bytes": (ctypes.c_size_t, [_i, _i, _i]),
    "evp_set_two_phase": (_i, [_vp, ctypes.POINTER(TwoPhaseParams), _vp, ctypes.c_size_t]),
    "evp_write_level_set": (_i, [_vp, _vp]),
    "evp_read_level_set": (_i, [_vp, _vp]),
    "evp_set_walls": (_i, [_vp, _d, _d, _d, _d]),
    "evp_write_fields": (_i, [_vp, _vp, _vp, _vp, _vp, _vp]),
    "evp_project": (_i, [_vp]),
    "evp_set_integrator": (_i, [_vp, _i]),
    "evp_step": (_i, [_vp, _d, _i, ctypes.c_uint]),
    "evp_step_batch": (_i, [ctypes.POINTER(_vp), _i, _d, _i, ctypes.c_uint]),
    "evp_read_fields": (_i, [_vp, ctypes.c_uint, _vp, _vp, _vp, _vp, _vp, _vp]),
    "evp_state_bytes": (ctypes.c_size_t, [_vp]),
    "evp_save_state": (_i, [_vp, _vp, ctypes.c_size_t]),
    "evp_load_state": (_i, [_vp, _vp, ctypes.c_size_t]),
    "evp_health": (_i, [_vp, ctypes.POINTER(_Health)]),
    "evp_health_enqueue": (_i, [_vp, _vp]),
    "evp_step_count": (_i, [_vp, ctypes.POINTER(ctypes.c_longlong)]),
    "evp_profile": (_i, [_vp, _i]),
    "evp_profile_read": (_i, [_vp, ctypes.POINTER(_Profile)]),
    "evp_destroy_grid": (_i, [_vp]),
}
for _name, (_res, _args) in symbols.items():
    _f = getattr(lib, _name)
    _f.restype = _res
    _f.argtypes = _args


class EvpError(RuntimeError):
    def __init__(self, status: int, where: str):
        msg = lib.evp_error_string(status).decode()
        detail = lib.evp_last_error().decode()
        super().__init__(f"{where}: {msg} ({status}){': ' + detail if detail else ''}")
        self.status = status


def _check(status: int, where: str):
    if status != 0:
        raise EvpError(status, where)


def workspace_bytes(nx, ny, nz, walls=False, precision=FP64) -> int:
    return int(lib.evp_workspace_bytes(nx, ny, nz, WALLS if walls else PERIODIC, precision))


def guard_regions(nx, ny, nz, walls=False, precision=FP64):
    """(byte offset, 8-byte words) of every guard region of this shape's workspace layout."""
    bc = WALLS if walls else PERIODIC
    n = lib.evp_guard_regions(nx, ny, nz, bc, precision, None, None, 0)
    _check(min(n, 0), "evp_guard_regions")
    off = (ctypes.c_longlong * n)()
    words = (ctypes.c_longlong * n)()
    _check(min(lib.evp_guard_regions(nx, ny, nz, bc, precision, off, words, n), 0), "evp_guard_regions")
    return list(zip(off, words))


def _torch():
    import torch
    return torch


def _dptr(t, shape, name):
    torch = _torch()
    if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous float64 CUDA tensor")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return ctypes.c_void_p(t.data_ptr())


class Grid:
    """One solve: nx x ny x nz cells in an lx x ly x lz box (walls=True: no-slip walls at
    y = -ly/2, +ly/2), FP64 or MIXED precision.  Device memory is one torch uint8 tensor; work is
    enqueued on ``stream`` (a torch.cuda.Stream; default: the current stream).
    static_workspace=True creates the grid with evp_create_grid_static instead: no device memory
    is allocated, the grid lives in the library's static workspace of the current device (one
    such grid per device at a time, at most STATIC_WORKSPACE_BYTES)."""

    def __init__(self, nx, ny, nz, lx, ly, lz, walls=False, precision=FP64, stream=None,
                 device="cuda", static_workspace=False):
        torch = _torch()
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self.lx, self.ly, self.lz = float(lx), float(ly), float(lz)
        self.walls = bool(walls)
        self.precision = precision
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        self.bytes = workspace_bytes(nx, ny, nz, walls, precision)
        if self.bytes == 0:
            raise ValueError(f"unsupported grid {nx}x{ny}x{nz} walls={walls}")
        h = ctypes.c_void_p()
        if static_workspace:
            self._ws = None
            _check(lib.evp_create_grid_static(self.nx, self.ny, self.nz, self.lx, self.ly,
                                              self.lz, WALLS if walls else PERIODIC, precision,
                                              ctypes.c_void_p(self.stream.cuda_stream),
                                              ctypes.byref(h)), "evp_create_grid_static")
            self._h = h
            self.device = self.stream.device
            return
        with torch.cuda.stream(self.stream):
            self._ws = torch.empty(self.bytes + 256, dtype=torch.uint8, device=device)
        base = self._ws.data_ptr()
        aligned = (base + 255) // 256 * 256
        _check(lib.evp_create_grid(self.nx, self.ny, self.nz, self.lx, self.ly, self.lz,
                                   WALLS if walls else PERIODIC, precision,
                                   ctypes.c_void_p(aligned), self.bytes,
                                   ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)),
               "evp_create_grid")
        self._h = h
        self.device = self._ws.device

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def handle(self):
        return self._h

    def set_stream(self, stream):
        _check(lib.evp_set_stream(self._h, ctypes.c_void_p(stream.cuda_stream)), "evp_set_stream")
        # the workspaces are used on the new stream from now on: tell the caching allocator, so
        # their memory is not handed to another allocation while work queued there still runs
        for buf in (self._ws, getattr(self, "_ws2", None)):
            if buf is not None:
                buf.record_stream(stream)
        self.stream = stream

    def set_rheology(self, model, rho=1.0, mu_s=0.0, mu_p=0.0, lam=1.0, tau_y=0.0, L2=1.0e4):
        _check(lib.evp_set_rheology(self._h, int(model), rho, mu_s, mu_p, lam, tau_y, L2),
               "evp_set_rheology")

    def set_transport(self, scheme=WENO5, kappa=0.0):
        """Stress advection scheme (WENO5 or HOUC5, Sec. 3) and artificial diffusion coefficient
        kappa (Sec. 3.1; 0 = off)."""
        _check(lib.evp_set_transport(self._h, int(scheme), float(kappa)), "evp_set_transport")

    def set_solid(self, alpha=None):
        """Fixed obstacle (Sec. 3.3.2): alpha = (alpha_u, alpha_v, alpha_w) solid volume fractions
        around the velocity points (float64 CUDA tensors of the grid's shape, kept referenced
        here while set), or None to remove it."""
        if alpha is None:
            _check(lib.evp_set_solid(self._h, None, None, None), "evp_set_solid")
            self._solid = None
            return
        s = self.shape
        ptrs = [_dptr(a, s, n) for a, n in zip(alpha, ("alpha_u", "alpha_v", "alpha_w"))]
        _check(lib.evp_set_solid(self._h, *ptrs), "evp_set_solid")
        self._solid = tuple(alpha)

    def set_two_phase(self, params=None, **kw):
        """Two-phase (bubbly-flow) path of Sec. 3.2 with TwoPhaseParams (or its fields as
        keywords: rho1, rho2, mu_s1, mu_s2, mu_p1, mu_p2, lam1, lam2, sigma, reinit_every,
        reinit_iters); None switches back to a single phase.  The level-set workspace is a
        torch uint8 tensor held here."""
        torch = _torch()
        if params is None and not kw:
            _check(lib.evp_set_two_phase(self._h, None, None, 0), "evp_set_two_phase")
            self._ws2 = None
            return
        if params is None:
            d = dict(rho1=1.0, rho2=1.0, mu_s1=0.0, mu_s2=0.0, mu_p1=0.0, mu_p2=0.0, lam1=1.0,
                     lam2=1.0, sigma=0.0, reinit_every=10, reinit_iters=2)
            d.update(kw)
            params = TwoPhaseParams(**d)
        n = int(lib.evp_two_phase_bytes(self.nx, self.ny, self.nz))
        with torch.cuda.stream(self.stream):
            buf = torch.empty(n + 256, dtype=torch.uint8, device=self.device)
        off = (-buf.data_ptr()) % 256
        _check(lib.evp_set_two_phase(self._h, ctypes.byref(params),
                                     ctypes.c_void_p(buf.data_ptr() + off), n), "evp_set_two_phase")
        self._ws2 = buf

    def write_level_set(self, phi):
        self._keep_phi = phi
        _check(lib.evp_write_level_set(self._h, _dptr(phi, self.shape, "phi")), "evp_write_level_set")

    def read_level_set(self):
        torch = _torch()
        with torch.cuda.stream(self.stream):
            out = torch.empty(self.shape, dtype=torch.float64, device=self.device)
        _check(lib.evp_read_level_set(self._h, ctypes.c_void_p(out.data_ptr())), "evp_read_level_set")
        return out

    def set_forcing(self, kind, amp=0.0, ky=0.0):
        _check(lib.evp_set_forcing(self._h, int(kind), amp, ky), "evp_set_forcing")

    def set_walls(self, u_bot=0.0, u_top=0.0, w_bot=0.0, w_top=0.0):
        _check(lib.evp_set_walls(self._h, u_bot, u_top, w_bot, w_top), "evp_set_walls")

    def set_integrator(self, scheme):
        """AB2 (Sec. 3.2.2, default) or RK3 (Sec. 3.3.1) for later steps; also "ab2" / "rk3"."""
        if isinstance(scheme, str):
            scheme = {"ab2": AB2, "rk3": RK3}[scheme.lower()]
        _check(lib.evp_set_integrator(self._h, int(scheme)), "evp_set_integrator")

    def write_fields(self, u, v, w, B, hist=None):
        s = self.shape
        args = [_dptr(u, s, "u"), _dptr(v, s, "v"), _dptr(w, s, "w"), _dptr(B, (6,) + s, "B"),
                _dptr(hist, (9,) + s, "hist") if hist is not None else None]
        self._keep = (u, v, w, B, hist)
        _check(lib.evp_write_fields(self._h, *args), "evp_write_fields")

    def project(self):
        _check(lib.evp_project(self._h), "evp_project")

    def step(self, dt, nsteps=1, flags=0):
        _check(lib.evp_step(self._h, float(dt), int(nsteps), int(flags)), "evp_step")

    def read_fields(self, which=("u", "v", "w", "p", "B")):
        torch = _torch()
        s = self.shape
        out = {}
        mask = 0
        bits = {"u": READ_U, "v": READ_V, "w": READ_W, "p": READ_P, "B": READ_B, "hist": READ_HIST}
        with torch.cuda.stream(self.stream):
            for k in which:
                shp = (6,) + s if k == "B" else (9,) + s if k == "hist" else s
                out[k] = torch.empty(shp, dtype=torch.float64, device=self.device)
                mask |= bits[k]
        ptr = lambda k: ctypes.c_void_p(out[k].data_ptr()) if k in out else None
        _check(lib.evp_read_fields(self._h, mask, ptr("u"), ptr("v"), ptr("w"), ptr("p"),
                                   ptr("B"), ptr("hist")), "evp_read_fields")
        return out

    def save_state(self):
        """Bitwise checkpoint of the state in a device uint8 tensor."""
        torch = _torch()
        n = int(lib.evp_state_bytes(self._h))
        with torch.cuda.stream(self.stream):
            buf = torch.empty(n + 256, dtype=torch.uint8, device=self.device)
        off = (-buf.data_ptr()) % 256
        view = buf[off:off + n]
        _check(lib.evp_save_state(self._h, ctypes.c_void_p(view.data_ptr()), n), "evp_save_state")
        return view

    def load_state(self, state):
        _check(lib.evp_load_state(self._h, ctypes.c_void_p(state.data_ptr()), state.numel()),
               "evp_load_state")

    def health(self):
        h = _Health()
        _check(lib.evp_health(self._h, ctypes.byref(h)), "evp_health")
        return {"nonfinite": h.nonfinite, "det_le0": h.det_le0, "trace_ge95": h.trace_ge95,
                "max_div": h.max_div, "energy": h.energy, "guard_bad": h.guard_bad}

    def health_enqueue(self, out5):
        """Enqueue the diagnostics on the grid's stream into out5, a float64 CUDA tensor of 5
        values, valid once the stream has passed this point; read it with health_values()."""
        torch = _torch()
        if not (out5.is_cuda and out5.dtype == torch.float64 and out5.is_contiguous()
                and out5.numel() >= 5):
            raise ValueError("out5 must be a contiguous float64 CUDA tensor of 5 values")
        _check(lib.evp_health_enqueue(self._h, ctypes.c_void_p(out5.data_ptr())),
               "evp_health_enqueue")

    @staticmethod
    def health_values(out5):
        v = [float(x) for x in out5[:5].cpu()]
        return {"nonfinite": int(v[0]), "det_le0": int(v[1]), "trace_ge95": int(v[2]),
                "max_div": v[3], "energy": v[4]}

    def step_count(self):
        n = ctypes.c_longlong()
        _check(lib.evp_step_count(self._h, ctypes.byref(n)), "evp_step_count")
        return n.value

    def profile(self, enable=True):
        _check(lib.evp_profile(self._h, 1 if enable else 0), "evp_profile")

    def profile_read(self):
        p = _Profile()
        _check(lib.evp_profile_read(self._h, ctypes.byref(p)), "evp_profile_read")
        return {name: {"launches": p.launches[k], "ms": p.ms[k]}
                for k, name in enumerate(KERNEL_NAMES)}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib.evp_destroy_grid(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def step_batch(grids, dt, nsteps=1, flags=0):
    """One launch per kernel for all grids (same shape, boundary type, precision and stream)."""
    arr = (ctypes.c_void_p * len(grids))(*[g.handle.value for g in grids])
    _check(lib.evp_step_batch(arr, len(grids), float(dt), int(nsteps), int(flags)),
           "evp_step_batch")
