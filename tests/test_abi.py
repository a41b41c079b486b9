"""The C-ABI library loads and exports every entry point include/evp.h declares; host-only paths
(workspace sizing, argument validation, error strings) behave as documented.  No GPU needed."""
import ctypes
import os
import re

import pytest

import paper_1803_09563_amd as evp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "evp.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(evp_[a-z_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    names = _declared()
    assert len(names) >= 18
    for n in names:
        assert hasattr(evp.lib, n), n
    assert set(names) == set(evp.symbols)


def test_workspace_bytes_valid_and_invalid_shapes():
    a = evp.workspace_bytes(32, 32, 32)
    b = evp.workspace_bytes(32, 32, 32, precision=evp.MIXED)
    c = evp.workspace_bytes(64, 48, 32, walls=True)
    assert a > 28 * 8 * 32 ** 3 and b < a and c > 0
    assert evp.workspace_bytes(30, 32, 32) > 0           # 30 = 2*3*5: radix-5 stage
    assert evp.workspace_bytes(40, 20, 480) > 0          # 5 2^a and 15 2^a
    assert evp.workspace_bytes(28, 32, 32) == 0          # 28 = 4*7: no radix 7
    assert evp.workspace_bytes(36, 32, 32) == 0          # 36 = 4*9: not in the size list
    assert evp.workspace_bytes(31, 32, 32) == 0          # odd nx
    assert evp.workspace_bytes(32, 28, 32) == 0          # periodic y needs an FFT size
    assert evp.workspace_bytes(32, 28, 32, walls=True) > 0
    assert evp.workspace_bytes(32, 3, 32, walls=True) == 0
    assert evp.workspace_bytes(32, 32, 32, precision=7) == 0


def test_workspace_covers_the_state():
    """FP64: 7 velocity/pressure fields, 21 stress/history planes, the half spectrum."""
    nx, ny, nz = 128, 128, 128
    n = nx * ny * nz
    need = 8 * n * (7 + 21) + 16 * (nx // 2 + 1) * ny * nz
    got = evp.workspace_bytes(nx, ny, nz)
    assert need <= got < need * 1.01


def test_guard_regions_follow_every_region():
    """Guard words after every workspace region (host-side layout query): each region ends on a
    256-byte boundary followed by at least 256 bytes of guard words, regions and guards alternate,
    and the last guard ends the workspace."""
    for shape, walls, prec in [((64, 48, 32), True, evp.FP64), ((32, 32, 32), False, evp.MIXED)]:
        regs = evp.guard_regions(*shape, walls=walls, precision=prec)
        assert len(regs) >= 20
        ends = [o + 8 * w for o, w in regs]
        assert all(w >= 32 for _, w in regs)
        assert all(e % 256 == 0 for e in ends)
        assert all(regs[i + 1][0] > ends[i] for i in range(len(regs) - 1))
        assert ends[-1] == evp.workspace_bytes(*shape, walls=walls, precision=prec)
    with pytest.raises(evp.EvpError):
        evp.guard_regions(28, 32, 32)


FFT_SIZES = {8, 10, 12, 16, 20, 24, 30, 32, 40, 48, 60, 64, 80, 96, 120, 128, 160, 192, 240, 256,
             320, 384, 480, 512}


def test_shape_rules_hold_for_arbitrary_arguments():
    """Property check of the host-side shape rules over arbitrary arguments: a workspace size (and
    guard regions ending exactly at it) exactly when nx, nz and periodic ny are FFT sizes, walls
    have 4 <= ny <= 1024, and the boundary type and precision are known; invalid arguments give 0
    or an error status, never a crash."""
    from hypothesis import given, settings, strategies as st

    dims = st.one_of(st.sampled_from(sorted(FFT_SIZES)), st.integers(-8, 1100))

    @settings(max_examples=400, deadline=None, derandomize=True)
    @given(nx=dims, ny=dims, nz=dims, bc=st.integers(-1, 2), prec=st.integers(-1, 2))
    def check(nx, ny, nz, bc, prec):
        ok = (bc in (0, 1) and prec in (0, 1) and nx in FFT_SIZES and nz in FFT_SIZES
              and (ny in FFT_SIZES if bc == 0 else 4 <= ny <= 1024))
        got = evp.lib.evp_workspace_bytes(nx, ny, nz, bc, prec)
        assert (got > 0) == ok, (nx, ny, nz, bc, prec, got)
        n = evp.lib.evp_guard_regions(nx, ny, nz, bc, prec, None, None, 0)
        assert (n > 0) == ok and (ok or n == -1)
        if ok:
            off = (ctypes.c_longlong * n)()
            words = (ctypes.c_longlong * n)()
            assert evp.lib.evp_guard_regions(nx, ny, nz, bc, prec, off, words, n) == n
            assert off[n - 1] + 8 * words[n - 1] == got

    check()


def test_error_strings_and_argument_errors():
    assert evp.lib.evp_error_string(0) == b"ok"
    assert evp.lib.evp_error_string(-2).startswith(b"workspace")
    h = ctypes.c_void_p()
    # invalid shape is rejected before any device call
    st = evp.lib.evp_create_grid(28, 32, 32, 1.0, 1.0, 1.0, 0, 0, ctypes.c_void_p(256), 1 << 30,
                                 None, ctypes.byref(h))
    assert st == -1 and b"nx=28" in evp.lib.evp_last_error()
    st = evp.lib.evp_create_grid(32, 32, 32, 1.0, 1.0, 1.0, 0, 0, None, 1 << 30, None,
                                 ctypes.byref(h))
    assert st == -2
    st = evp.lib.evp_create_grid(32, 32, 32, 1.0, 1.0, 1.0, 0, 0, ctypes.c_void_p(4096 + 8),
                                 1 << 30, None, ctypes.byref(h))
    assert st == -2 and b"aligned" in evp.lib.evp_last_error()
    st = evp.lib.evp_create_grid(32, 32, 32, 1.0, 1.0, 1.0, 0, 0, ctypes.c_void_p(4096), 1024,
                                 None, ctypes.byref(h))
    assert st == -2 and b"needs" in evp.lib.evp_last_error()
    st = evp.lib.evp_create_grid(32, 32, 32, -1.0, 1.0, 1.0, 0, 0, ctypes.c_void_p(4096),
                                 1 << 30, None, ctypes.byref(h))
    assert st == -1
    assert evp.lib.evp_step(None, 1e-3, 1, 0) == -1
    assert evp.lib.evp_destroy_grid(None) == 0
    arr = (ctypes.c_void_p * 1)(None)
    assert evp.lib.evp_step_batch(arr, 0, 1e-3, 1, 0) == -1          # empty batch
    assert evp.lib.evp_step_batch(arr, 1, 1e-3, 1, 0) == -1
    big = (ctypes.c_void_p * (evp.MAX_BATCH + 1))()
    assert evp.lib.evp_step_batch(big, evp.MAX_BATCH + 1, 1e-3, 1, 0) == -1   # above the maximum


def test_no_cpu_fallback_in_package():
    """The package path never imports the oracle or numpy-based solvers."""
    pkg = os.path.join(ROOT, "paper_1803_09563_amd")
    for fn in os.listdir(pkg):
        if fn.endswith(".py"):
            src = open(os.path.join(pkg, fn)).read()
            assert "import oracle" not in src and "from oracle" not in src, fn
