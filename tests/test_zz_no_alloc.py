"""evp_create_grid_static, the entry point that allocates nothing (its workspace is the library's
static device array), against evp_create_grid with a caller workspace: the same seeded inputs and
steps must give the same fields.  Two static grids in a row, the second smaller, so the second
reuses the array the first left behind (its state must be cleared on creation)."""
import ctypes

import numpy as np
import pytest

from paper_1803_09563_amd import inputs

from harness import gpu_state, to_dev

pytestmark = pytest.mark.gpu

# (nx, ny, nz, walls, precision, model); the second case is the smaller one
CASES = [(48, 40, 32, True, 0, inputs.SARAMITO), (32, 16, 24, False, 1, inputs.FENE_P)]


def _setup(G, wl_rheo, walls):
    G.set_rheology(**wl_rheo)
    G.set_forcing(inputs.FORCE_CONST_X, 0.3, 0.0)
    if walls:
        G.set_walls(0.1, -0.2, 0.05, 0.0)


def _run(static, nx, ny, nz, walls, precision, model, fields, steps=6):
    import paper_1803_09563_amd as evp
    L = 2 * np.pi
    G = evp.Grid(nx, ny, nz, L, 2.0 if walls else L * ny / nx, L * nz / nx, walls=walls,
                 precision=precision, static_workspace=static)
    rheo = dict(model=model, mu_s=0.01, mu_p=0.02, lam=0.5, tau_y=0.002 if model == inputs.SARAMITO else 0.0,
                L2=50.0)
    _setup(G, rheo, walls)
    G.write_fields(*to_dev(*fields))
    G.project()
    G.step(1e-3, steps)
    out = gpu_state(G, ("u", "v", "w", "p", "B", "hist"))
    h = G.health()
    G.close()
    return out, h


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    yield


def test_static_grid_matches_caller_workspace_twice():
    import paper_1803_09563_amd as evp
    for n, (nx, ny, nz, walls, prec, model) in enumerate(CASES):
        print(f"[no_alloc] case {n}: {nx}x{ny}x{nz} walls={walls} precision={prec}", flush=True)
        fields = inputs.random_state((nz, ny, nx), 100 + n, walls=walls)
        assert evp.workspace_bytes(nx, ny, nz, walls, prec) <= evp.STATIC_WORKSPACE_BYTES
        ref, href = _run(False, nx, ny, nz, walls, prec, model, fields)
        got, hgot = _run(True, nx, ny, nz, walls, prec, model, fields)
        for k in ref:
            scale = max(np.abs(ref[k]).max(), 1e-300)
            err = np.abs(got[k] - ref[k]).max() / scale
            # the same kernels on the same inputs: identical up to FP64 rounding (bitwise here)
            assert err <= 1e-12, (n, k, err)
            assert np.array_equal(got[k], ref[k]), (n, k, err)
        assert hgot["nonfinite"] == 0 and hgot["max_div"] == href["max_div"]


def test_static_grid_limits():
    import paper_1803_09563_amd as evp
    h = ctypes.c_void_p()
    # beyond the static workspace: a clear error, nothing created
    st = evp.lib.evp_create_grid_static(256, 128, 128, 1.0, 1.0, 1.0, 0, 0, None, ctypes.byref(h))
    assert st == -2 and b"static workspace" in evp.lib.evp_last_error() and not h.value
    # one static grid per device at a time
    G = evp.Grid(16, 16, 16, 1.0, 1.0, 1.0, static_workspace=True)
    st = evp.lib.evp_create_grid_static(16, 16, 16, 1.0, 1.0, 1.0, 0, 0, None, ctypes.byref(h))
    assert st == -3 and not h.value
    G.close()
    G2 = evp.Grid(16, 16, 16, 1.0, 1.0, 1.0, static_workspace=True)
    G2.close()
