"""Workspace guard words, a check for out-of-bounds writes (not part of the method): every region
of a grid's workspace is followed by words holding a fixed pattern.  A fresh grid and every step
path leave them intact; words overwritten from the host are counted by evp_health."""
import numpy as np
import pytest

from paper_1803_09563_amd import inputs

from harness import gpu_grid, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1803_09563_amd  # noqa: F401  (fails loudly without libevp.so)
    yield


def _workload(nx, ny, nz, walls):
    L = 2 * np.pi
    return inputs.Workload(f"g{nx}x{ny}x{nz}", nx, ny, nz, L, 2.0 if walls else L * ny / nx, L * nz / nx,
                           walls, inputs.SARAMITO, 0.01, 0.02, 0.5, tau_y=0.002)


@pytest.mark.parametrize("walls", [False, True])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("integrator", ["ab2", "rk3"])
def test_steps_leave_guards_intact(walls, precision, integrator):
    import paper_1803_09563_amd as evp
    prec = evp.FP64 if precision == "fp64" else evp.MIXED
    nx, ny, nz = 48, 20 if walls else 24, 16
    wl = _workload(nx, ny, nz, walls)
    G = evp.Grid(nx, ny, nz, wl.lx, wl.ly, wl.lz, walls=walls, precision=prec)
    G.set_rheology(**wl.rheology())
    if integrator == "rk3":
        G.set_integrator(evp.RK3)
    assert G.health()["guard_bad"] == 0
    u, v, w, B = inputs.random_state(wl.shape, 5, walls=walls)
    G.write_fields(*to_dev(u, v, w, B))
    G.project()
    G.step(1e-3, 6)
    assert G.health()["guard_bad"] == 0
    G.close()


def test_overwritten_guard_words_are_counted():
    import torch
    import paper_1803_09563_amd as evp
    nx, ny, nz = 32, 20, 16
    wl = _workload(nx, ny, nz, True)
    G = gpu_grid(wl)
    regions = evp.guard_regions(nx, ny, nz, walls=True)
    assert G.health()["guard_bad"] == 0
    base = (-G._ws.data_ptr()) % 256          # the grid's workspace starts at the aligned address
    hit = [regions[0], regions[len(regions) // 2], regions[-1]]
    saved = []
    for off, words in hit:
        a = base + off + 8 * (words - 1)     # last guard word of the region
        saved.append((a, G._ws[a:a + 8].clone()))
        G._ws[a:a + 8] = 0
    torch.cuda.synchronize()
    assert G.health()["guard_bad"] == len(hit)
    for a, old in saved:
        G._ws[a:a + 8] = old
    torch.cuda.synchronize()
    assert G.health()["guard_bad"] == 0
    G.close()
