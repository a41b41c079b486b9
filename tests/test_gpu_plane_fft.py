"""Periodic batches with at least 256 z planes of nx == ny <= 128 take the fused projection passes
(divergence + x and y transforms in one kernel, inverse y and x transforms in another, one block
per z plane).  Each grid of such a batch must match the oracle (FP64 1e-10, mixed 1e-4 per
field) and the same grid stepped alone, which takes the separate line-transform passes."""
import numpy as np
import pytest

import oracle
from paper_1803_09563_amd import inputs

from harness import assert_close, field_errors, gpu_grid, gpu_state, oracle_solver, oracle_state, to_dev
from test_gpu_parity import _wl

pytestmark = pytest.mark.gpu

MODELS3 = ("saramito", "fene_p", "oldroyd_b")


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1803_09563_amd  # noqa: F401  (fails loudly without libevp.so)
    yield


def _batch(n, nz, count, precision, seed0):
    out = []
    for i in range(count):
        wl = _wl(n, n, nz, False, MODELS3[i % 3], force=(inputs.FORCE_CONST_X, 0.2, 0.0))
        wl.precision = precision
        out.append((wl, inputs.random_state(wl.shape, seed0 + i, amp_u=0.1)))
    return out


# 8 x 32^3 and 16 x 16^3 (256 planes each), 2 x 128 x 128 x 128 is left to the bench
@pytest.mark.parametrize("n,nz,count", [(32, 32, 8), (16, 16, 16)])
def test_plane_batch_fp64_parity(n, nz, count):
    import paper_1803_09563_amd as evp
    cases = _batch(n, nz, count, "fp64", 300)
    grids = []
    for wl, fields in cases:
        G = gpu_grid(wl)
        G.write_fields(*to_dev(*fields))
        grids.append(G)
    evp.step_batch(grids, 1e-3, 20)
    for (wl, fields), G in zip(cases, grids):
        s = oracle_solver(wl)
        s.write_fields(*fields)
        s.step(1e-3, 20)
        assert_close(oracle_state(s), gpu_state(G), 1e-10, f"{wl.name} FP64 batch of {count}, 20 steps")


def test_plane_batch_mixed_parity():
    import paper_1803_09563_amd as evp
    cases = _batch(24, 24, 12, "mixed", 400)          # 288 planes
    grids = []
    for wl, fields in cases:
        G = gpu_grid(wl)
        G.write_fields(*to_dev(*fields))
        grids.append(G)
    evp.step_batch(grids, 1e-3, 20)
    for (wl, fields), G in zip(cases, grids):
        s = oracle_solver(wl)
        s.write_fields(*fields)
        s.step(1e-3, 20)
        assert_close(oracle_state(s), gpu_state(G), 1e-4, f"{wl.name} mixed batch, 20 steps", p_tol=1e-3)


# 128^2 and 96^2 planes: the largest plane that fits in LDS, and a radix-3 length.  The fused
# passes use the same transforms, twiddles and two-for-one formulas in the same order as the
# separate passes, so every grid of the batch must equal the grid stepped alone bit for bit; the
# first grid is also compared with the oracle.
@pytest.mark.parametrize("n,nz,count,precision", [(128, 8, 32, "fp64"), (96, 64, 4, "mixed"),
                                                  (64, 16, 16, "fp64")])
def test_plane_batch_equals_single(n, nz, count, precision):
    import paper_1803_09563_amd as evp
    cases = _batch(n, nz, count, precision, 500)
    batched = []
    for wl, fields in cases:
        G = gpu_grid(wl)
        G.write_fields(*to_dev(*fields))
        batched.append(G)
    evp.step_batch(batched, 1e-3, 10)
    # the fused passes at this plane size against the oracle too (first grid of the batch)
    wl0, fields0 = cases[0]
    s = oracle_solver(wl0)
    s.write_fields(*fields0)
    s.step(1e-3, 10)
    if precision == "fp64":
        assert_close(oracle_state(s), gpu_state(batched[0]), 1e-10, f"{wl0.name} FP64 fused passes, 10 steps")
    else:
        assert_close(oracle_state(s), gpu_state(batched[0]), 1e-4, f"{wl0.name} mixed fused passes, 10 steps",
                     p_tol=1e-3)
    for (wl, fields), b in zip(cases, batched):
        a = gpu_grid(wl)
        a.write_fields(*to_dev(*fields))
        a.step(1e-3, 10)
        sa, sb = gpu_state(a), gpu_state(b)
        a.close()
        for k in sa:
            assert np.array_equal(sa[k], sb[k]), (wl.name, k, field_errors(sa, sb))
