"""Parity of the HIP path (through the C-ABI) with the FP64 oracle on the same seeded inputs.

Bars: single predictor stage and projection 1e-12 (FP64 rounding order only); full FP64 steps
1e-10 max relative error per field after up to 100 steps; mixed precision 1e-4 per field.
Shapes span several tiles with ragged tails (x tile 64, y tile 4, FFT line groups).
"""
import numpy as np
import pytest

import oracle
from paper_1803_09563_amd import inputs

from harness import assert_close, gpu_grid, gpu_state, oracle_solver, oracle_state, to_dev

pytestmark = pytest.mark.gpu

MODELS = {
    "oldroyd_b": dict(model=inputs.OLDROYD_B, mu_s=0.01, mu_p=0.02, lam=0.5),
    "fene_p": dict(model=inputs.FENE_P, mu_s=0.01, mu_p=0.02, lam=0.5, L2=50.0),
    "saramito": dict(model=inputs.SARAMITO, mu_s=0.01, mu_p=0.02, lam=0.5, tau_y=0.002),
}


def _wl(nx, ny, nz, walls, model, **kw):
    m = dict(MODELS[model])
    L = 2 * np.pi
    wl = inputs.Workload(f"t{nx}x{ny}x{nz}", nx, ny, nz, L, 2.0 if walls else L * ny / nx,
                         L * nz / nx, walls, m.pop("model"), m.pop("mu_s"), m.pop("mu_p"),
                         m.pop("lam"), **m)
    for k, v in kw.items():
        setattr(wl, k, v)
    return wl


SHAPES = {"periodic": (48, 24, 16, False), "walls": (32, 22, 24, True)}


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1803_09563_amd  # noqa: F401  (fails loudly without libevp.so)
    yield


@pytest.mark.parametrize("model", list(MODELS))
@pytest.mark.parametrize("bc", list(SHAPES))
def test_predictor_stage_parity(model, bc):
    nx, ny, nz, walls = SHAPES[bc]
    wl = _wl(nx, ny, nz, walls, model, force=(inputs.FORCE_SIN_X_OF_Y, 0.7, 2.0),
             wall_velocity=(0.2, -0.1, 0.05, 0.3))
    u, v, w, B = inputs.random_state(wl.shape, 11, walls=walls)
    rng = np.random.default_rng(12)
    hist = 0.1 * rng.standard_normal((9,) + wl.shape)
    s = oracle_solver(wl)
    s.write_fields(u, v, w, B, hist)
    s.step(1e-3, 1, flags=oracle.Solver.STOP_AFTER_PREDICTOR)
    G = gpu_grid(wl)
    G.write_fields(*to_dev(u, v, w, B, hist))
    G.step(1e-3, 1, flags=2)
    got = gpu_state(G, ("u", "v", "w", "B", "hist"))
    assert_close(oracle_state(s), got, 1e-12, f"predictor {model} {bc}")
    ref_hist = np.concatenate([s.RT, s.RU])
    scale = np.abs(ref_hist).max(axis=(1, 2, 3))
    err = np.abs(got["hist"] - ref_hist).max(axis=(1, 2, 3)) / np.maximum(scale, 1e-300)
    assert err.max() < 1e-11, err


@pytest.mark.parametrize("bc", list(SHAPES))
def test_euler_start_and_freeze(bc):
    nx, ny, nz, walls = SHAPES[bc]
    wl = _wl(nx, ny, nz, walls, "saramito")
    u, v, w, B = inputs.random_state(wl.shape, 5, walls=walls)
    s = oracle_solver(wl)
    s.write_fields(u, v, w, B)
    s.step(2e-3, 3, flags=oracle.Solver.FREEZE_VELOCITY)
    G = gpu_grid(wl)
    G.write_fields(*to_dev(u, v, w, B))
    G.step(2e-3, 3, flags=1)
    got = gpu_state(G, ("u", "v", "w", "B"))
    assert np.array_equal(got["u"], s.u) and np.array_equal(got["w"], s.w)
    assert_close(oracle_state(s), got, 1e-12, "freeze")


@pytest.mark.parametrize("bc", list(SHAPES))
def test_projection_parity(bc):
    nx, ny, nz, walls = SHAPES[bc]
    wl = _wl(nx, ny, nz, walls, "oldroyd_b")
    u, v, w, B = inputs.random_state(wl.shape, 21, walls=walls)
    s = oracle_solver(wl)
    s.write_fields(u, v, w, B)
    us, vs, ws, p = oracle.project(s.g, s.u, s.v, s.w, 1.0)
    G = gpu_grid(wl)
    G.write_fields(*to_dev(u, v, w, B))
    G.project()
    got = gpu_state(G, ("u", "v", "w", "p"))
    ref = {"u": us, "v": vs, "w": ws, "p": p}
    assert_close(ref, got, 1e-12, f"projection {bc}")
    div = np.abs(oracle.divergence(s.g, got["u"], got["v"], got["w"])).max()
    umax = max(np.abs(got[k]).max() for k in "uvw")
    assert div * min(s.g.dx, s.g.dy, s.g.dz) / umax < 1e-12


@pytest.mark.parametrize("ny", [4, 17, 40, 256, 320, 1024])
def test_projection_parity_wall_heights(ny):
    """The channel solve over wall-normal sizes: one partly filled row segment (4), a last
    segment of one row (17), a ragged one (40), all sixteen segments of a block (256), and the
    sequential sweep that serves ny > 256 (320, and the largest allowed, 1024).  The bar is
    1e-12 up to ny = 256 and grows as (ny / 256)^2 beyond: the two sides solve the wall-normal
    Neumann systems with different algorithms (precomputed-pivot Thomas sweeps against a banded
    LU), whose rounding differences grow with the systems' condition number, about ny^2 for the
    lowest modes (1.2e-12 on v at ny = 1024, p within 5e-14)."""
    nx, nz = 16, 12
    wl = _wl(nx, ny, nz, True, "oldroyd_b")
    u, v, w, B = inputs.random_state(wl.shape, 23 + ny, walls=True)
    s = oracle_solver(wl)
    s.write_fields(u, v, w, B)
    us, vs, ws, p = oracle.project(s.g, s.u, s.v, s.w, 1.0)
    G = gpu_grid(wl)
    G.write_fields(*to_dev(u, v, w, B))
    G.project()
    got = gpu_state(G, ("u", "v", "w", "p"))
    tol = 1e-12 * max(1.0, (ny / 256) ** 2)
    assert_close({"u": us, "v": vs, "w": ws, "p": p}, got, tol, f"projection walls ny={ny}")
    div = np.abs(oracle.divergence(s.g, got["u"], got["v"], got["w"])).max()
    umax = max(np.abs(got[k]).max() for k in "uvw")
    assert div * min(s.g.dx, s.g.dy, s.g.dz) / umax < tol


@pytest.mark.parametrize("shape", [(40, 20, 30, False), (10, 60, 20, False), (80, 12, 60, True),
                                   (30, 9, 480, True), (320, 10, 8, False), (240, 6, 10, True)])
def test_projection_parity_radix5(shape):
    """Transform lengths with a radix-5 stage (5 2^a and 15 2^a) in x, y (periodic) and z."""
    nx, ny, nz, walls = shape
    wl = _wl(nx, ny, nz, walls, "oldroyd_b")
    u, v, w, B = inputs.random_state(wl.shape, 31 + nx, walls=walls)
    s = oracle_solver(wl)
    s.write_fields(u, v, w, B)
    us, vs, ws, p = oracle.project(s.g, s.u, s.v, s.w, 1.0)
    G = gpu_grid(wl)
    G.write_fields(*to_dev(u, v, w, B))
    G.project()
    got = gpu_state(G, ("u", "v", "w", "p"))
    assert_close({"u": us, "v": vs, "w": ws, "p": p}, got, 1e-12, f"projection {shape}")
    div = np.abs(oracle.divergence(s.g, got["u"], got["v"], got["w"])).max()
    umax = max(np.abs(got[k]).max() for k in "uvw")
    assert div * min(s.g.dx, s.g.dy, s.g.dz) / umax < 1e-12


@pytest.mark.parametrize("shape", [(8, 8, 512, False), (16, 6, 512, True), (512, 8, 8, False),
                                   (8, 512, 8, False)])
def test_projection_parity_longest_lines(shape):
    """The longest transform lines (512 points) in each direction, on thin grids."""
    nx, ny, nz, walls = shape
    wl = _wl(nx, ny, nz, walls, "oldroyd_b")
    u, v, w, B = inputs.random_state(wl.shape, 51 + nz, walls=walls)
    s = oracle_solver(wl)
    s.write_fields(u, v, w, B)
    us, vs, ws, p = oracle.project(s.g, s.u, s.v, s.w, 1.0)
    G = gpu_grid(wl)
    G.write_fields(*to_dev(u, v, w, B))
    G.project()
    got = gpu_state(G, ("u", "v", "w", "p"))
    assert_close({"u": us, "v": vs, "w": ws, "p": p}, got, 1e-12, f"projection {shape}")


@pytest.mark.parametrize("shape", [(8, 8, 8, False), (8, 4, 8, True)])
def test_smallest_grid_steps_parity(shape):
    """The smallest grids allowed (8 cells per FFT direction, 4 between walls): one partly filled
    32 x 8 predictor tile per plane.  FP64 to 1e-10 and mixed to 1e-4 after 20 Saramito steps."""
    import paper_1803_09563_amd as evp
    nx, ny, nz, walls = shape
    wl = _wl(nx, ny, nz, walls, "saramito", wall_velocity=(0.1, -0.1, 0.0, 0.05) if walls else (0, 0, 0, 0))
    u, v, w, B = inputs.random_state(wl.shape, 61, walls=walls)
    s = oracle_solver(wl)
    s.write_fields(u, v, w, B)
    s.project()
    s.step(1e-3, 20)
    ref = oracle_state(s)
    for prec, tol in ((evp.FP64, 1e-10), (evp.MIXED, 1e-4)):
        G = gpu_grid(wl, precision=prec)
        G.write_fields(*to_dev(u, v, w, B))
        G.project()
        G.step(1e-3, 20)
        assert_close(ref, gpu_state(G), tol, f"smallest grid {shape} precision {prec}",
                     p_tol=1e-3 if prec == evp.MIXED else None)


@pytest.mark.parametrize("walls", [False, True])
def test_radix5_grid_steps_parity(walls):
    """Saramito steps on a grid with radix-5 transform lengths: FP64 to 1e-10, mixed to 1e-4."""
    nx, ny, nz = (40, 20, 30) if not walls else (60, 14, 40)
    wl = _wl(nx, ny, nz, walls, "saramito")
    u, v, w, B = inputs.random_state(wl.shape, 41, walls=walls)
    s = oracle_solver(wl)
    s.write_fields(u, v, w, B)
    s.project()
    s.step(1e-3, 10)
    ref = oracle_state(s)
    for prec, tol in (("fp64", 1e-10), ("mixed", 1e-4)):
        import paper_1803_09563_amd as evp
        G = gpu_grid(wl, precision=evp.FP64 if prec == "fp64" else evp.MIXED)
        G.write_fields(*to_dev(u, v, w, B))
        G.project()
        G.step(1e-3, 10)
        got = gpu_state(G)
        assert_close(ref, got, tol, f"radix-5 grid {prec}", p_tol=1e-3 if prec == "mixed" else None)


def test_zero_steps_change_nothing():
    """Zero steps (alone and as a batch) leave the state and the step count exactly as they were."""
    import paper_1803_09563_amd as evp
    wl = _wl(32, 22, 24, True, "saramito")
    u, v, w, B = inputs.random_state(wl.shape, 71, walls=True)
    G = gpu_grid(wl)
    G.write_fields(*to_dev(u, v, w, B))
    G.project()
    G.step(1e-3, 2)
    which = ("u", "v", "w", "p", "B", "hist")
    before, n0 = gpu_state(G, which), G.step_count()
    G.step(1e-3, 0)
    evp.step_batch([G], 1e-3, 0)
    after = gpu_state(G, which)
    assert G.step_count() == n0
    for k in which:
        assert np.array_equal(before[k], after[k]), k


def test_taylor_green_32_full_parity_100_steps():
    wl = inputs.taylor_green_periodic(32)
    u, v, w, B = inputs.initial_fields(wl)
    s = oracle_solver(wl)
    s.write_fields(u, v, w, B)
    s.step(wl.dt, wl.steps)
    G = gpu_grid(wl)
    G.write_fields(*to_dev(u, v, w, B))
    G.step(wl.dt, wl.steps)
    assert_close(oracle_state(s), gpu_state(G), 1e-10, "taylor-green 32^3, 100 steps")


@pytest.mark.parametrize("case", ["kolmogorov_saramito_48", "channel_fene_p_64x48x32",
                                  "channel_saramito_48x36x24", "couette_oldroyd_b_32x20x16"])
def test_full_step_parity_100_steps(case):
    if case == "kolmogorov_saramito_48":
        wl = inputs.kolmogorov_saramito(48)
    elif case == "channel_fene_p_64x48x32":
        wl = inputs.channel_fene_p(64, 48, 32, precision="fp64")
    elif case == "channel_saramito_48x36x24":
        wl = inputs.channel_saramito(48, 36, 24)
        wl.tau_y = 2e-3          # some cells yield within 100 steps, some do not
    else:
        wl = _wl(32, 20, 16, True, "oldroyd_b", wall_velocity=(-1.0, 1.0, 0.0, 0.0),
                 init="zero")
    u, v, w, B = inputs.initial_fields(wl)
    s = oracle_solver(wl)
    s.write_fields(u, v, w, B)
    G = gpu_grid(wl)
    G.write_fields(*to_dev(u, v, w, B))
    if wl.project_initial:
        s.project()
        G.project()
    s.step(wl.dt, 100)
    G.step(wl.dt, 100)
    assert_close(oracle_state(s), gpu_state(G), 1e-10, f"{case}, 100 steps")


def test_mixed_stage_fine_spacing():
    """FP32 WENO weights on a fine grid near B = I (smoothness indicators ~ eps h^2): the
    predictor stays finite and within the mixed tolerance of the FP64 oracle."""
    import paper_1803_09563_amd as evp
    wl = inputs.channel_fene_p(64, 256, 16, precision="mixed")
    u, v, w, B = inputs.initial_fields(wl)
    s = oracle_solver(wl)
    s.write_fields(u, v, w, B)
    s.step(wl.dt, 2, flags=oracle.Solver.STOP_AFTER_PREDICTOR)
    G = gpu_grid(wl, precision=evp.MIXED)
    G.write_fields(*to_dev(u, v, w, B))
    G.step(wl.dt, 2, flags=2)
    got = gpu_state(G, ("u", "v", "w", "B"))
    assert all(np.isfinite(x).all() for x in got.values())
    assert_close(oracle_state(s), got, 1e-4, "mixed fine spacing")


@pytest.mark.parametrize("case", ["kolmogorov_saramito_48", "channel_fene_p_64x48x32"])
def test_mixed_precision_error(case):
    import paper_1803_09563_amd as evp
    if case == "kolmogorov_saramito_48":
        wl = inputs.kolmogorov_saramito(48)
    else:
        wl = inputs.channel_fene_p(64, 48, 32, precision="mixed")
    u, v, w, B = inputs.initial_fields(wl)
    s = oracle_solver(wl)
    s.write_fields(u, v, w, B)
    s.project()
    s.step(wl.dt, 200)
    G = gpu_grid(wl, precision=evp.MIXED)
    G.write_fields(*to_dev(u, v, w, B))
    G.project()
    G.step(wl.dt, 200)
    assert_close(oracle_state(s), gpu_state(G), 1e-4, f"mixed {case}, 200 steps", p_tol=1e-3)


def test_batch_equals_single_bitwise():
    import paper_1803_09563_amd as evp
    wls = [inputs.kolmogorov_saramito(32), inputs.kolmogorov_saramito(32)]
    wls[1].model, wls[1].L2, wls[1].tau_y = inputs.FENE_P, 60.0, 0.0
    wls[1].seed = 99
    singles, batched = [], []
    for wl in wls:
        u, v, w, B = inputs.initial_fields(wl)
        a, b = gpu_grid(wl), gpu_grid(wl)
        for G in (a, b):
            G.write_fields(*to_dev(u, v, w, B))
            G.project()
        a.step(wl.dt, 20)
        singles.append(a)
        batched.append(b)
    evp.step_batch(batched, 1e-3, 20)
    for a, b in zip(singles, batched):
        sa, sb = gpu_state(a), gpu_state(b)
        for k in sa:
            assert np.array_equal(sa[k], sb[k]), k


def test_checkpoint_resume_bitwise():
    """Raw checkpoint (evp_save_state / evp_load_state): bitwise continuation."""
    wl = inputs.kolmogorov_saramito(32)
    u, v, w, B = inputs.initial_fields(wl)
    a = gpu_grid(wl)
    a.write_fields(*to_dev(u, v, w, B))
    a.project()
    a.step(wl.dt, 10)
    ck = a.save_state()
    b = gpu_grid(wl)
    b.load_state(ck)
    assert b.step_count() == 10
    a.step(wl.dt, 10)
    b.step(wl.dt, 10)
    sa, sb = gpu_state(a), gpu_state(b)
    for k in ("u", "v", "w", "p", "B"):
        assert np.array_equal(sa[k], sb[k]), k


def test_checkpoint_through_fp64_fields():
    """Portable checkpoint through read_fields/write_fields with the AB2 history: exact up to the
    rounding of B = (B - I) + I in FP64."""
    wl = inputs.kolmogorov_saramito(32)
    u, v, w, B = inputs.initial_fields(wl)
    a = gpu_grid(wl)
    a.write_fields(*to_dev(u, v, w, B))
    a.project()
    a.step(wl.dt, 10)
    ck = gpu_state(a, ("u", "v", "w", "B", "hist"))
    b = gpu_grid(wl)
    b.write_fields(*to_dev(ck["u"], ck["v"], ck["w"], ck["B"], ck["hist"]))
    a.step(wl.dt, 10)
    b.step(wl.dt, 10)
    err = assert_close(gpu_state(a), gpu_state(b), 1e-10, "fp64 checkpoint")
    assert max(v for k, v in err.items() if k != "p") < 1e-13, err


def test_determinism():
    wl = inputs.channel_fene_p(64, 48, 32, precision="fp64")
    u, v, w, B = inputs.initial_fields(wl)
    res = []
    for _ in range(2):
        G = gpu_grid(wl)
        G.write_fields(*to_dev(u, v, w, B))
        G.project()
        G.step(wl.dt, 10)
        res.append(gpu_state(G))
        res[-1]["health"] = G.health()
    for k in ("u", "v", "w", "p", "B"):
        assert np.array_equal(res[0][k], res[1][k]), k
    assert res[0]["health"] == res[1]["health"]


def test_health_counts_match_oracle():
    wl = _wl(32, 24, 16, False, "fene_p")
    u, v, w, B = inputs.random_state(wl.shape, 3, amp_b=0.3)
    B[0, 0, 0, :5] = 60.0          # trace beyond 0.95 L^2
    B[1, 1, 2, 3] = 5.0            # det < 0
    u[2, 3, 4] = np.nan
    s = oracle_solver(wl)
    s.write_fields(u, v, w, B)
    G = gpu_grid(wl)
    G.write_fields(*to_dev(u, v, w, B))
    h, ref = G.health(), s.health()
    for k in ("nonfinite", "det_le0", "trace_ge95"):
        assert h[k] == ref[k], (k, h, ref)
    u[2, 3, 4] = 0.0
    s.write_fields(u, v, w, B)
    G.write_fields(*to_dev(u, v, w, B))
    h, ref = G.health(), s.health()
    assert abs(h["energy"] - ref["energy"]) <= 1e-12 * ref["energy"]
    assert abs(h["max_div"] - ref["max_div"]) <= 1e-12 * ref["max_div"]
