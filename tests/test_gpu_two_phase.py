"""Parity of the two-phase (bubbly-flow) path of Sec. 3.2 on the GPU with the oracle's
TwoPhaseSolver: level-set transport and reinitialisation stages 1e-12, full FP64 steps (level
set, stress, momentum with surface tension, split projection) 1e-10; Laplace's law on the GPU.
All skipped while the device path is switched off."""
import numpy as np
import pytest

import oracle
from oracle import two_phase as tp
from paper_1803_09563_amd import inputs

from harness import assert_close, gpu_grid, gpu_state, oracle_state, to_dev
from test_gpu_parity import _wl

# The two-phase device path is switched off (evp_set_two_phase returns EVP_ERR_DISABLED): its
# first run on the device ended in a memory fault whose cause is not yet identified, so these
# cases stay off the device until one is shown.
pytestmark = [pytest.mark.gpu,
              pytest.mark.skip(reason="two-phase device path switched off: unexplained memory "
                                      "fault on its first device run")]


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1803_09563_amd  # noqa: F401  (fails loudly without libevp.so)
    yield


def _centres(wl):
    x = (np.arange(wl.nx) + 0.5) * wl.dx
    y = wl.y0 + (np.arange(wl.ny) + 0.5) * wl.dy
    z = (np.arange(wl.nz) + 0.5) * wl.dz
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    return X, Y, Z


def _drop(wl, c, R):
    X, Y, Z = _centres(wl)
    return np.sqrt((X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2) - R


def _pair(wl, params, fields, phi):
    g = oracle.Grid(wl.nx, wl.ny, wl.nz, wl.lx, wl.ly, wl.lz, walls=wl.walls)
    r = oracle.Rheology(**wl.rheology(), adv=wl.adv, kappa=wl.kappa)
    s = tp.TwoPhaseSolver(g, r, tp.TwoPhase(**params), forcing=wl.force,
                          walls_uv=wl.wall_velocity)
    s.write_fields(*fields)
    s.write_level_set(phi)
    G = gpu_grid(wl)
    G.set_two_phase(**params)
    G.write_fields(*to_dev(*fields))
    G.write_level_set(to_dev(phi)[0])
    return s, G


def _phi(G):
    import torch
    out = G.read_level_set()
    torch.cuda.synchronize()
    return out.cpu().numpy()


PARAMS = dict(rho1=1.0, rho2=0.5, mu_s1=0.02, mu_s2=0.05, mu_p1=0.03, mu_p2=0.01, lam1=0.5,
              lam2=0.8, sigma=0.05, reinit_every=4, reinit_iters=2)


@pytest.mark.parametrize("walls", [False, True])
def test_level_set_transport_parity(walls):
    wl = _wl(32, 24, 16, walls, "oldroyd_b", wall_velocity=(0.2, -0.1, 0.0, 0.1))
    fields = inputs.random_state(wl.shape, 61, walls=walls)
    phi = _drop(wl, (wl.lx / 2, wl.y0 + wl.ly / 2, wl.lz / 2), 0.6)
    params = dict(PARAMS, reinit_every=0)
    s, G = _pair(wl, params, fields, phi)
    s.step(2e-3, 3, flags=oracle.Solver.FREEZE_VELOCITY)
    G.step(2e-3, 3, flags=1)
    ref = s.phi
    got = _phi(G)
    assert np.abs(got - ref).max() < 1e-12 * np.abs(ref).max()
    assert_close(oracle_state(s), gpu_state(G, ("u", "v", "w", "B")), 1e-12, "freeze with phi")


@pytest.mark.parametrize("walls", [False, True])
def test_reinitialisation_parity(walls):
    wl = _wl(32, 24, 16, walls, "oldroyd_b")
    z = np.zeros(wl.shape)
    B = np.zeros((6,) + wl.shape)
    B[0] = B[3] = B[5] = 1.0
    X, Y, Z = _centres(wl)
    phi = _drop(wl, (wl.lx / 2, wl.y0 + wl.ly / 2, wl.lz / 2), 0.6) * (1.0 + 0.3 * np.cos(X))
    params = dict(PARAMS, reinit_every=1, reinit_iters=3)
    s, G = _pair(wl, params, (z, z, z, B), phi)
    s.step(1e-3, 2, flags=oracle.Solver.FREEZE_VELOCITY)
    G.step(1e-3, 2, flags=1)
    assert np.abs(_phi(G) - s.phi).max() < 1e-12 * np.abs(s.phi).max()


@pytest.mark.parametrize("model", ["oldroyd_b", "fene_p", "saramito"])
@pytest.mark.parametrize("walls", [False, True])
def test_two_phase_full_step_parity(model, walls):
    wl = _wl(32, 24, 16, walls, model, wall_velocity=(-0.3, 0.3, 0.0, 0.0),
             force=(inputs.FORCE_CONST_X, 0.2, 0.0))
    u, v, w, B = inputs.random_state(wl.shape, 62, amp_u=0.1, walls=walls)
    g = oracle.Grid(wl.nx, wl.ny, wl.nz, wl.lx, wl.ly, wl.lz, walls=walls)
    u, v, w, _ = oracle.project(g, u, v, w, 1.0)
    phi = _drop(wl, (wl.lx / 2, wl.y0 + wl.ly / 2, wl.lz / 2), 0.7)
    s, G = _pair(wl, PARAMS, (u, v, w, B), phi)
    s.step(1e-3, 12)
    G.step(1e-3, 12)
    ref = oracle_state(s)
    assert_close(ref, gpu_state(G), 1e-10, f"two-phase {model} walls={walls}, 12 steps")
    assert np.abs(_phi(G) - s.phi).max() < 1e-10 * np.abs(s.phi).max()


def test_static_drop_laplace_on_gpu():
    wl = _wl(32, 32, 32, False, "oldroyd_b")
    wl.lx = wl.ly = wl.lz = 2 * np.pi
    z = np.zeros(wl.shape)
    B = np.zeros((6,) + wl.shape)
    B[0] = B[3] = B[5] = 1.0
    R, sigma = 1.2, 0.5
    params = dict(rho1=1.0, rho2=0.2, mu_s1=0.1, mu_s2=0.1, sigma=sigma, reinit_every=0,
                  reinit_iters=0)
    phi = _drop(wl, (np.pi, np.pi, np.pi), R)
    s, G = _pair(wl, params, (z, z, z, B), phi)
    G.step(2e-3, 20)
    st = gpu_state(G, ("u", "v", "w", "p"))
    inside, outside = phi < -0.5 * R, phi > 1.0
    jump = st["p"][inside].mean() - st["p"][outside].mean()
    assert abs(jump / (2 * sigma / R) - 1) < 0.08, jump
    s.step(2e-3, 20)
    assert_close(oracle_state(s), st, 1e-10, "static drop")


def test_two_phase_batch_equals_single():
    import paper_1803_09563_amd as evp
    wl = _wl(32, 24, 16, False, "oldroyd_b")
    singles, batched = [], []
    for seed, R in ((63, 0.6), (64, 0.8)):
        u, v, w, B = inputs.random_state(wl.shape, seed, amp_u=0.1)
        phi = _drop(wl, (wl.lx / 2, wl.ly / 2, wl.lz / 2), R)
        pair = []
        for _ in range(2):
            G = gpu_grid(wl)
            G.set_two_phase(**PARAMS)
            G.write_fields(*to_dev(u, v, w, B))
            G.write_level_set(to_dev(phi)[0])
            G.project()
            pair.append(G)
        pair[0].step(1e-3, 6)
        singles.append(pair[0])
        batched.append(pair[1])
    evp.step_batch(batched, 1e-3, 6)
    for a, b in zip(singles, batched):
        sa, sb = gpu_state(a), gpu_state(b)
        for k in sa:
            assert np.array_equal(sa[k], sb[k]), k
        assert np.array_equal(_phi(a), _phi(b))


def test_two_phase_argument_errors():
    import paper_1803_09563_amd as evp
    wl = _wl(32, 24, 16, False, "oldroyd_b")
    m = gpu_grid(wl, precision=evp.MIXED)
    with pytest.raises(evp.EvpError) as e:
        m.set_two_phase(**PARAMS)
    assert e.value.status == -1
    G = gpu_grid(wl)
    G.set_integrator("rk3")
    with pytest.raises(evp.EvpError):
        G.set_two_phase(**PARAMS)
    G.set_integrator("ab2")
    G.set_two_phase(**PARAMS)
    with pytest.raises(evp.EvpError):
        G.set_integrator("rk3")
    with pytest.raises(evp.EvpError):
        G.set_solid(to_dev(*[np.zeros(wl.shape)] * 3))
    with pytest.raises(evp.EvpError):
        G.set_two_phase(rho1=-1.0)
    single = gpu_grid(wl)
    z = to_dev(*[np.zeros(wl.shape)] * 3)
    B = np.zeros((6,) + wl.shape)
    B[0] = B[3] = B[5] = 1.0
    for x in (G, single):
        x.write_fields(*z, to_dev(B)[0])
    with pytest.raises(evp.EvpError) as e:
        evp.step_batch([G, single], 1e-3, 1)
    assert e.value.status == -4
