"""Serving loop: continuous batching over the C-ABI.  Each request's result is bitwise the same
alone and in the mix, also when a shape group holds enough z planes (256 and more) for the fused
plane projection passes; a served request matches the oracle; the HBM budget and slot caps bind; a
request that blows up (NaN) is retired with an error without touching the others; the health
check enqueued without waiting gives the numbers of the waiting one."""
import numpy as np
import pytest

from paper_1803_09563_amd import inputs

pytestmark = pytest.mark.gpu


def _requests(n=10, seed=7, steps=(20, 60), sizes=(32, 48)):
    from paper_1803_09563_amd.serving import make_requests
    reqs = make_requests(n, rate=None, seed=seed, step_range=steps, sizes=sizes)
    for i, r in enumerate(reqs):
        r.arrival = 0.002 * i            # staggered: later requests join running batches
    return reqs


def _alone(wl):
    import torch
    import paper_1803_09563_amd as evp
    from paper_1803_09563_amd.serving import device_initial_fields
    G = evp.Grid(wl.nx, wl.ny, wl.nz, wl.lx, wl.ly, wl.lz, walls=wl.walls,
                 precision=evp.MIXED if wl.precision == "mixed" else evp.FP64)
    G.set_rheology(**wl.rheology())
    G.set_forcing(*wl.force)
    G.write_fields(*device_initial_fields(wl))
    G.project()
    G.step(wl.dt, wl.steps)
    out = G.read_fields(("u", "v", "w", "p", "B"))
    torch.cuda.synchronize()
    return {k: t.cpu().numpy() for k, t in out.items()}, G.health()


def test_results_identical_alone_and_in_the_mix():
    from paper_1803_09563_amd.serving import Server
    reqs = _requests()
    stats = Server(keep_fields=True, chunk=7).run(reqs, time_limit=120)
    assert stats["requests"] == len(reqs) and stats["errors"] == 0
    assert stats["launches"] < sum(-(-r.wl.steps // 7) for r in reqs)   # batching happened
    for r in reqs:
        ref, _ = _alone(r.wl)
        for k in ("u", "v", "w", "p", "B"):
            assert np.array_equal(ref[k], r.fields[k]), (r.rid, k)
    assert stats["p99_latency_s"] >= stats["p50_latency_s"] > 0


@pytest.mark.parametrize("sizes,n", [((32,), 8), ((96, 128), 6)])
def test_fused_plane_groups_identical_alone_and_in_the_mix(sizes, n):
    """All requests arrive together: 8 x 32^3 (256 planes) or 96^3 and 128^3 grids (3 x 96 and
    2 x 128 planes) share a launch, which then takes the fused plane projection passes; each
    request alone takes the separate passes."""
    from paper_1803_09563_amd.serving import Server
    reqs = _requests(n=n, seed=23, steps=(10, 20), sizes=sizes)
    for r in reqs:
        r.arrival = 0.0
    planes = {}
    for r in reqs:
        planes[r.wl.nx] = planes.get(r.wl.nx, 0) + r.wl.nz
    assert max(planes.values()) >= 256, planes
    stats = Server(keep_fields=True, chunk=5).run(reqs, time_limit=120)
    assert stats["requests"] == n and stats["errors"] == 0
    for r in reqs:
        ref, _ = _alone(r.wl)
        for k in ("u", "v", "w", "p", "B"):
            assert np.array_equal(ref[k], r.fields[k]), (r.rid, r.wl.nx, k)


def test_served_request_matches_oracle():
    """One request served in a mix, against the FP64 oracle from the same initial fields (the
    device-generated fields are read back and handed to the oracle): mixed-precision bar."""
    import torch
    from paper_1803_09563_amd.serving import Server, device_initial_fields
    from harness import assert_close, oracle_solver
    reqs = _requests(n=5, seed=31, steps=(30, 40), sizes=(32, 48))
    Server(keep_fields=True, chunk=7).run(reqs, time_limit=120)
    r = reqs[1]
    u, v, w, B = [t.cpu().numpy() for t in device_initial_fields(r.wl)]
    torch.cuda.synchronize()
    s = oracle_solver(r.wl)
    s.write_fields(u, v, w, B)
    s.project()
    s.step(r.wl.dt, r.wl.steps)
    ref = {"u": s.u, "v": s.v, "w": s.w, "p": s.p, "B": s.B}
    assert_close(ref, r.fields, 1e-4, f"served request {r.rid}", p_tol=1e-3)


def test_health_enqueue_equals_health():
    import torch
    import paper_1803_09563_amd as evp
    wl = _requests(n=1, seed=3, sizes=(48,))[0].wl
    from paper_1803_09563_amd.serving import device_initial_fields
    G = evp.Grid(wl.nx, wl.ny, wl.nz, wl.lx, wl.ly, wl.lz, precision=evp.MIXED)
    G.set_rheology(**wl.rheology())
    G.set_forcing(*wl.force)
    G.write_fields(*device_initial_fields(wl))
    G.project()
    G.step(wl.dt, 5)
    out = torch.empty(5, dtype=torch.float64, device="cuda")
    G.health_enqueue(out)
    torch.cuda.synchronize()
    hv = G.health_values(out)
    assert hv == {k: v for k, v in G.health().items() if k in hv}


def test_budget_and_slots_bind():
    import paper_1803_09563_amd as evp
    from paper_1803_09563_amd.serving import Server
    reqs = _requests(n=8, seed=11)
    for r in reqs:
        r.arrival = 0.0
    per = max(evp.workspace_bytes(r.wl.nx, r.wl.ny, r.wl.nz, False, evp.MIXED) for r in reqs)
    srv = Server(budget_bytes=2.5 * per, max_active=3, chunk=10)
    stats = srv.run(reqs, time_limit=120)
    assert stats["requests"] == 8 and stats["errors"] == 0
    assert stats["peak_active"] <= 3 and stats["peak_hbm_bytes"] <= 2.5 * per


def test_failure_is_isolated():
    from paper_1803_09563_amd.serving import Server
    reqs = _requests(n=6, seed=5)
    bad = reqs[2]
    bad.wl.extra = dict(bad.wl.extra, inject_nan=True)
    Server(keep_fields=True, chunk=5).run(reqs, time_limit=120)
    assert bad.status == "error"
    for r in reqs:
        if r is bad:
            continue
        assert r.status == "done"
        ref, _ = _alone(r.wl)
        assert np.array_equal(ref["u"], r.fields["u"]) and np.array_equal(ref["B"], r.fields["B"])
