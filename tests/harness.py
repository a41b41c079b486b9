"""Shared test helpers: run one workload through the oracle and through the HIP path (C-ABI) from
the same seeded inputs, and compare per field."""
from __future__ import annotations

import numpy as np

import oracle
from paper_1803_09563_amd import inputs


def oracle_solver(wl: inputs.Workload):
    g = oracle.Grid(wl.nx, wl.ny, wl.nz, wl.lx, wl.ly, wl.lz, walls=wl.walls)
    r = oracle.Rheology(**wl.rheology(), adv=wl.adv, kappa=wl.kappa)
    return oracle.Solver(g, r, forcing=wl.force, walls_uv=wl.wall_velocity)


def gpu_grid(wl: inputs.Workload, precision=None, stream=None):
    import paper_1803_09563_amd as evp
    prec = precision if precision is not None else (evp.MIXED if wl.precision == "mixed" else evp.FP64)
    G = evp.Grid(wl.nx, wl.ny, wl.nz, wl.lx, wl.ly, wl.lz, walls=wl.walls, precision=prec,
                 stream=stream)
    G.set_rheology(**wl.rheology())
    G.set_forcing(*wl.force)
    G.set_transport(wl.adv, wl.kappa)
    if wl.walls:
        G.set_walls(*wl.wall_velocity)
    return G


def to_dev(*arrs):
    import torch
    return [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in arrs]


def gpu_state(G, which=("u", "v", "w", "p", "B")):
    import torch
    out = G.read_fields(which)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


def oracle_state(s):
    return {"u": s.u, "v": s.v, "w": s.w, "p": s.p, "B": s.B}


def field_errors(ref: dict, got: dict):
    """Max errors: velocity components relative to the largest velocity magnitude, B - I
    components relative to the largest |B - I|, p relative to max |p - mean p| (floored at
    1e-6 rho U^2, so a flow whose pressure is identically zero compares rounding noise against
    a physical pressure scale)."""
    err = {}
    vmax = max(np.abs(ref[k]).max() for k in ("u", "v", "w"))
    for k in ("u", "v", "w"):
        err[k] = float(np.abs(got[k] - ref[k]).max() / max(vmax, 1e-300))
    if "B" in ref and "B" in got:
        I6 = np.array([1.0, 0, 0, 1.0, 0, 1.0])[:, None, None, None]
        rb, gb = ref["B"] - I6, got["B"] - I6
        bmax = np.abs(rb).max()
        names = ("Bxx", "Bxy", "Bxz", "Byy", "Byz", "Bzz")
        for c in range(6):
            err[names[c]] = float(np.abs(gb[c] - rb[c]).max() / max(bmax, 1e-300))
    if "p" in ref and "p" in got:
        rp = ref["p"] - ref["p"].mean()
        gp = got["p"] - got["p"].mean()
        err["p"] = float(np.abs(gp - rp).max() / max(np.abs(rp).max(), 1e-6 * vmax ** 2, 1e-300))
    return err


def assert_close(ref, got, tol, what="", p_tol=None):
    """All fields within tol; the pressure within p_tol (default tol)."""
    err = field_errors(ref, got)
    p_tol = tol if p_tol is None else p_tol
    bad = {k: v for k, v in err.items() if not (v <= (p_tol if k == "p" else tol))}
    assert not bad, f"{what}: fields above {tol}: {bad} (all: {err})"
    return err
