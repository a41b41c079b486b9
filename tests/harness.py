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
    """Fields of a GPU grid as numpy arrays; also checks that no kernel has written past the end
    of a workspace region (the guard words after every region are intact)."""
    import torch
    out = G.read_fields(which)
    torch.cuda.synchronize()
    assert G.health()["guard_bad"] == 0, "a kernel wrote over workspace guard words"
    return {k: v.cpu().numpy() for k, v in out.items()}


def oracle_state(s):
    return {"u": s.u, "v": s.v, "w": s.w, "p": s.p, "B": s.B}


# A field smaller than this share of its group's largest component (velocity components, the
# six components of B - I) is compared against that share instead of its own maximum: its rounding
# error comes from arithmetic on the larger components, so an own-scale figure for it would measure
# the others' size, not its own accuracy.
FLOOR = 1e-3


def field_errors(ref: dict, got: dict, shared: bool = False):
    """Max error of each field over the reference's max of that same field, |x - x_ref|_inf /
    max(|x_ref|_inf, FLOOR * group scale), where the group scale is the largest velocity component
    (u, v, w) or the largest |B - I| component (B); p is compared after removing its mean, against
    max |p_ref - mean| floored at 1e-6 rho U^2 (a flow whose pressure is identically zero then
    compares rounding noise against a physical pressure scale).  shared=True divides every field
    by its group scale instead (the looser figure)."""
    err = {}
    vmax = max(np.abs(ref[k]).max() for k in ("u", "v", "w"))
    for k in ("u", "v", "w"):
        own = np.abs(ref[k]).max()
        den = vmax if shared else max(own, FLOOR * vmax)
        err[k] = float(np.abs(got[k] - ref[k]).max() / max(den, 1e-300))
    if "B" in ref and "B" in got:
        I6 = np.array([1.0, 0, 0, 1.0, 0, 1.0])[:, None, None, None]
        rb, gb = ref["B"] - I6, got["B"] - I6
        bmax = np.abs(rb).max()
        names = ("Bxx", "Bxy", "Bxz", "Byy", "Byz", "Bzz")
        for c in range(6):
            own = np.abs(rb[c]).max()
            den = bmax if shared else max(own, FLOOR * bmax)
            err[names[c]] = float(np.abs(gb[c] - rb[c]).max() / max(den, 1e-300))
    if "p" in ref and "p" in got:
        rp = ref["p"] - ref["p"].mean()
        gp = got["p"] - got["p"].mean()
        err["p"] = float(np.abs(gp - rp).max() / max(np.abs(rp).max(), 1e-6 * vmax ** 2, 1e-300))
    return err


def assert_close(ref, got, tol, what="", p_tol=None):
    """All fields within tol (each against its own scale, see field_errors); the pressure within
    p_tol (default tol)."""
    err = field_errors(ref, got)
    p_tol = tol if p_tol is None else p_tol
    bad = {k: v for k, v in err.items() if not (v <= (p_tol if k == "p" else tol))}
    assert not bad, f"{what}: fields above {tol}: {bad} (all: {err})"
    return err
