"""Continuous-batching serving loop for rheology parameter-sweep solves.

Requests (one solve each: grid n^3, model, Wi / Bi / beta, number of steps) arrive over time.  The
loop

* admits an arrived request when its workspace (``evp_workspace_bytes``) fits the HBM budget and an
  active slot is free (FIFO, no overtaking);
* keeps every admitted solve's fields resident on the device;
* groups active solves by shape; each group owns a HIP stream and advances up to ``MAX_BATCH``
  solves per ``evp_step_batch`` launch, in chunks of a few steps, so groups of different shapes
  overlap on the device and new requests join at chunk boundaries;
* retires a solve when its steps are done: the health check (and the optional field copy) is
  enqueued on the group's stream behind an event, the loop goes on, and once the event has
  passed the solve's result is read and its workspace freed, which lets waiting requests in.

Latency of a request = completion time - arrival time.  Every step runs in the library's kernels;
this module only schedules.
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np

from . import FP64, MAX_BATCH, MIXED, Grid, step_batch, workspace_bytes
from . import inputs

__all__ = ["Request", "Server", "device_initial_fields"]


def device_initial_fields(wl: inputs.Workload, device="cuda"):
    """Kolmogorov initial state generated on the device from the request's seed (u = sin 4y +
    uniform noise, v = w = noise, B = I).  Seeded torch generator: the same request always gets the
    same fields, alone or in a mix."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(wl.seed))
    shp = wl.shape
    yc = wl.y0 + (torch.arange(wl.ny, device=device, dtype=torch.float64) + 0.5) * wl.dy
    amp = wl.noise
    noise = lambda: (torch.rand(shp, generator=g, device=device, dtype=torch.float64) * 2 - 1) * amp
    u = torch.sin(4.0 * yc)[None, :, None].expand(shp).contiguous() + noise()
    v = noise()
    w = noise()
    if wl.extra.get("inject_nan"):
        u[0, 0, 0] = float("nan")       # failure-isolation tests
    B = torch.zeros((6,) + shp, device=device, dtype=torch.float64)
    B[0] = 1.0
    B[3] = 1.0
    B[5] = 1.0
    return u, v, w, B


@dataclass
class Request:
    rid: int
    arrival: float
    wl: inputs.Workload
    grid: object = None
    remaining: int = 0
    admitted: float = -1.0
    finished: float = -1.0
    status: str = "pending"
    health: dict = None
    fields: dict = None
    nbytes: int = 0

    @property
    def latency(self):
        return self.finished - self.arrival


@dataclass
class _Group:
    stream: object
    active: list = field(default_factory=list)
    inflight: object = None      # (event, [(batch, k)])
    rr: int = 0                  # round-robin start


class Server:
    """budget_bytes: HBM budget for resident solves; max_active: slot cap; chunk: steps per
    launch; keep_fields: copy final u, v, w, p, B of each solve (tests)."""

    def __init__(self, budget_bytes=200e9, max_active=256, chunk=25, keep_fields=False,
                 device="cuda", max_batch=MAX_BATCH):
        import torch
        self.torch = torch
        self.budget = float(budget_bytes)
        self.max_active = int(max_active)
        self.chunk = int(chunk)
        self.keep_fields = keep_fields
        self.device = device
        self.max_batch = int(max_batch)
        self.admit_stream = torch.cuda.Stream(device=device)
        self.groups = {}
        self.used = 0
        self.peak_used = 0
        self.n_active = 0
        self.peak_active = 0
        self.launches = 0
        self.retiring = []           # (request, group, event, pinned health values, fields)

    # -- helpers --------------------------------------------------------------------------------
    def _prec(self, wl):
        return MIXED if wl.precision == "mixed" else FP64

    def _key(self, wl):
        return (wl.nx, wl.ny, wl.nz, wl.walls, self._prec(wl), wl.dt)

    def _admit(self, r: Request, now):
        torch = self.torch
        wl = r.wl
        key = self._key(wl)
        grp = self.groups.get(key)
        if grp is None:
            grp = self.groups[key] = _Group(stream=torch.cuda.Stream(device=self.device))
        with torch.cuda.stream(self.admit_stream):
            G = Grid(wl.nx, wl.ny, wl.nz, wl.lx, wl.ly, wl.lz, walls=wl.walls,
                     precision=self._prec(wl), stream=self.admit_stream, device=self.device)
            G.set_rheology(**wl.rheology())
            G.set_forcing(*wl.force)
            G.write_fields(*device_initial_fields(wl, self.device))
            if wl.project_initial:
                G.project()
            ev = torch.cuda.Event()
            ev.record(self.admit_stream)
        grp.stream.wait_event(ev)
        G.set_stream(grp.stream)
        r.grid = G
        r.remaining = wl.steps
        r.admitted = now
        r.status = "active"
        grp.active.append(r)
        self.used += r.nbytes
        self.n_active += 1
        self.peak_used = max(self.peak_used, self.used)
        self.peak_active = max(self.peak_active, self.n_active)

    def _begin_retire(self, r: Request, grp: _Group):
        """Take a finished solve out of its group and enqueue its health check (and field copy)
        on the group's stream behind an event; nothing waits here."""
        torch = self.torch
        G = r.grid
        grp.active.remove(r)
        hv = torch.empty(5, dtype=torch.float64, pin_memory=True)
        fields = None
        with torch.cuda.stream(grp.stream):
            hd = torch.empty(5, dtype=torch.float64, device=self.device)
            G.health_enqueue(hd)
            hv.copy_(hd, non_blocking=True)
            if self.keep_fields:
                dev = G.read_fields(("u", "v", "w", "p", "B"))
                fields = {k: torch.empty(t.shape, dtype=t.dtype, pin_memory=True)
                          for k, t in dev.items()}
                for k, t in dev.items():
                    fields[k].copy_(t, non_blocking=True)
                    t.record_stream(grp.stream)
            ev = torch.cuda.Event()
            ev.record(grp.stream)
        self.retiring.append((r, grp, ev, hv, fields))

    def _finish_retire(self, item, now):
        """The solve's event has passed: record its result, free its workspace and budget."""
        r, grp, ev, hv, fields = item
        h = Grid.health_values(hv)
        r.health = h
        r.status = "error" if (h["nonfinite"] > 0) else "done"
        if fields is not None:
            r.fields = {k: t.numpy() for k, t in fields.items()}
        r.finished = now
        r.grid.close()
        r.grid = None
        self.used -= r.nbytes
        self.n_active -= 1

    def _launch(self, grp: _Group):
        torch = self.torch
        act = grp.active
        n = len(act)
        order = act[grp.rr % n:] + act[:grp.rr % n]
        grp.rr += self.max_batch
        work = []
        with torch.cuda.stream(grp.stream):
            for b0 in range(0, n, self.max_batch):
                batch = order[b0:b0 + self.max_batch]
                k = min(self.chunk, min(r.remaining for r in batch))
                step_batch([r.grid for r in batch], batch[0].wl.dt, k)
                self.launches += 1
                work.append((batch, k))
            ev = torch.cuda.Event()
            ev.record(grp.stream)
        grp.inflight = (ev, work)

    # -- main loop ------------------------------------------------------------------------------
    def run(self, requests, time_limit=None):
        """Serve `requests` (iterable of Request, any order).  Returns a stats dict."""
        torch = self.torch
        reqs = sorted(requests, key=lambda r: (r.arrival, r.rid))
        for r in reqs:
            r.nbytes = workspace_bytes(r.wl.nx, r.wl.ny, r.wl.nz, r.wl.walls, self._prec(r.wl))
            if r.nbytes > self.budget:
                raise ValueError(f"request {r.rid} alone exceeds the HBM budget")
        pending = deque(reqs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        done = []
        while pending or self.retiring or any(g.active for g in self.groups.values()):
            now = time.perf_counter() - t0
            if time_limit is not None and now > time_limit:
                raise TimeoutError("serving run exceeded its time limit")
            progressed = False
            # 1. completed chunks -> step accounting; finished solves start retiring
            for grp in self.groups.values():
                if grp.inflight is not None and grp.inflight[0].query():
                    for batch, k in grp.inflight[1]:
                        for r in batch:
                            r.remaining -= k
                    grp.inflight = None
                    for r in [r for r in grp.active if r.remaining <= 0]:
                        self._begin_retire(r, grp)
                    progressed = True
            # 2. retirements whose health check has completed free their workspace
            if self.retiring:
                still = []
                for item in self.retiring:
                    if item[2].query():
                        self._finish_retire(item, time.perf_counter() - t0)
                        done.append(item[0])
                        progressed = True
                    else:
                        still.append(item)
                self.retiring = still
            # 3. admission (FIFO: the head request blocks later ones until it fits)
            now = time.perf_counter() - t0
            while (pending and pending[0].arrival <= now and self.n_active < self.max_active
                   and self.used + pending[0].nbytes <= self.budget):
                self._admit(pending.popleft(), now)
                progressed = True
            # 4. launch the next chunk for every idle group
            for grp in self.groups.values():
                if grp.inflight is None and grp.active:
                    self._launch(grp)
                    progressed = True
            if not progressed:
                time.sleep(5e-5)
        makespan = time.perf_counter() - t0
        lat = np.array([r.latency for r in done]) if done else np.zeros(1)
        cell_steps = float(sum(r.wl.ncell * r.wl.steps for r in done))
        return {
            "requests": len(done),
            "errors": sum(1 for r in done if r.status != "done"),
            "makespan_s": makespan,
            "cell_steps_per_s": cell_steps / makespan,
            "p50_latency_s": float(np.percentile(lat, 50)),
            "p99_latency_s": float(np.percentile(lat, 99)),
            "mean_latency_s": float(lat.mean()),
            "peak_hbm_bytes": int(self.peak_used),
            "peak_active": int(self.peak_active),
            "launches": int(self.launches),
        }


def make_requests(n_requests=500, rate=None, seed=inputs.SEED, step_range=(100, 1000),
                  sizes=(32, 48, 64, 96, 128)):
    """Requests from the seeded sweep generator (Poisson arrivals at `rate`/s; None = burst)."""
    return [Request(rid=i, arrival=t, wl=wl) for i, (t, wl) in
            enumerate(inputs.serving_requests(n_requests, seed=seed, sizes=sizes, rate=rate,
                                              step_range=step_range))]
