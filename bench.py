#!/usr/bin/env python3
"""Throughput of one full solver step (stress transport + momentum predictor + FFT/tridiagonal
pressure projection) on one MI355X, in cell-steps per second.

Headline workload: channel 512 x 256 x 256 (4 pi x 2 x 2 pi, periodic x and z, no-slip walls at
y = -1, +1), Saramito elastoviscoplastic fluid (Wi = 2, Bi = 0.2, beta = 0.1, Re = 5000), constant
pressure gradient, parabola + seeded 5 % noise projected to a divergence-free field, B = I,
dt = 1e-3.  FP64 is the headline `value`; the mixed form (FP32 stress transport and momentum, FP64
Poisson right-hand side, FFTs, tridiagonal solve and correction) is measured beside it.  Inputs are
resident in HBM when timing starts.

The JSON line (rank 0) also carries: the dominant kernel's HBM roofline fraction (per-kernel HIP
events inside a second timed region), per-field errors of both forms against the oracle and of the
mixed form against the FP64 GPU path after the configurations' step counts, the 128^3 periodic
Kolmogorov workload and the 256 x 128 x 128 FENE-P channel, the RK3 integrator, stress-transport
variants, the serving sweep, and the CPU oracle timed on this host on a short sample of the
headline workload.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
# algorithmic bytes per cell and step of the fused predictor: read u (3 FP64), B (6), RT (6),
# RU (3); write B (6), RT (6), u* (3 FP64), RU (3)
PRED_BYTES = {"fp64": 24 + 6 * 8 * 4 + 3 * 8 * 2 + 24, "mixed": 24 + 6 * 4 * 4 + 3 * 4 * 2 + 24}
# whole step: predictor + Poisson RHS/x-FFT (32) + 3 spectrum passes (48) + inverse x-FFT and
# correction (72)
STEP_BYTES = {k: v + 32 + 48 + 72 for k, v in PRED_BYTES.items()}
# RK3 stress divergence: read B^k (6), read and write u* (3 FP64 each way)
STRESS_DIV_BYTES = {"fp64": 6 * 8 + 48, "mixed": 6 * 4 + 48}

PRED_SOURCES = [os.path.join(HERE, "paper_1803_09563_amd", "csrc", f)
                for f in ("k_predictor_zm.hip", "weno.h")]
# rocprofv3 summaries of the predictor on the headline workload: HBM bytes per launch
# (FETCH_SIZE / WRITE_SIZE) and SQ counters, each tagged with the kernel sources' hash
TRAFFIC_FILE = os.path.join(HERE, "profiles", "predictor_channel512_hbm_traffic.txt")
COUNTER_FILE = os.path.join(HERE, "profiles", "predictor_channel512_sq_counters.txt")
RHEOLOGY_TEXT = {"kolmogorov128": "Saramito Wi=1 Bi=0.5 beta=0.5 Re=1000",
                 "channel_fene_p": "FENE-P L^2=900 Wi=5 beta=0.9 Re=2000",
                 "channel_saramito": "Saramito Wi=2 Bi=0.2 beta=0.1 Re=5000"}


def pred_source_hash():
    """sha256[:16] of the predictor's sources (kernel file and its WENO header, concatenated)."""
    import hashlib
    h = hashlib.sha256()
    for f in PRED_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _tagged(path, key, conv):
    """Value of `key = ...` in a committed profile summary, or None if the kernel sources changed
    since it was taken (or it is missing)."""
    import re
    try:
        text = open(path).read()
        sha = pred_source_hash()
    except OSError:
        return None
    m = re.search(r"sha256\[:16\] = ([0-9a-f]{16})", text)
    t = re.search(rf"{key} = ([0-9.]+)", text)
    if not m or not t or m.group(1) != sha:
        return None
    return conv(t.group(1))


def _args():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="channel_saramito",
                    choices=("channel_saramito", "channel_fene_p", "kolmogorov128"),
                    help="timed workload (the default is the headline; the others for profiling)")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=3, help="oracle steps after one warm-up step")
    ap.add_argument("--no-errors", action="store_true", help="skip the per-field error runs")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-rk3", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip the other workloads")
    ap.add_argument("--serving-requests", type=int, default=500)
    ap.add_argument("--quiet", action="store_true")
    return ap.parse_args()


QUIET = False


def _log(msg):
    if not QUIET:
        print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _workload(name):
    from paper_1803_09563_amd import inputs
    return {"kolmogorov128": lambda: inputs.kolmogorov_saramito(128),
            "channel_fene_p": inputs.channel_fene_p,
            "channel_saramito": inputs.channel_saramito}[name]()


def _grid(wl, precision, integrator="ab2", adv=0, kappa=0.0, model=None):
    import torch
    import paper_1803_09563_amd as evp
    from paper_1803_09563_amd import inputs
    prec = evp.MIXED if precision == "mixed" else evp.FP64
    G = evp.Grid(wl.nx, wl.ny, wl.nz, wl.lx, wl.ly, wl.lz, walls=wl.walls, precision=prec)
    rh = wl.rheology()
    if model is not None:
        rh["model"] = model
    G.set_rheology(**rh)
    G.set_forcing(*wl.force)
    if wl.walls:
        G.set_walls(*wl.wall_velocity)
    G.set_integrator(integrator)
    G.set_transport(adv, kappa)
    u, v, w, B = [torch.from_numpy(a).cuda() for a in inputs.initial_fields(wl)]
    G.write_fields(u, v, w, B)
    G.project()
    del u, v, w, B
    return G


def run_gpu(wl, precision, steps, warmup, **kw):
    """Warm-up, then `steps` steps timed with events on the library's stream, then a second
    `steps`-step region with per-kernel HIP events (evp_profile)."""
    import torch
    G = _grid(wl, precision, **kw)
    G.step(wl.dt, warmup)
    torch.cuda.synchronize()
    tag = f"{wl.name} {precision} {kw}"
    stream = G.stream
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    t0.record(stream)
    G.step(wl.dt, steps)
    t1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms = t0.elapsed_time(t1)
    _log(f"{tag}: timed {steps} steps in {ms:.2f} ms (wall {wall * 1e3:.2f} ms)")
    G.profile(True)
    G.step(wl.dt, steps)
    prof = G.profile_read()
    G.profile(False)
    h = G.health()
    G.close()
    del G
    torch.cuda.empty_cache()
    return {"ms": ms, "wall_s": wall, "prof": prof, "health": h}


def gpu_state_after(wl, precision, nsteps):
    """Fields (numpy) after nsteps steps from the projected initial state."""
    import torch
    G = _grid(wl, precision)
    G.step(wl.dt, nsteps)
    out = G.read_fields(("u", "v", "w", "p", "B"))
    torch.cuda.synchronize()
    st = {k: t.cpu().numpy() for k, t in out.items()}
    G.close()
    del G, out
    torch.cuda.empty_cache()
    return st


FLOOR = 1e-3


def field_errors(ref, got):
    """Per field, |x - x_ref|_inf / max(|x_ref|_inf, FLOOR * group scale), the groups being the
    velocity components and the six components of B - I (tau is G (B - I) for Saramito); p after
    removing the mean, against max |p_ref - mean| (floored at 1e-6 U^2)."""
    err = {}
    vmax = max(float(np.abs(ref[k]).max()) for k in "uvw")
    for k in "uvw":
        den = max(float(np.abs(ref[k]).max()), FLOOR * vmax, 1e-300)
        err[k] = float(np.abs(got[k] - ref[k]).max()) / den
    I6 = np.array([1.0, 0, 0, 1.0, 0, 1.0])[:, None, None, None]
    rb = ref["B"] - I6
    gb = got["B"] - I6
    bmax = float(np.abs(rb).max())
    for c, name in enumerate(("Bxx", "Bxy", "Bxz", "Byy", "Byz", "Bzz")):
        den = max(float(np.abs(rb[c]).max()), FLOOR * bmax, 1e-300)
        err[name] = float(np.abs(gb[c] - rb[c]).max()) / den
    rp = ref["p"] - ref["p"].mean()
    gp = got["p"] - got["p"].mean()
    err["p"] = float(np.abs(gp - rp).max()) / max(float(np.abs(rp).max()), 1e-6 * vmax ** 2, 1e-300)
    return err


def _summ(err):
    return {"max_velocity_stress": max(v for k, v in err.items() if k != "p"), "p": err["p"],
            "per_field": err}


def d2d_copy_gbs(nbytes=1 << 30, reps=20):
    """Bandwidth of the runtime's device-to-device copy (torch copy_) of nbytes, timed with events;
    GB/s counts both directions.  A measured reference beside the published 8 TB/s."""
    import torch
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    src.fill_(1)
    dst.copy_(src)
    torch.cuda.synchronize()
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(reps):
        dst.copy_(src)
    t1.record()
    torch.cuda.synchronize()
    gbs = 2.0 * nbytes * reps / (t0.elapsed_time(t1) * 1e-3) / 1e9
    _log(f"device-to-device copy: {gbs:.0f} GB/s")
    del src, dst
    torch.cuda.empty_cache()
    return gbs


def serving(n_requests):
    """Rheology sweep served with continuous batching: a burst run (all requests at t = 0) gives
    the saturated throughput; a Poisson run at 0.7 of that request rate gives latencies."""
    from paper_1803_09563_amd.serving import Server, make_requests
    burst = Server(budget_bytes=200e9).run(make_requests(n_requests, rate=None), time_limit=600)
    _log(f"serving burst: {burst}")
    rate = 0.7 * n_requests / burst["makespan_s"]
    pois = Server(budget_bytes=200e9).run(make_requests(n_requests, rate=rate), time_limit=600)
    _log(f"serving poisson: {pois}")
    return {"requests": n_requests, "precision": "mixed", "hbm_budget_bytes": 200e9,
            "saturated_cell_steps_per_s": burst["cell_steps_per_s"],
            "burst_makespan_s": burst["makespan_s"], "burst_p50_s": burst["p50_latency_s"],
            "burst_p99_s": burst["p99_latency_s"],
            "poisson_rate_per_s": rate, "p50_latency_s": pois["p50_latency_s"],
            "p99_latency_s": pois["p99_latency_s"], "cell_steps_per_s": pois["cell_steps_per_s"],
            "peak_active": pois["peak_active"], "peak_hbm_bytes": pois["peak_hbm_bytes"],
            "errors": burst["errors"] + pois["errors"]}


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def cpu_baseline(wl, steps):
    """The oracle (FP64 C predictor with OpenMP + numpy projection) on this host: projection of the
    initial state, one warm-up step (the Euler start), then `steps` timed steps.  Returns the
    baseline record and the oracle's final state (after 1 + steps steps)."""
    import oracle
    from paper_1803_09563_amd import inputs

    g = oracle.Grid(wl.nx, wl.ny, wl.nz, wl.lx, wl.ly, wl.lz, walls=wl.walls)
    s = oracle.Solver(g, oracle.Rheology(**wl.rheology()), forcing=wl.force,
                      walls_uv=wl.wall_velocity)
    s.write_fields(*inputs.initial_fields(wl))
    s.project()
    s.step(wl.dt, 1)
    _log(f"cpu oracle: warm-up step done, timing {steps} steps")
    t = time.perf_counter()
    s.step(wl.dt, steps)
    el = time.perf_counter() - t
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    _log(f"cpu oracle: {steps} steps in {el:.2f} s on {threads} threads")
    rec = {"value": wl.ncell * steps / el, "unit": "cell-steps/s", "cores": threads,
           "kind": "oracle", "nproc": os.cpu_count(), "cpu_model": _cpu_model(),
           "sample": f"{steps} FP64 steps of the same {wl.nx}x{wl.ny}x{wl.nz} workload after the "
                     f"initial projection and 1 warm-up step (C predictor on {threads} OpenMP "
                     f"threads + numpy FFT/Thomas projection), {el:.1f} s"}
    return rec, {"u": s.u, "v": s.v, "w": s.w, "p": s.p, "B": s.B}


def _kernel_us(prof):
    return {k: round(v["ms"] / max(v["launches"], 1) * 1e3, 2) for k, v in prof.items()
            if v["launches"]}


def _leg(wl, prec, steps, warmup, **kw):
    r = run_gpu(wl, prec, steps, warmup, **kw)
    pk = r["prof"]["predictor"]
    p_ms = pk["ms"] / max(pk["launches"], 1)
    return {"value": wl.ncell * steps / (r["ms"] * 1e-3), "unit": "cell-steps/s", "steps": steps,
            "ms_per_step": r["ms"] / steps, "predictor_avg_us": p_ms * 1e3,
            "predictor_hbm_frac": PRED_BYTES[prec] * wl.ncell / (p_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "step_hbm_frac": STEP_BYTES[prec] * wl.ncell * steps / (r["ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "kernel_avg_us": _kernel_us(r["prof"])}, r


def main():
    global QUIET
    a = _args()
    QUIET = a.quiet
    if a.gpus != 1:
        print(json.dumps({"error": "single-GPU benchmark: --gpus must be 1 (sharding the step over "
                          "several GPUs is not implemented; see the design notes for how it would "
                          "shard)", "n_gpus": a.gpus}))
        sys.exit(2)
    from paper_1803_09563_amd import inputs

    wl = _workload(a.workload)
    fp64, r64 = _leg(wl, "fp64", a.steps, a.warmup)
    value = fp64["value"]
    pred_ms = fp64["predictor_avg_us"] * 1e-3
    achieved = PRED_BYTES["fp64"] * wl.ncell / (pred_ms * 1e-3) / 1e9
    headline = a.workload == "channel_saramito"
    out = {
        "metric": "cell-steps/s (stress+FFT projection) FP64 vs mixed; p50/p99 sweep-solve latency",
        "value": value,
        "unit": "cell-steps/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": fp64["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded, shaped like the paper's workloads; no dataset)",
        "config": {"workload": wl.name,
                   "grid": f"{wl.nx}x{wl.ny}x{wl.nz} " + ("channel" if wl.walls else "periodic"),
                   "rheology": RHEOLOGY_TEXT.get(a.workload, ""), "dt": wl.dt,
                   "precision": "fp64"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": _tagged(TRAFFIC_FILE, "traffic_bytes_per_launch_double", int)
                     if headline else None,
                     "valu_busy": _tagged(COUNTER_FILE, "valu_busy_double", float)
                     if headline else None,
                     "kernel": "predictor (fused stress + momentum stencil; interior and wall "
                               "tile rows)",
                     "bytes_per_cell": PRED_BYTES["fp64"], "cells_per_launch": wl.ncell,
                     "avg_launch_us": pred_ms * 1e3},
        "step_hbm_frac": fp64["step_hbm_frac"],
        "kernel_avg_us": {"fp64": fp64["kernel_avg_us"]},
    }
    if not a.no_mixed:
        mixed, _ = _leg(wl, "mixed", a.steps, a.warmup)
        mixed["speedup_vs_fp64"] = mixed["value"] / value
        out["mixed"] = mixed
        out["kernel_avg_us"]["mixed"] = mixed.pop("kernel_avg_us")
    out["d2d_copy_gbs"] = d2d_copy_gbs()
    out["predictor_frac_of_d2d_copy"] = achieved / out["d2d_copy_gbs"]
    if not a.no_errors and not a.no_mixed:
        # mixed against the FP64 GPU path (itself pinned to the oracle) after the configurations'
        # step counts: 512 x 256 x 256 Saramito 200 steps, 256 x 128 x 128 FENE-P 500 steps
        fe = {}
        for wle in (inputs.channel_saramito(), inputs.channel_fene_p(precision="fp64")):
            ref = gpu_state_after(wle, "fp64", wle.steps)
            got = gpu_state_after(wle, "mixed", wle.steps)
            fe[f"mixed_vs_fp64_gpu_{wle.name}_{wle.steps}_steps"] = _summ(field_errors(ref, got))
            del ref, got
            _log(f"field errors mixed vs FP64 GPU, {wle.name}: "
                 f"{fe[f'mixed_vs_fp64_gpu_{wle.name}_{wle.steps}_steps']['max_velocity_stress']:.2e}")
        out["field_errors"] = fe
    if not a.no_extra and headline:
        out["extra"] = {}
        for name, wle, precs in (("kolmogorov128", inputs.kolmogorov_saramito(128), ("fp64", "mixed")),
                                 ("channel_fene_p", inputs.channel_fene_p(), ("mixed",))):
            d = {"workload": wle.name, "cells": wle.ncell, "rheology": RHEOLOGY_TEXT[name]}
            for prec in precs:
                d[prec], _ = _leg(wle, prec, a.steps, a.warmup)
            out["extra"][name] = d
    if not a.no_rk3:
        # the paper's other integrator (Sec. 3.3.1): three substeps per step, same workload and dt
        n_rk = max(a.steps // 3, 1)
        rk = run_gpu(wl, "fp64", n_rk, a.warmup, integrator="rk3")
        sd = rk["prof"]["stress_div"]
        sd_ms = sd["ms"] / max(sd["launches"], 1)
        out["rk3"] = {"value": wl.ncell * n_rk / (rk["ms"] * 1e-3), "unit": "cell-steps/s",
                      "steps": n_rk, "ms_per_step": rk["ms"] / n_rk, "precision": "fp64",
                      "kernel_avg_us": _kernel_us(rk["prof"]),
                      "stress_div_hbm_frac": STRESS_DIV_BYTES["fp64"] * wl.ncell / (sd_ms * 1e-3)
                      / 1e9 / HBM_PEAK_GBS}
    if not a.no_variants:
        # stress-transport variants on the same workload (FP64 AB2): HOUC5 advection, artificial
        # diffusion switched on (kappa > 0; the trigger test runs in every cell), Neo-Hookean
        out["variants"] = {}
        n_v = max(a.steps // 2, 1)
        for name, kw in (("houc5", dict(adv=1)), ("artificial_diffusion", dict(kappa=1e-3)),
                         ("neo_hookean", dict(model=3))):
            r = run_gpu(wl, "fp64", n_v, a.warmup, **kw)
            pk_v = r["prof"]["predictor"]
            out["variants"][name] = {"value": wl.ncell * n_v / (r["ms"] * 1e-3),
                                     "unit": "cell-steps/s", "steps": n_v,
                                     "predictor_avg_us": pk_v["ms"] / max(pk_v["launches"], 1) * 1e3}
    if not a.no_serving:
        out["serving"] = serving(a.serving_requests)
    if not a.no_cpu_baseline:
        rec, ref = cpu_baseline(wl, a.cpu_steps)
        out["cpu_baseline"] = rec
        if not a.no_errors:
            n = 1 + a.cpu_steps
            fe = out.setdefault("field_errors", {})
            for prec in ("fp64", "mixed") if not a.no_mixed else ("fp64",):
                got = gpu_state_after(wl, prec, n)
                fe[f"{prec}_vs_oracle_{wl.name}_{n}_steps"] = _summ(field_errors(ref, got))
                del got
                _log(f"field errors {prec} vs oracle after {n} steps: "
                     f"{fe[f'{prec}_vs_oracle_{wl.name}_{n}_steps']['max_velocity_stress']:.2e}")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
