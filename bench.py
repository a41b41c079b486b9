#!/usr/bin/env python3
"""Throughput of one full solver step (stress transport + momentum predictor + FFT pressure
projection) on one MI355X, in cell-steps per second.

Workload: triply periodic 128^3 box (2 pi), Saramito elastoviscoplastic fluid (Wi = 1, Bi = 0.5,
beta = 0.5, Re = 1000), Kolmogorov forcing f_x = sin 4y, initial u = sin 4y + seeded uniform noise
(1e-2), projected; dt = 1e-3.  FP64 is the headline; the mixed form (FP32 stress and momentum,
FP64 projection) is measured beside it.  Inputs are resident in HBM when timing starts.

Prints one JSON line (rank 0).  Also reports the dominant kernel's HBM roofline fraction from
per-kernel HIP-event timing inside the timed region, and the CPU oracle timed on this host.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

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


TRAFFIC_FILE = os.path.join(HERE, "profiles", "predictor_kolmogorov128_hbm_traffic.txt")
COUNTER_FILE = os.path.join(HERE, "profiles", "predictor_kolmogorov128_sq_counters.txt")
RHEOLOGY_TEXT = {"kolmogorov128": "Saramito Wi=1 Bi=0.5 beta=0.5 Re=1000",
                 "channel_fene_p": "FENE-P L^2=900 Wi=5 beta=0.9 Re=2000",
                 "channel_saramito": "Saramito Wi=2 Bi=0.2 beta=0.1 Re=5000"}
PRED_SOURCES = [os.path.join(HERE, "paper_1803_09563_amd", "csrc", f)
                for f in ("k_predictor_zm.hip", "weno.h")]


def pred_source_hash():
    """sha256[:16] of the predictor's sources (kernel file and its WENO header, concatenated)."""
    import hashlib
    h = hashlib.sha256()
    for f in PRED_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(precision="double"):
    """HBM bytes per predictor launch from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE summary,
    or None if the kernel source changed since the counters were taken (or no summary exists)."""
    import re
    try:
        text = open(TRAFFIC_FILE).read()
        sha = pred_source_hash()
    except OSError:
        return None
    m = re.search(r"sha256\[:16\] = ([0-9a-f]{16})", text)
    t = re.search(rf"traffic_bytes_per_launch_{precision} = (\d+)", text)
    if not m or not t or m.group(1) != sha:
        return None
    return int(t.group(1))


def measured_valu_busy():
    """Fraction of SIMD cycles the FP64 predictor keeps the vector ALU busy, from the committed
    rocprofv3 SQ-counter summary, or None if the kernel source changed since it was taken."""
    import re
    try:
        text = open(COUNTER_FILE).read()
        sha = pred_source_hash()
    except OSError:
        return None
    m = re.search(r"sha256\[:16\] = ([0-9a-f]{16})", text)
    t = re.search(r"valu_busy_double = ([0-9.]+)", text)
    if not m or not t or m.group(1) != sha:
        return None
    return float(t.group(1))


def _args():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--n", type=int, default=128, help="grid size (n^3)")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=0, help="oracle steps (0 = size to ~15 s)")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-rk3", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--serving-requests", type=int, default=500)
    ap.add_argument("--no-channel", action="store_true")
    ap.add_argument("--workload", default="kolmogorov128",
                    choices=("kolmogorov128", "channel_fene_p", "channel_saramito"),
                    help="main workload (the channel ones are for profiling runs)")
    ap.add_argument("--quiet", action="store_true")
    return ap.parse_args()


def _log(msg, quiet=False):
    if not quiet:
        print(f"[bench] {msg}", file=sys.stderr, flush=True)


def run_gpu(wl, precision, steps, warmup, quiet, integrator="ab2", adv=0, kappa=0.0, model=None):
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
    G.set_integrator(integrator)
    G.set_transport(adv, kappa)
    u, v, w, B = [torch.from_numpy(a).cuda() for a in inputs.initial_fields(wl)]
    G.write_fields(u, v, w, B)
    G.project()
    G.step(wl.dt, warmup)
    torch.cuda.synchronize()
    tag = f"{precision} {integrator} adv={adv} kappa={kappa} model={rh['model']}"
    _log(f"{tag}: warmup {warmup} steps done", quiet)

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
    _log(f"{tag}: timed {steps} steps in {ms:.2f} ms (wall {wall * 1e3:.2f} ms)", quiet)

    # per-kernel HIP-event timing on the library's stream, over a second timed region
    G.profile(True)
    G.step(wl.dt, steps)
    prof = G.profile_read()
    G.profile(False)
    h = G.health()
    G.close()
    return {"ms": ms, "wall_s": wall, "prof": prof, "health": h}


def d2d_copy_gbs(quiet, nbytes=1 << 30, reps=20):
    """Bandwidth of the runtime's device-to-device copy (torch copy_, hipMemcpy path) of nbytes,
    timed with events over reps copies; GB/s counts both directions.  A measured reference beside
    the published 8 TB/s, not a peak: the step's own correction kernel streams faster."""
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
    _log(f"device-to-device copy: {gbs:.0f} GB/s", quiet)
    del src, dst
    return gbs


def serving(n_requests, quiet):
    """Rheology sweep served with continuous batching: a burst run (all requests at t = 0) gives
    the saturated throughput; a Poisson run at 0.7 of that request rate gives latencies."""
    from paper_1803_09563_amd.serving import Server, make_requests
    burst = Server(budget_bytes=200e9).run(make_requests(n_requests, rate=None), time_limit=600)
    _log(f"serving burst: {burst}", quiet)
    rate = 0.7 * n_requests / burst["makespan_s"]
    pois = Server(budget_bytes=200e9).run(make_requests(n_requests, rate=rate), time_limit=600)
    _log(f"serving poisson: {pois}", quiet)
    return {"requests": n_requests, "precision": "mixed", "hbm_budget_bytes": 200e9,
            "saturated_cell_steps_per_s": burst["cell_steps_per_s"],
            "burst_makespan_s": burst["makespan_s"], "burst_p50_s": burst["p50_latency_s"],
            "burst_p99_s": burst["p99_latency_s"],
            "poisson_rate_per_s": rate, "p50_latency_s": pois["p50_latency_s"],
            "p99_latency_s": pois["p99_latency_s"], "cell_steps_per_s": pois["cell_steps_per_s"],
            "peak_active": pois["peak_active"], "peak_hbm_bytes": pois["peak_hbm_bytes"],
            "errors": burst["errors"] + pois["errors"]}


def cpu_baseline(wl, steps, quiet):
    import numpy as np
    import oracle
    from paper_1803_09563_amd import inputs

    g = oracle.Grid(wl.nx, wl.ny, wl.nz, wl.lx, wl.ly, wl.lz, walls=wl.walls)
    s = oracle.Solver(g, oracle.Rheology(**wl.rheology()), forcing=wl.force)
    s.write_fields(*inputs.initial_fields(wl))
    s.project()
    s.step(wl.dt, 1)                                   # warm-up (also the Euler start)
    if steps <= 0:
        t = time.perf_counter()
        s.step(wl.dt, 1)
        one = time.perf_counter() - t
        steps = max(1, min(100, int(15.0 / max(one, 1e-3))))
    t = time.perf_counter()
    s.step(wl.dt, steps)
    el = time.perf_counter() - t
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    _log(f"cpu oracle: {steps} steps in {el:.2f} s on {threads} threads", quiet)
    return {"value": wl.ncell * steps / el, "unit": "cell-steps/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{steps} FP64 steps of the same {wl.nx}x{wl.ny}x{wl.nz} workload after 1 warm-up step "
                      f"(C predictor on {threads} OpenMP threads + numpy FFT projection), "
                      f"{el:.1f} s"}


def main():
    a = _args()
    if a.gpus != 1:
        print(json.dumps({"error": "single-GPU benchmark: --gpus must be 1 (sharding the step over "
                          "several GPUs is not implemented)", "n_gpus": a.gpus}))
        sys.exit(2)
    import torch
    from paper_1803_09563_amd import inputs

    wl = {"kolmogorov128": lambda: inputs.kolmogorov_saramito(a.n),
          "channel_fene_p": inputs.channel_fene_p,
          "channel_saramito": inputs.channel_saramito}[a.workload]()
    res = {"fp64": run_gpu(wl, "fp64", a.steps, a.warmup, a.quiet)}
    if not a.no_mixed:
        res["mixed"] = run_gpu(wl, "mixed", a.steps, a.warmup, a.quiet)

    def rate(r):
        return wl.ncell * a.steps / (r["ms"] * 1e-3)

    f = res["fp64"]
    value = rate(f)
    copy_gbs = d2d_copy_gbs(a.quiet)
    ms_step = f["ms"] / a.steps
    pk = f["prof"]["predictor"]
    pred_ms = pk["ms"] / max(pk["launches"], 1)
    achieved = PRED_BYTES["fp64"] * wl.ncell / (pred_ms * 1e-3) / 1e9
    kernels = {}
    for prec, r in res.items():
        kernels[prec] = {k: round(v["ms"] / max(v["launches"], 1) * 1e3, 2)
                         for k, v in r["prof"].items() if v["launches"]}
    out = {
        "metric": "cell-steps/s (stress+FFT projection) FP64 vs mixed; p50/p99 sweep-solve latency",
        "value": value,
        "unit": "cell-steps/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded Kolmogorov-forced Saramito flow)",
        "config": {"workload": wl.name,
                   "grid": f"{wl.nx}x{wl.ny}x{wl.nz} " + ("channel" if wl.walls else "periodic"),
                   "rheology": RHEOLOGY_TEXT.get(a.workload, ""), "dt": wl.dt,
                   "precision": "fp64"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": (measured_traffic("double")
                                 if a.n == 128 and a.workload == "kolmogorov128" else None),
                     "valu_busy": (measured_valu_busy()
                                   if a.n == 128 and a.workload == "kolmogorov128" else None),
                     "kernel": "predictor (fused stress + momentum stencil)",
                     "bytes_per_cell": PRED_BYTES["fp64"], "avg_launch_us": pred_ms * 1e3},
        "step_hbm_frac": STEP_BYTES["fp64"] * value / 1e9 / HBM_PEAK_GBS,
        "d2d_copy_gbs": copy_gbs,
        "predictor_frac_of_d2d_copy": achieved / copy_gbs,
        "kernel_avg_us": kernels,
    }
    if "mixed" in res:
        m = res["mixed"]
        mv = rate(m)
        mp = m["prof"]["predictor"]
        mpred = mp["ms"] / max(mp["launches"], 1)
        out["mixed"] = {"value": mv, "ms_per_step": m["ms"] / a.steps, "speedup_vs_fp64": mv / value,
                        "predictor_avg_us": mpred * 1e3,
                        "predictor_hbm_frac": PRED_BYTES["mixed"] * wl.ncell / (mpred * 1e-3) / 1e9 / HBM_PEAK_GBS,
                        "step_hbm_frac": STEP_BYTES["mixed"] * mv / 1e9 / HBM_PEAK_GBS}
    if not a.no_rk3:
        # the paper's other integrator (Sec. 3.3.1): three substeps per step, same workload and dt
        rk = run_gpu(wl, "fp64", max(a.steps // 3, 1), a.warmup, a.quiet, integrator="rk3")
        n_rk = max(a.steps // 3, 1)
        sd = rk["prof"]["stress_div"]
        sd_ms = sd["ms"] / max(sd["launches"], 1)
        out["rk3"] = {"value": wl.ncell * n_rk / (rk["ms"] * 1e-3), "unit": "cell-steps/s",
                      "steps": n_rk, "ms_per_step": rk["ms"] / n_rk, "precision": "fp64",
                      "kernel_avg_us": {k: round(v["ms"] / max(v["launches"], 1) * 1e3, 2)
                                        for k, v in rk["prof"].items() if v["launches"]},
                      "stress_div_hbm_frac": STRESS_DIV_BYTES["fp64"] * wl.ncell / (sd_ms * 1e-3)
                      / 1e9 / HBM_PEAK_GBS}
    if not a.no_variants:
        # stress-transport variants on the same workload (FP64 AB2): HOUC5 advection, artificial
        # diffusion switched on (kappa > 0; the trigger test runs in every cell), Neo-Hookean
        out["variants"] = {}
        n_v = max(a.steps // 2, 1)
        for name, kw in (("houc5", dict(adv=1)), ("artificial_diffusion", dict(kappa=1e-3)),
                         ("neo_hookean", dict(model=3))):
            r = run_gpu(wl, "fp64", n_v, a.warmup, a.quiet, **kw)
            pk_v = r["prof"]["predictor"]
            out["variants"][name] = {"value": wl.ncell * n_v / (r["ms"] * 1e-3),
                                     "unit": "cell-steps/s", "steps": n_v,
                                     "predictor_avg_us": pk_v["ms"] / max(pk_v["launches"], 1) * 1e3}
    if not a.no_channel and a.workload == "kolmogorov128":
        # the channel workloads (periodic x and z, no-slip walls in y: FFT in x and z, tridiagonal
        # solve in y), FENE-P 256x128x128 in the mixed form and Saramito 512x256x256 in both forms
        out["channel"] = {}
        for wl_c, precs in ((inputs.channel_fene_p(), ("mixed",)),
                            (inputs.channel_saramito(), ("fp64", "mixed"))):
            d = {"workload": wl_c.name, "cells": wl_c.ncell}
            n_c = wl_c.steps if a.steps == 200 else a.steps
            for prec in precs:
                r = run_gpu(wl_c, prec, n_c, a.warmup, a.quiet)
                pk_c = r["prof"]["predictor"]
                pc_ms = pk_c["ms"] / max(pk_c["launches"], 1)
                d[prec] = {"value": wl_c.ncell * n_c / (r["ms"] * 1e-3), "unit": "cell-steps/s",
                           "steps": n_c, "ms_per_step": r["ms"] / n_c,
                           "predictor_hbm_frac": PRED_BYTES[prec] * wl_c.ncell / (pc_ms * 1e-3)
                           / 1e9 / HBM_PEAK_GBS,
                           "kernel_avg_us": {k: round(v["ms"] / max(v["launches"], 1) * 1e3, 2)
                                             for k, v in r["prof"].items() if v["launches"]}}
            out["channel"][wl_c.name] = d
    if not a.no_serving:
        out["serving"] = serving(a.serving_requests, a.quiet)
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, a.cpu_steps, a.quiet)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
