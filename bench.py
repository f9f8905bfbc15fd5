#!/usr/bin/env python3
"""Throughput of the per-event MadFlow integrand on one MI355X.

A step is one VEGAS iteration over one batch of events: Philox uniforms,
VEGAS map, phase space, cuts, PDFs, colour- and helicity-summed |M|^2,
weights, compensated sums, histogram, reduction and grid refinement.  The
default workload is g g -> t tbar g g at 13 TeV with pT > 20 GeV and
Delta R > 0.4 on the gluons, 1e7 events per iteration, FP64.

Prints one JSON line with events/s, the roofline figure of the event kernel
(algorithmic flops over its HIP-event-timed duration), the FP32-amplitude
form with its measured error, and the CPU oracle timed on the host cores.
"""
from __future__ import annotations

import argparse
import importlib.util
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "events/s for gg→tt̄gg (FP64 vs FP32+Kahan at stated error); % vector roofline"
PEAK_FP64_TFLOPS = 78.6      # MI355X vector FP64 (256 CUs x 2.4 GHz x 128 flop/clk)
PEAK_FP32_TFLOPS = 157.3     # MI355X vector FP32 (packed)

# Per-event flops outside |M|^2 (Philox is integer work): VEGAS map 5 D,
# kinematics, phase space with massive rescaling, cuts, two PDF evaluations,
# weight and accumulation.  Counted from the kernel source, see the design doc.
OTHER_FLOPS = {2: 420, 3: 720, 4: 1030}

WORKLOADS = {
    "ttx": dict(process="gg_ttx", n_g=2, cuts={}, events=1_000_000),
    "ttxg": dict(process="gg_ttxg", n_g=3, cuts=dict(ptmin_g=20.0, etamax_g=2.5), events=10_000_000),
    "ttxgg": dict(process="gg_ttxgg", n_g=4, cuts=dict(ptmin_g=20.0, drmin_gg=0.4), events=10_000_000),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def me_flops(n_g):
    path = os.path.join(ROOT, "paper_2106_10279_amd", "csrc", "gen_amplitudes.py")
    spec = importlib.util.spec_from_file_location("gen_amplitudes", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod.flop_count(n_g)["per_event"]


def timed_run(api, torch, proc, pdf, n_events, steps, warmup, precision, seed):
    if warmup > 0:
        api.integrate(proc, 13000.0, pdf, n_events, warmup, seed, precision=precision,
                      keep_weights=False)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    r = api.integrate(proc, 13000.0, pdf, n_events, steps, seed, precision=precision,
                      keep_weights=False, profile=True, start_iter=warmup)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return r, wall, e0.elapsed_time(e1) / 1e3


def roofline(flops_per_event, n_events, kernel_ms_total, steps, peak):
    per_launch_s = kernel_ms_total / steps / 1e3
    achieved = flops_per_event * n_events / per_launch_s / 1e12
    return {"bound": "alu", "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
            "frac": round(achieved / peak, 4), "traffic": None,
            "kernel": "event_kernel", "avg_launch_ms": round(kernel_ms_total / steps, 3),
            "flops_per_event": flops_per_event}


def precision_error(api, torch, proc, pdf, grid, n, seed):
    """FP32 amplitudes vs FP64 on the same events and grid."""
    w64 = api.evaluate_weights(proc, 13000.0, pdf, n, seed=seed, it=0, grid=grid)
    w32 = api.evaluate_weights(proc, 13000.0, pdf, n, seed=seed, it=0, grid=grid,
                               precision="fp32_kahan")
    w64 = w64.cpu().double()
    w32 = w32.cpu().double()
    nz = w64 != 0
    rel = ((w32[nz] - w64[nz]) / w64[nz]).abs()
    I64 = w64.sum().item()
    I32 = w32.sum().item()
    return {"events": n, "event_rel_max": float(rel.max()),
            "event_rel_p999": float(rel.quantile(0.999)) if rel.numel() < 2**24 else None,
            "event_rel_median": float(rel.median()),
            "integral_rel": abs(I32 / I64 - 1.0)}


def cpu_baseline(wl, pdf, budget_s):
    import oracle as O
    threads = max(1, min(os.cpu_count() or 1, 16))
    proc = O.Process(n_g=wl["n_g"], **wl["cuts"])
    n0 = 8 * threads
    t0 = time.perf_counter()
    O.integrate(proc, 13000.0, pdf, n0, 1, 0, n_threads=threads, keep_weights=False)
    dt = time.perf_counter() - t0
    n = max(n0, int(n0 * budget_s / max(dt, 1e-3)))
    t0 = time.perf_counter()
    O.integrate(proc, 13000.0, pdf, n, 1, 0, n_threads=threads, keep_weights=False)
    dt = time.perf_counter() - t0
    return {"value": round(n / dt, 2), "unit": "events/s", "cores": threads, "kind": "oracle",
            "sample": f"1 iteration x {n} events of {wl['process']} (same cuts, uniform grid), "
                      f"{dt:.1f} s on {threads} host threads"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="ttxgg", choices=sorted(WORKLOADS))
    ap.add_argument("--events", type=int, default=None)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="only run a plain device-to-device copy of this many bytes (3 times), "
                         "the reference kernel for scaling rocprofv3 FETCH_SIZE / WRITE_SIZE")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {args.gpus} is not supported "
              "(multi-GPU event sharding is a design note only)", file=sys.stderr)
        sys.exit(2)

    import torch
    if args.copy_bytes:
        n = args.copy_bytes // 8
        src = torch.arange(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": 8 * n, "launches": 3}), flush=True)
        return
    import workloads as W
    from paper_2106_10279_amd import api

    wl = WORKLOADS[args.workload]
    n_events = args.events or wl["events"]
    pdf = W.synthetic_pdf()
    proc = api.Process(wl["process"], **wl["cuts"])
    flops = me_flops(wl["n_g"]) + OTHER_FLOPS[wl["n_g"]]

    log(f"[bench] {wl['process']} fp64: {args.warmup} warm-up + {args.steps} timed iterations "
        f"x {n_events} events")
    r64, wall64, ev64 = timed_run(api, torch, proc, pdf, n_events, args.steps, args.warmup, "fp64",
                                  args.seed)
    value = args.steps * n_events / wall64
    log(f"[bench] fp64 done: {value:.4g} events/s, sigma = {r64.sigma:.6g} +- {r64.sigma_err:.3g} pb")
    out = {
        "metric": METRIC, "value": round(value, 2), "unit": "events/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(wall64 / args.steps * 1e3, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{wl['process']} LO at sqrt(s) = 13 TeV, {n_events} events per "
                               f"iteration, VEGAS 50 bins/dim, synthetic gluon PDF grid 100 x 50",
                   "process": wl["process"], "events_per_step": n_events, "cuts": wl["cuts"],
                   "sqrt_s_gev": 13000.0, "m_top": 173.0, "w_top": 1.5, "alpha_s": 0.118,
                   "seed": args.seed, "amplitude_precision": "fp64"},
        "roofline": roofline(flops, n_events, r64.event_kernel_ms, args.steps, PEAK_FP64_TFLOPS),
        "result_pb": {"sigma": r64.sigma, "sigma_err": r64.sigma_err, "chi2_dof": r64.chi2_dof},
        "stream_timed_s": round(ev64, 4),
    }
    if not args.no_fp32:
        log("[bench] fp32 amplitudes with fp64 compensated accumulation")
        r32, wall32, _ = timed_run(api, torch, proc, pdf, n_events, args.steps, args.warmup,
                                   "fp32_kahan", args.seed)
        v32 = args.steps * n_events / wall32
        err = precision_error(api, torch, proc, pdf, r64.grid, min(n_events, 1 << 20), args.seed + 1)
        out["fp32_kahan"] = {
            "value": round(v32, 2), "unit": "events/s",
            "ms_per_step": round(wall32 / args.steps * 1e3, 3),
            "roofline": roofline(flops, n_events, r32.event_kernel_ms, args.steps, PEAK_FP32_TFLOPS),
            "sigma": r32.sigma, "sigma_err": r32.sigma_err, "error_vs_fp64": err,
        }
        log(f"[bench] fp32 done: {v32:.4g} events/s, integral rel err {err['integral_rel']:.2e}")
    if not args.no_cpu_baseline:
        log(f"[bench] CPU oracle baseline (~{args.cpu_seconds:.0f} s)")
        out["cpu_baseline"] = cpu_baseline(wl, pdf, args.cpu_seconds)
        log(f"[bench] cpu done: {out['cpu_baseline']['value']} events/s")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
