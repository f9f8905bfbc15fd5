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
import hashlib
import importlib.util
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "events/s for gg→tt̄gg (FP64 vs FP32+Kahan at stated error); % vector roofline"
PEAK_FP64_TFLOPS = 78.6      # MI355X vector FP64 (256 CUs x 2.4 GHz x 128 flop/clk)
PEAK_FP32_TFLOPS = 157.3     # MI355X vector FP32 (packed)

# Per-event flops outside |M|^2 (Philox is integer work): VEGAS map 5 D,
# kinematics, phase space with massive rescaling (about 40 per particle, plus
# 10 per particle per Newton step), cuts (about 50), two PDF evaluations
# (about 170 each), weight and accumulation (about 25); estimated from the
# kernel source.
OTHER_FLOPS = {2: 420, 3: 720, 4: 1030}

WORKLOADS = {
    "ttx": dict(process="gg_ttx", n_g=2, cuts={}, events=1_000_000),
    "ttxg": dict(process="gg_ttxg", n_g=3, cuts=dict(ptmin_g=20.0, etamax_g=2.5), events=10_000_000),
    "ttxgg": dict(process="gg_ttxgg", n_g=4, cuts=dict(ptmin_g=20.0, drmin_gg=0.4), events=10_000_000),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def me_flops(n_g, colour="full"):
    path = os.path.join(ROOT, "paper_2106_10279_amd", "csrc", "gen_amplitudes.py")
    spec = importlib.util.spec_from_file_location("gen_amplitudes", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod.flop_count(n_g, colour)["per_event"]


def timed_run(api, torch, proc, pdf, n_events, steps, warmup, precision, seed, colour="full"):
    if warmup > 0:
        api.integrate(proc, 13000.0, pdf, n_events, warmup, seed, precision=precision,
                      keep_weights=False, colour=colour)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    r = api.integrate(proc, 13000.0, pdf, n_events, steps, seed, precision=precision,
                      keep_weights=False, profile=True, start_iter=warmup, colour=colour)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return r, wall, e0.elapsed_time(e1) / 1e3


# Sources of the event kernel; HBM traffic measured with rocprofv3 counters is
# reported only while their hash matches the one recorded with the counters.
KERNEL_SOURCES = ("mf_kernels.hpp", "mf_device.hpp", "gen_amplitudes.py", "mf_unweight.hpp")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "amp_kernel_gg_ttxgg_traffic.txt")


def kernel_source_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2106_10279_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(key):
    """HBM bytes per launch (FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0, scaled by the
    copy-kernel calibration) for `key`, or None if not measured for the current
    kernel sources."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    vals = {}
    with open(TRAFFIC_FILE) as fh:
        for line in fh:
            if "=" in line and not line.lstrip().startswith("#"):
                k, v = line.split("=", 1)
                vals[k.strip()] = v.strip()
    if vals.get("source_hash") != kernel_source_hash() or key not in vals:
        return None
    return int(float(vals[key]))


def roofline(n_g, me_flops_event, other_flops_event, n_events, r, peak, traffic_key=None):
    """Roofline of the dominant kernel over the timed iterations, from its
    HIP-event durations recorded on the library's stream.  For n_g >= 3 that
    is amp_kernel (helicity amplitudes and colour sum of the events that pass
    threshold and cuts); for n_g = 2 the fused event kernel (amplitudes of the
    passing events plus phase space, PDF and accumulation of all events)."""
    launches = len(r.iter_event_ms) * (r.n_batches if n_g >= 3 else 1)
    n_pass = float(np.sum(r.iter_pass))
    if n_g >= 3:
        t_s = float(np.sum(r.iter_amp_ms)) / 1e3
        flops = n_pass * me_flops_event
        kernel = "amp_kernel"
    else:
        t_s = float(np.sum(r.iter_event_ms)) / 1e3
        flops = n_pass * me_flops_event + len(r.iter_event_ms) * n_events * other_flops_event
        kernel = "event_kernel"
    achieved = flops / t_s / 1e12
    t_all = float(np.sum(r.iter_event_ms)) / 1e3
    all_flops = n_pass * me_flops_event + len(r.iter_event_ms) * n_events * other_flops_event
    return {"bound": "alu", "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
            "frac": round(achieved / peak, 4),
            "traffic": measured_traffic(traffic_key) if traffic_key else None,
            "kernel": kernel, "launches": launches, "avg_launch_ms": round(t_s * 1e3 / launches, 3),
            "flops_per_passing_event": me_flops_event if n_g >= 3 else me_flops_event + other_flops_event,
            "pass_fraction": round(n_pass / (len(r.iter_event_ms) * n_events), 4),
            "per_event_kernels": {"ms_per_iteration": round(t_all * 1e3 / len(r.iter_event_ms), 3),
                                  "achieved_tflops": round(all_flops / t_all / 1e12, 3)}}


def precision_error(api, torch, proc, pdf, grid, n, seed):
    """FP32 amplitudes vs FP64 on the same n events and grid, on the device."""
    w64 = api.evaluate_weights(proc, 13000.0, pdf, n, seed=seed, it=0, grid=grid)
    w32 = api.evaluate_weights(proc, 13000.0, pdf, n, seed=seed, it=0, grid=grid,
                               precision="fp32_kahan")
    nz = w64 != 0
    rel = ((w32[nz] - w64[nz]) / w64[nz]).abs()
    srt = torch.sort(rel).values
    k = srt.numel()
    I64 = w64.sum().item()
    I32 = w32.sum().item()
    out = {"events": n, "nonzero": k, "event_rel_max": float(srt[-1]),
           "event_rel_p999": float(srt[min(k - 1, int(0.999 * k))]),
           "event_rel_median": float(srt[k // 2]), "integral_rel": abs(I32 / I64 - 1.0)}
    del w64, w32, rel, srt
    torch.cuda.empty_cache()
    return out


def adjoint_run(api, torch, pdf, n_events, n_iter, seed):
    """g g -> t tbar forward integration plus the adjoint (d sigma / d m_t,
    d sigma / d alpha_s); events/s counts forward + adjoint per event."""
    proc = api.Process("gg_ttx")
    api.integrate_grad(proc, 13000.0, pdf, n_events, 1, seed)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r, g = api.integrate_grad(proc, 13000.0, pdf, n_events, n_iter, seed)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return {"workload": f"gg_ttx LO + adjoint, {n_events} events x {n_iter} iterations, FP64",
            "value": round(n_events * n_iter / dt, 2), "unit": "events/s (forward + adjoint)",
            "sigma_pb": r.sigma, "sigma_err_pb": r.sigma_err, "dsigma_dmt_pb_per_gev": g.dsigma_dmt,
            "dsigma_dalphas_pb": g.dsigma_dalphas}


PEAK_HBM_GBS = 8000.0        # MI355X HBM3E


def unweight_run(api, torch, proc, pdf, grid, n_events, seed, n_f, reps=5):
    """Hit-or-miss unweighting (mf_unweight: count, write and record kernels)
    of one extra iteration's weights on the refined grid.  The call is timed
    with HIP events on its stream (median of reps); the roofline is that of its
    dominant kernel, the count pass (Philox uniform and decision per event),
    from the library's HIP-event timing of that kernel in further calls with
    profiling on: algorithmic bytes are the 8-byte weight of every event."""
    it = 1000
    r = api.integrate(proc, 13000.0, pdf, n_events, 1, seed, grid_in=grid, start_iter=it,
                      keep_weights=True)
    w = r.weights
    first = api.unweight(proc, 13000.0, w, r.w_max, seed, it, grid=r.grid_last)
    cap = first.n_kept
    stream = torch.cuda.current_stream()
    times, kms = [], []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        ev = api.unweight(proc, 13000.0, w, r.w_max, seed, it, grid=r.grid_last, capacity=cap)
        e1.record(stream)
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
        assert ev.n_kept == cap
    for _ in range(reps):
        ev = api.unweight(proc, 13000.0, w, r.w_max, seed, it, grid=r.grid_last, capacity=cap,
                          profile=True)
        kms.append(ev.kernel_ms)
    t = float(np.median(times)) / 1e3
    kms = np.array(kms)
    tc = float(kms[:, 0].mean()) / 1e3
    alg = n_events * 8
    achieved = alg / tc / 1e9
    del w, r, first, ev
    torch.cuda.empty_cache()
    return {"workload": f"hit-or-miss unweighting of {n_events} {proc.process} weights (one "
                        f"iteration on the refined grid) with lab-frame records",
            "value": round(n_events / t, 2), "unit": "events/s", "kept": cap,
            "efficiency": round(cap / n_events, 6), "ms_per_call": round(t * 1e3, 4),
            "kernel_ms": {"count": round(tc * 1e3, 4), "write": round(float(kms[:, 1].mean()), 4),
                          "record": round(float(kms[:, 2].mean()), 4)},
            "roofline": {"bound": "hbm", "achieved": round(achieved, 2), "peak": PEAK_HBM_GBS,
                         "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4),
                         "traffic": measured_traffic(f"unweight_count_{n_events}"),
                         "kernel": "unweight_count_kernel", "launches": reps,
                         "avg_launch_ms": round(tc * 1e3, 4), "bytes_per_launch": alg}}


def cpu_baseline(wl, pdf, budget_s):
    """The oracle on a bounded sample of the same workload: one iteration on a
    uniform grid, sized by two calibration runs to about budget_s seconds."""
    import oracle as O
    threads = max(1, min(os.cpu_count() or 1, 16))
    proc = O.Process(n_g=wl["n_g"], **wl["cuts"])
    n = 8 * threads
    rate = None
    for _ in range(2):
        t0 = time.perf_counter()
        O.integrate(proc, 13000.0, pdf, n, 1, 0, n_threads=threads, keep_weights=False)
        dt = time.perf_counter() - t0
        rate = n / max(dt, 1e-3)
        if dt > 0.3 * budget_s:
            break
        n = max(n, int(0.1 * budget_s * rate))
    n = max(n, int(budget_s * rate))
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
    ap.add_argument("--fp32-events", type=int, default=100_000_000,
                    help="events per iteration of the FP32-amplitude leg (gg_ttxgg at 1e8)")
    ap.add_argument("--fp32-steps", type=int, default=3)
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-unweight", action="store_true")
    ap.add_argument("--no-leading-colour", action="store_true")
    ap.add_argument("--no-colour-mc", action="store_true")
    ap.add_argument("--adjoint-events", type=int, default=10_000_000)
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
    f_me, f_other = me_flops(wl["n_g"]), OTHER_FLOPS[wl["n_g"]]

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
        "roofline": roofline(wl["n_g"], f_me, f_other, n_events, r64, PEAK_FP64_TFLOPS,
                             f"{args.workload}_fp64_{n_events}"),
        "result_pb": {"sigma": r64.sigma, "sigma_err": r64.sigma_err, "chi2_dof": r64.chi2_dof},
        "stream_timed_s": round(ev64, 4),
    }
    if not args.no_unweight:
        log(f"[bench] unweighting {n_events} weights")
        out["unweight"] = unweight_run(api, torch, proc, pdf, r64.grid, n_events, args.seed,
                                       wl["n_g"])
        log(f"[bench] unweighting done: {out['unweight']['ms_per_call']} ms per call, "
            f"{out['unweight']['kept']} kept")
    if not args.no_fp32:
        n32 = args.fp32_events if args.workload == "ttxgg" else n_events
        log(f"[bench] fp32 amplitudes with fp64 compensated accumulation: {args.warmup} warm-up + "
            f"{args.fp32_steps} timed iterations x {n32} events")
        r32, wall32, _ = timed_run(api, torch, proc, pdf, n32, args.fp32_steps, args.warmup,
                                   "fp32_kahan", args.seed)
        v32 = args.fp32_steps * n32 / wall32
        log(f"[bench] fp32 done: {v32:.4g} events/s; error vs fp64 on {n32} events")
        err = precision_error(api, torch, proc, pdf, r64.grid, n32, args.seed + 1)
        out["fp32_kahan"] = {
            "value": round(v32, 2), "unit": "events/s", "events_per_step": n32,
            "steps": args.fp32_steps, "ms_per_step": round(wall32 / args.fp32_steps * 1e3, 3),
            "roofline": roofline(wl["n_g"], f_me, f_other, n32, r32, PEAK_FP32_TFLOPS,
                                 f"{args.workload}_fp32_{n32}"),
            "sigma": r32.sigma, "sigma_err": r32.sigma_err,
            "error_vs_fp64": err,
            "note": "packed FP32 disabled at compile time: FP32 issues at the FP64 vector rate",
        }
        log(f"[bench] fp32 integral rel err {err['integral_rel']:.2e}, event max {err['event_rel_max']:.2e}")
    if not args.no_leading_colour:
        log(f"[bench] leading-colour approximation, fp64: {args.warmup} warm-up + {args.steps} timed "
            f"iterations x {n_events} events")
        rlc, walllc, _ = timed_run(api, torch, proc, pdf, n_events, args.steps, args.warmup, "fp64",
                                   args.seed, colour="leading")
        vlc = args.steps * n_events / walllc
        f_lc = me_flops(wl["n_g"], "leading")
        out["leading_colour"] = {
            "value": round(vlc, 2), "unit": "events/s", "events_per_step": n_events,
            "steps": args.steps, "ms_per_step": round(walllc / args.steps * 1e3, 3),
            "roofline": roofline(wl["n_g"], f_lc, f_other, n_events, rlc, PEAK_FP64_TFLOPS),
            "sigma": rlc.sigma, "sigma_err": rlc.sigma_err,
            "sigma_over_full_colour": rlc.sigma / r64.sigma,
            "note": "colour matrix replaced by (N^2-1) N^(n-1)/2^n times the identity: a different "
                    "integrand; same seed as the fp64 line, its VEGAS grid adapts to this integrand",
        }
        log(f"[bench] leading colour done: {vlc:.4g} events/s, sigma / sigma_full = "
            f"{rlc.sigma / r64.sigma:.4f}")
    legs = (("sampled", "colour_mc", "one colour assignment (adjoint indices) per event"),
            ("flow", "colour_flow", "one colour flow per event, drawn among the flows with a "
                                    "non-vanishing factor"))
    for mode, key, what in legs if not args.no_colour_mc and wl["n_g"] >= 3 else ():
        log(f"[bench] Monte Carlo over colours ({mode}), fp64: {args.warmup} warm-up + {args.steps} "
            f"timed iterations x {n_events} events")
        rmc, wallmc, _ = timed_run(api, torch, proc, pdf, n_events, args.steps, args.warmup, "fp64",
                                   args.seed, colour=mode)
        vmc = args.steps * n_events / wallmc
        f_mc = me_flops(wl["n_g"], mode)
        # the price of the sampling: per-event weight variance against the full colour
        # sum, on the same events and the same (final) grid of the fp64 line
        ws = api.integrate(proc, 13000.0, pdf, n_events, 1, args.seed, grid_in=r64.grid,
                           start_iter=args.warmup + args.steps, colour=mode).weights
        wf = api.integrate(proc, 13000.0, pdf, n_events, 1, args.seed, grid_in=r64.grid,
                           start_iter=args.warmup + args.steps).weights
        var_ratio = float(ws.var().item()) / float(wf.var().item())
        del ws, wf
        out[key] = {
            "value": round(vmc, 2), "unit": "events/s", "events_per_step": n_events,
            "steps": args.steps, "ms_per_step": round(wallmc / args.steps * 1e3, 3),
            "roofline": roofline(wl["n_g"], f_mc, f_other, n_events, rmc, PEAK_FP64_TFLOPS),
            "sigma": rmc.sigma, "sigma_err": rmc.sigma_err,
            "weight_variance_vs_full_colour": round(var_ratio, 3),
            "full_colour_equivalent_events_per_s": round(vmc / var_ratio, 2),
            "note": what + " (Philox block 0x80000001), unbiased; the variance ratio is the factor "
                    "on events needed for the full-colour error",
        }
        log(f"[bench] colour Monte Carlo ({mode}) done: {vmc:.4g} events/s, weight variance "
            f"x{var_ratio:.2f}")
    if not args.no_adjoint:
        log(f"[bench] adjoint: gg_ttx forward + gradient, {args.adjoint_events} events x 3 iterations")
        out["adjoint"] = adjoint_run(api, torch, pdf, args.adjoint_events, 3, args.seed)
        log(f"[bench] adjoint done: {out['adjoint']['value']:.4g} events/s")
    if not args.no_cpu_baseline:
        log(f"[bench] CPU oracle baseline (~{args.cpu_seconds:.0f} s)")
        out["cpu_baseline"] = cpu_baseline(wl, pdf, args.cpu_seconds)
        log(f"[bench] cpu done: {out['cpu_baseline']['value']} events/s")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
