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
OTHER_FLOPS = {2: 420, 3: 720, 4: 1030, 5: 1340}
# p p -> t tbar adds the q qbar channel to the amplitude kernel: on each of the
# 8 helicity lanes with a non-vanishing beam current, two massive spinors (14
# each), the top bilinear (64) and its contraction with the beam current and
# |.|^2 / s (11); then the 16-lane sum.
QQBAR_FLOPS = 8 * (2 * 14 + 64 + 11) + 15
# p p -> t tbar g, helicity-recycled: per event 8 lanes each build the beam
# chains X1, X2 of one beam combination (two massless spinors 28, the gluon
# polarisation 13, s12 11, two chains of 205, scaling 16) and the top chains
# Y3, Y4 of one top combination (two massive spinors 28, polarisation 13, two
# chains of 232 with the mass term and the Breit-Wigner factor, scaling 48,
# s 2), 4 + 4 of them the currents J and K (64 each); then 32 configurations
# of 312 (four chain contractions, the three-gluon term, the 5 x 5 colour
# form) after a per-lane setup of 47, and two 8-lane sums.
QQBAR_TTXG_FLOPS = 8 * (478 + 555) + 8 * 64 + 8 * 47 + 32 * 312 + 14
# p p -> t tbar g g, helicity-recycled, one wave per event.  First pass, 64
# lanes (line x spinor pair x attachment): the line's two spinors (28), the
# momenta (8), one vertex-and-propagator step from each end (2 x 187: slash
# 64, propagator 123), three bilinears (3 x 64); the attachment a gluon
# polarisation (13) on 32 lanes, the composite current (184) on 32; J after a
# three-gluon vertex (150) on 16.  Second pass, 64 lanes: spinors 28,
# polarisation 13, momenta 16, two steps 374, three bilinears 192.  Then 64
# configurations of 2495: reciprocals and momenta 40, the current products
# 86, the 38 terms' contractions and scalings (384 + 256 + 480 + 132 + 242 +
# 34 + 128 + 147), their signed additions into the 11 colour-basis sums
# (112 x 2) and the colour sum with the 11 x 11 Gram matrix (342); two 32-lane
# sums.
QQBAR_TTXGG_FLOPS = (64 * 602 + 32 * 13 + 32 * 184 + 16 * 150) + 64 * 623 + 64 * 2495 + 62

WORKLOADS = {
    "ttx": dict(process="gg_ttx", n_g=2, cuts={}, events=1_000_000),
    "ttxg": dict(process="gg_ttxg", n_g=3, cuts=dict(ptmin_g=20.0, etamax_g=2.5), events=10_000_000),
    "ttxgg": dict(process="gg_ttxgg", n_g=4, cuts=dict(ptmin_g=20.0, drmin_gg=0.4), events=10_000_000),
    "ttxggg": dict(process="gg_ttxggg", n_g=5, cuts=dict(ptmin_g=20.0, drmin_gg=0.4), events=1_000_000),
    "ppttx": dict(process="pp_ttx", n_g=2, cuts={}, events=10_000_000, quarks=True),
    "ppttxg": dict(process="pp_ttxg", n_g=3, cuts=dict(ptmin_g=20.0, etamax_g=2.5), events=10_000_000, quarks=True),
    "ppttxgg": dict(process="pp_ttxgg", n_g=4, cuts=dict(ptmin_g=20.0, drmin_gg=0.4), events=1_000_000, quarks=True),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def me_flops(n_g, colour="full"):
    path = os.path.join(ROOT, "paper_2106_10279_amd", "csrc", "gen_amplitudes.py")
    spec = importlib.util.spec_from_file_location("gen_amplitudes", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod.flop_count(n_g, colour)["per_event"]


def timed_run(api, torch, proc, pdf, n_events, steps, warmup, precision, seed, colour="full", grid_in=None,
              keep_weights=True, helicity="sum"):
    """One warm-up call of `warmup` iterations, then one timed call of `steps`
    iterations (continuing the Philox iteration counter).  The last timed
    iteration stores its per-event weights into a buffer allocated before the
    timed region, as integrate returns them."""
    if warmup > 0:
        api.integrate(proc, 13000.0, pdf, n_events, warmup, seed, precision=precision,
                      keep_weights=False, colour=colour, grid_in=grid_in, helicity=helicity)
    w = torch.empty(n_events, dtype=torch.float64, device="cuda") if keep_weights else None
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    r = api.integrate(proc, 13000.0, pdf, n_events, steps, seed, precision=precision,
                      keep_weights=keep_weights, weights_out=w, profile=True, start_iter=warmup,
                      colour=colour, grid_in=grid_in, helicity=helicity)
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
    HIP-event durations recorded on the library's stream: amp_kernel, the
    helicity amplitudes and colour sum of the events that pass threshold and
    cuts (mf_integrate runs phase space, amplitudes and accumulation as three
    kernels for every process)."""
    launches = len(r.iter_event_ms) * r.n_batches
    n_pass = float(np.sum(r.iter_pass))
    t_s = float(np.sum(r.iter_amp_ms)) / 1e3
    flops = n_pass * me_flops_event
    achieved = flops / t_s / 1e12
    t_all = float(np.sum(r.iter_event_ms)) / 1e3
    all_flops = n_pass * me_flops_event + len(r.iter_event_ms) * n_events * other_flops_event
    return {"bound": "alu", "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
            "frac": round(achieved / peak, 4),
            "traffic": measured_traffic(traffic_key) if traffic_key else None,
            "kernel": "amp_kernel", "launches": launches, "avg_launch_ms": round(t_s * 1e3 / launches, 3),
            "flops_per_passing_event": me_flops_event,
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


# Algorithmic flops per passing event of the adjoint kernel (grad_kernel_ttx),
# counted from its source like the forward code (+, -, x = 1, FMA = 2): per
# helicity configuration the forward amplitudes (624) and their reverse sweep
# (s-channel terms 480, top-exchange terms 748, amplitude adjoints 16), for 16
# configurations; the momentum-only quantities and their reverse (about 650);
# phase space, PDFs and weight forward and backward through the Newton root
# (about 1000).
ADJOINT_FLOPS = 16 * (624 + 480 + 748 + 16) + 650 + 1000


def adjoint_run(api, torch, pdf, n_events, n_iter, seed):
    """g g -> t tbar forward integration plus the adjoint (d sigma / d m_t,
    d sigma / d alpha_s); events/s counts forward + adjoint per event.  The
    roofline is that of the adjoint kernel from the library's HIP-event timing
    of each of its launches."""
    proc = api.Process("gg_ttx")
    api.integrate_grad(proc, 13000.0, pdf, n_events, 1, seed)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r, g = api.integrate_grad(proc, 13000.0, pdf, n_events, n_iter, seed, profile=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    t_grad = float(np.sum(g.iter_grad_ms)) / 1e3
    n_pass = float(np.sum(r.iter_pass))
    achieved = n_pass * ADJOINT_FLOPS / t_grad / 1e12
    return {"workload": f"gg_ttx LO + adjoint, {n_events} events x {n_iter} iterations, FP64",
            "value": round(n_events * n_iter / dt, 2), "unit": "events/s (forward + adjoint)",
            "sigma_pb": r.sigma, "sigma_err_pb": r.sigma_err, "dsigma_dmt_pb_per_gev": g.dsigma_dmt,
            "dsigma_dalphas_pb": g.dsigma_dalphas,
            "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP64_TFLOPS,
                         "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP64_TFLOPS, 4), "traffic": None,
                         "kernel": "grad_kernel_ttx", "launches": n_iter,
                         "avg_launch_ms": round(t_grad * 1e3 / n_iter, 3),
                         "flops_per_passing_event": ADJOINT_FLOPS,
                         "pass_fraction": round(n_pass / (n_iter * n_events), 4),
                         "forward_event_kernel_ms": round((float(np.sum(r.iter_event_ms)) - t_grad * 1e3)
                                                          / n_iter, 3)}}


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


def host_cpu():
    """CPU model and physical core count of this host (from /proc/cpuinfo)."""
    model, cores = None, set()
    phys = core = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                k, _, v = line.partition(":")
                k, v = k.strip(), v.strip()
                if k == "model name" and model is None:
                    model = v
                elif k == "physical id":
                    phys = v
                elif k == "core id":
                    core = v
                elif not k and phys is not None:
                    cores.add((phys, core))
                    phys = core = None
        if phys is not None:
            cores.add((phys, core))
    except OSError:
        pass
    return model, (len(cores) or None)


def usable_cpus():
    """Host CPUs this process may run on: its affinity mask, capped by a
    cgroup CPU quota when one is set."""
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    try:
        with open("/sys/fs/cgroup/cpu.max") as fh:
            quota, period = fh.read().split()[:2]
        if quota != "max":
            n = min(n, max(1, math.ceil(int(quota) / int(period))))
    except (OSError, ValueError):
        pass
    return max(1, n)


def cpu_baseline(wl, pdf, budget_s, grid=None, start_iter=0):
    """The oracle on a bounded sample of the same workload: one iteration on
    `grid` (the GPU run's adapted grid, so that the pass fraction matches the
    timed GPU iterations), on every host CPU the process may use, sized by
    calibration runs to about budget_s seconds."""
    import oracle as O
    threads = usable_cpus()
    proc = O.Process(n_g=wl["n_g"], **wl["cuts"])
    n = 8 * threads
    rate = None
    for _ in range(2):
        t0 = time.perf_counter()
        O.integrate(proc, 13000.0, pdf, n, 1, 0, n_threads=threads, keep_weights=False, grid=grid,
                    start_iter=start_iter)
        dt = time.perf_counter() - t0
        rate = n / max(dt, 1e-3)
        if dt > 0.3 * budget_s:
            break
        n = max(n, int(0.1 * budget_s * rate))
    n = max(n, int(budget_s * rate))
    t0 = time.perf_counter()
    o = O.integrate(proc, 13000.0, pdf, n, 1, 0, n_threads=threads, keep_weights=False, grid=grid,
                    start_iter=start_iter)
    dt = time.perf_counter() - t0
    model, phys = host_cpu()
    return {"value": round(n / dt, 2), "unit": "events/s", "cores": threads, "kind": "oracle",
            "per_thread": round(n / dt / threads, 2), "host_logical_cpus": os.cpu_count(),
            "host_physical_cores": phys, "cpu_model": model,
            "pass_fraction": round(o.n_pass / n, 4),
            "sample": f"1 iteration x {n} events of {wl['process']} (same cuts, "
                      f"{'the GPU run' + chr(39) + 's adapted grid' if grid is not None else 'uniform grid'}), "
                      f"{dt:.1f} s on {threads} threads, one per CPU this process may use (host: "
                      f"{os.cpu_count()} logical CPUs, {phys} physical cores, {model})"}


def config_leg(api, torch, name, n_events, n_iter, seeds, events_note=""):
    """A workload of the parity plan timed like the headline: per seed one
    warm-up iteration, then n_iter timed iterations; events/s over all seeds,
    with the roofline of its dominant kernel."""
    import workloads as W
    wl = WORKLOADS[name]
    pdf = W.synthetic_pdf(quarks=wl.get("quarks", False))
    proc = api.Process(wl["process"], **wl["cuts"])
    qq = {2: QQBAR_FLOPS, 3: QQBAR_TTXG_FLOPS, 4: QQBAR_TTXGG_FLOPS}[wl["n_g"]] if wl.get("quarks") else 0
    f_me, f_other = me_flops(wl["n_g"]) + qq, OTHER_FLOPS[wl["n_g"]]
    total, walls, sig, roof = 0, 0.0, [], []
    for seed in seeds:
        r, wall, _ = timed_run(api, torch, proc, pdf, n_events, n_iter, 1, "fp64", seed)
        total += n_events * n_iter
        walls += wall
        sig.append((r.sigma, r.sigma_err, r.chi2_dof))
        roof.append(roofline(wl["n_g"], f_me, f_other, n_events, r, PEAK_FP64_TFLOPS))
        del r
    torch.cuda.empty_cache()
    best = roof[-1]
    if len(roof) > 1:
        # durations and flops summed over the seeds
        t = sum(x["avg_launch_ms"] * x["launches"] for x in roof)
        fl = sum(x["achieved"] * x["avg_launch_ms"] * x["launches"] for x in roof)
        best = dict(roof[-1], achieved=round(fl / t, 3), frac=round(fl / t / PEAK_FP64_TFLOPS, 4),
                    launches=sum(x["launches"] for x in roof), avg_launch_ms=round(t / sum(x["launches"] for x in roof), 3),
                    pass_fraction=round(float(np.mean([x["pass_fraction"] for x in roof])), 4))
    return {"workload": f"{wl['process']} at 13 TeV, {n_events} events x {n_iter} iterations, seeds "
                        f"{list(seeds)}, FP64{events_note}",
            "value": round(total / walls, 2), "unit": "events/s", "ms_per_step": round(walls / (n_iter * len(seeds)) * 1e3, 3),
            "roofline": best, "sigma_pb": [s[0] for s in sig], "sigma_err_pb": [s[1] for s in sig],
            "chi2_dof": [s[2] for s in sig]}


def flop_record(n_g):
    path = os.path.join(ROOT, "paper_2106_10279_amd", "csrc", "gen_amplitudes.py")
    spec = importlib.util.spec_from_file_location("gen_amplitudes", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod.flop_count(n_g)


# Leading colour of t tbar g g g: each of the 120 x 128 partial amplitudes
# squared and added (4 flop) in place of the colour sum.
LC_FLOPS_NG5 = 120 * 128 * 4


def ttxggg_leg(api, torch, n_events, n_iter, precision, colour="full"):
    """g g -> t tbar g g g (five gluons): one warm-up iteration, then n_iter
    timed ones.  Two rooflines from the library's HIP-event timing of every
    launch: the amplitude kernel (object stages and partial amplitudes of the
    passing events, VALU) and the matrix-core colour sum (algorithmic flops of
    the symmetric quadratic form, 29040 per helicity configuration).  With
    the leading-colour sum the amplitude kernel squares and adds the
    amplitudes itself (LC_FLOPS_NG5 more per event) and a short kernel adds
    its 20 partial sums per event; there is no colour roofline."""
    import workloads as W
    wl = WORKLOADS["ttxggg"]
    pdf = W.synthetic_pdf()
    proc = api.Process(wl["process"], **wl["cuts"])
    c = flop_record(5)
    lc = colour == "leading"
    r, wall, _ = timed_run(api, torch, proc, pdf, n_events, n_iter, 1, precision, 0, colour=colour)
    n_pass = float(np.sum(r.iter_pass))
    launches = len(r.iter_event_ms) * r.n_batches
    t_amp = float(np.sum(r.iter_amp_ms)) / 1e3
    t_col = float(np.sum(r.iter_colour_ms)) / 1e3
    t_all = float(np.sum(r.iter_event_ms)) / 1e3
    f32 = precision != "fp64"
    vpeak = PEAK_FP32_TFLOPS if f32 else PEAK_FP64_TFLOPS
    mpeak = 157.3 if f32 else 78.6        # dense matrix-core FP32 / FP64
    amp_per_event = c["amplitudes"] + (LC_FLOPS_NG5 if lc else 0)
    amp_fl = n_pass * amp_per_event
    col_fl = n_pass * c["colour"]
    out = {"workload": f"gg_ttxggg at 13 TeV (pT > 20 GeV, Delta R > 0.4 on the gluons), {n_events} events x "
                       f"{n_iter} iterations, amplitudes {precision}"
                       + (", leading-colour sum" if lc else ""),
           "value": round(n_events * n_iter / wall, 2), "unit": "events/s",
           "ms_per_step": round(wall / n_iter * 1e3, 3), "sigma_pb": r.sigma, "sigma_err_pb": r.sigma_err,
           "pass_fraction": round(n_pass / (n_iter * n_events), 4), "batches_per_iteration": r.n_batches,
           "flops_per_passing_event": ({"amplitudes_and_squares": amp_per_event} if lc
                                       else {"amplitudes": c["amplitudes"], "colour": c["colour"]}),
           "roofline": {"bound": "alu", "achieved": round(amp_fl / t_amp / 1e12, 3), "peak": vpeak,
                        "unit": "TFLOP/s", "frac": round(amp_fl / t_amp / 1e12 / vpeak, 4), "traffic": None,
                        "kernel": "amp_kernel_ng5", "launches": launches,
                        "avg_launch_ms": round(t_amp * 1e3 / launches, 3)},
           "colour_roofline": None if lc else
                              {"bound": "mfma", "achieved": round(col_fl / t_col / 1e12, 3), "peak": mpeak,
                               "unit": "TFLOP/s", "frac": round(col_fl / t_col / 1e12 / mpeak, 4),
                               "traffic": None, "kernel": "colour_kernel_ng5", "launches": launches,
                               "avg_launch_ms": round(t_col * 1e3 / launches, 3)},
           "per_event_kernels_ms_per_iteration": round(t_all * 1e3 / n_iter, 3)}
    if lc:
        out["lc_sum_ms_per_launch"] = round(t_col * 1e3 / launches, 4)
    del r
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="ttxgg", choices=sorted(k for k in WORKLOADS if k not in ("ttxggg", "ppttx", "ppttxg", "ppttxgg")))
    ap.add_argument("--no-ttxggg", action="store_true", help="skip the g g -> t tbar g g g legs")
    ap.add_argument("--ttxggg-events", type=int, default=1_000_000)
    ap.add_argument("--ttxggg-only", action="store_true",
                    help="only the g g -> t tbar g g g legs (for profiling them alone)")
    ap.add_argument("--ttxggg-steps", type=int, default=3)
    ap.add_argument("--pp-only", action="store_true",
                    help="only the p p legs (for profiling them alone)")
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
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the legs of the other workloads (g g -> t tbar at 1e5 x 5 and 1e8 x 5, "
                         "g g -> t tbar g at 1e7 x 10 for seeds 0-4, p p -> t tbar at 1e8 x 5, "
                         "p p -> t tbar g at 1e7 x 10, p p -> t tbar g g at 1e6 x 3)")
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

    if args.pp_only:
        log("[bench] p p -> t tbar, 1e8 x 5; p p -> t tbar g, 1e7 x 10; p p -> t tbar g g, 1e6 x 3")
        print(json.dumps({"pptx_1e8x5": config_leg(api, torch, "ppttx", 100_000_000, 5, [0]),
                          "pptxg_1e7x10": config_leg(api, torch, "ppttxg", 10_000_000, 10, [0]),
                          "pptxgg_1e6x3": config_leg(api, torch, "ppttxgg", 1_000_000, 3, [0])}), flush=True)
        return
    if args.ttxggg_only:
        legs = {}
        for prec in ("fp64",) + (() if args.no_fp32 else ("fp32_kahan",)):
            log(f"[bench] g g -> t tbar g g g, {args.ttxggg_events} events x {args.ttxggg_steps} iterations, {prec}")
            legs[f"ttxggg_{prec}"] = ttxggg_leg(api, torch, args.ttxggg_events, args.ttxggg_steps, prec)
        log(f"[bench] g g -> t tbar g g g, leading colour, {args.ttxggg_events} events x {args.ttxggg_steps} "
            f"iterations, fp64")
        legs["ttxggg_lc_fp64"] = ttxggg_leg(api, torch, args.ttxggg_events, args.ttxggg_steps, "fp64", "leading")
        print(json.dumps(legs), flush=True)
        return

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
                                   "fp32_kahan", args.seed, grid_in=r64.grid)
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
            "note": "on the FP64 leg's adapted grid (same pass fraction); packed FP32 instructions "
                    "disabled at compile time, so the peak is the packed rate the code does not use",
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
    if not args.no_colour_mc:
        log(f"[bench] Monte Carlo over helicities, fp64: {args.warmup} warm-up + {args.steps} timed "
            f"iterations x {n_events} events")
        rh, wallh, _ = timed_run(api, torch, proc, pdf, n_events, args.steps, args.warmup, "fp64",
                                 args.seed, helicity="sampled")
        vh = args.steps * n_events / wallh
        ws = api.integrate(proc, 13000.0, pdf, n_events, 1, args.seed, grid_in=r64.grid,
                           start_iter=args.warmup + args.steps, helicity="sampled").weights
        wf = api.integrate(proc, 13000.0, pdf, n_events, 1, args.seed, grid_in=r64.grid,
                           start_iter=args.warmup + args.steps).weights
        var_ratio = float(ws.var().item()) / float(wf.var().item())
        del ws, wf
        out["helicity_mc"] = {
            "value": round(vh, 2), "unit": "events/s", "events_per_step": n_events,
            "steps": args.steps, "ms_per_step": round(wallh / args.steps * 1e3, 3),
            "roofline": roofline(wl["n_g"], f_me, f_other, n_events, rh, PEAK_FP64_TFLOPS),
            "sigma": rh.sigma, "sigma_err": rh.sigma_err,
            "weight_variance_vs_helicity_sum": round(var_ratio, 3),
            "helicity_sum_equivalent_events_per_s": round(vh / var_ratio, 2),
            "note": "one helicity configuration per event (Philox block 0x80000002), N_h |M_h|^2, "
                    "unbiased; every configuration is still evaluated by the cooperative kernel (one "
                    "lane each) and the drawn one kept, so the roofline counts the full per-event work",
        }
        log(f"[bench] helicity Monte Carlo done: {vh:.4g} events/s, weight variance x{var_ratio:.2f}")
    if not args.no_configs and args.workload == "ttxgg":
        log("[bench] g g -> t tbar, 1e5 x 5 and 1e8 x 5; g g -> t tbar g, 1e7 x 10, seeds 0-4; "
            "p p -> t tbar, 1e8 x 5; p p -> t tbar g, 1e7 x 10; p p -> t tbar g g, 1e6 x 3")
        out["ttx_1e5x5"] = config_leg(api, torch, "ttx", 100_000, 5, [0])
        out["ttx_1e8x5"] = config_leg(api, torch, "ttx", 100_000_000, 5, [0],
                                      " (the scaled run: 1e5 events do not fill 256 compute units)")
        out["ttxg_1e7x10"] = config_leg(api, torch, "ttxg", 10_000_000, 10, [0, 1, 2, 3, 4])
        out["pptx_1e8x5"] = config_leg(api, torch, "ppttx", 100_000_000, 5, [0],
                                       " (g g and the q qbar channels u ubar, ubar u, d dbar, dbar d; synthetic "
                                       "quark tables)")
        out["pptxg_1e7x10"] = config_leg(api, torch, "ppttxg", 10_000_000, 10, [0],
                                         " (g g and the q qbar channels; synthetic quark tables)")
        out["pptxgg_1e6x3"] = config_leg(api, torch, "ppttxgg", 1_000_000, 3, [0],
                                         " (g g and the q qbar channels; synthetic quark tables)")
        log(f"[bench] configs done: ttx {out['ttx_1e8x5']['value']:.4g}, ttxg {out['ttxg_1e7x10']['value']:.4g}, "
            f"pp ttx {out['pptx_1e8x5']['value']:.4g}, pp ttxg {out['pptxg_1e7x10']['value']:.4g}, "
            f"pp ttxgg {out['pptxgg_1e6x3']['value']:.4g} events/s")
    if not args.no_ttxggg and args.workload == "ttxgg":
        for prec in ("fp64", "fp32_kahan"):
            log(f"[bench] g g -> t tbar g g g, {args.ttxggg_events} events x {args.ttxggg_steps} iterations, {prec}")
            out[f"ttxggg_{prec}"] = ttxggg_leg(api, torch, args.ttxggg_events, args.ttxggg_steps, prec)
            log(f"[bench] ttxggg {prec} done: {out[f'ttxggg_{prec}']['value']:.4g} events/s")
        log(f"[bench] g g -> t tbar g g g, leading colour, fp64")
        out["ttxggg_lc_fp64"] = ttxggg_leg(api, torch, args.ttxggg_events, args.ttxggg_steps, "fp64", "leading")
        log(f"[bench] ttxggg leading colour done: {out['ttxggg_lc_fp64']['value']:.4g} events/s")
    if not args.no_adjoint:
        log(f"[bench] adjoint: gg_ttx forward + gradient, {args.adjoint_events} events x 3 iterations")
        out["adjoint"] = adjoint_run(api, torch, pdf, args.adjoint_events, 3, args.seed)
        log(f"[bench] adjoint done: {out['adjoint']['value']:.4g} events/s")
    if not args.no_cpu_baseline:
        log(f"[bench] CPU oracle baseline (~{args.cpu_seconds:.0f} s)")
        out["cpu_baseline"] = cpu_baseline(wl, pdf, args.cpu_seconds, grid=r64.grid,
                                           start_iter=args.warmup + args.steps)
        log(f"[bench] cpu done: {out['cpu_baseline']['value']} events/s")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
