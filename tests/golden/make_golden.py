"""Writes the oracle's reference integrations stored in this folder.

Only the CPU oracle (`oracle/`) and the input module (`workloads`) are used:
no value here comes from the GPU library.  Each file holds one oracle
integration at the reduced sizes of the parity plan:

* ``integration_gg_ttxg_1e6x10.json``: g g -> t tbar g, pT_g > 20 GeV,
  |eta_g| < 2.5, 1e6 events x 10 iterations, seed 0;
* ``integration_gg_ttxgg_1e5x10.json``: g g -> t tbar g g, pT > 20 GeV on
  both gluons, Delta R > 0.4, 1e5 events x 10 iterations, seed 0.

Stored: per-iteration I_j, V_j and passing-event counts, the combined sigma,
its error and chi^2/dof, w_max, the grid the last iteration ran on and the
final refined grid, the last histogram, and the last iteration's weights of
every 97th event with the oracle's flags (bit 3: near a cut edge, bit 4:
ill-conditioned PDF value).  The integration runs one iteration per call,
each resumed from the grid of the one before (bit-identical to one call of
all iterations), so that every iteration's counts and the grid of the last
iteration are known.  The oracle runs on 8 threads; the
thread count changes the grids only at the rounding level.

Rounding drift (``--drift``, added to an existing file): the same
integration with the oracle's sources built with fused multiply-add
contraction (``oracle/Makefile`` target libmfo_fma.so), a second correct FP64
implementation that differs only in rounding.  Bins do not move with the
grid, but every weight depends on its bins' widths through J_V, and the next
grid is refined from those weights, so after several iterations rounding
differences in the grid grow well above 1e-12.  Stored under "drift": the
largest relative differences of I_j, V_j, sigma, w_max and the last
histogram, and the largest absolute difference of the final grid, between
the two builds; and "w_max_event", the index of the last iteration's largest
weight (plain build).

Run from the repository root:  python tests/golden/make_golden.py [--drift] [name ...]
"""
from __future__ import annotations

import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle as O  # noqa: E402
import workloads as W  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
THREADS = 8
SAMPLE_STRIDE = 97

CASES = {
    "integration_gg_ttxg_1e6x10": dict(n_g=3, cuts=dict(ptmin_g=20.0, etamax_g=2.5),
                                       n_events=1_000_000, n_iter=10, seed=0),
    "integration_gg_ttxgg_1e5x10": dict(n_g=4, cuts=dict(ptmin_g=20.0, drmin_gg=0.4),
                                        n_events=100_000, n_iter=10, seed=0),
}


def run(name: str) -> dict:
    c = CASES[name]
    proc = O.Process(n_g=c["n_g"], **c["cuts"])
    pdf = W.synthetic_pdf()
    N, n_iter, seed = c["n_events"], c["n_iter"], c["seed"]
    t0 = time.time()
    # one iteration per call, each resumed from the previous grid: the same
    # result as one call of n_iter iterations, with every iteration's counts
    I, V, passes = [], [], []
    g = None
    for j in range(n_iter):
        grid_last = g
        r = O.integrate(proc, W.SQRT_S, pdf, N, 1, seed, n_threads=THREADS, grid=g,
                        start_iter=j, keep_weights=(j == n_iter - 1))
        I.append(r.iter_sigma[0])
        V.append(r.iter_var[0])
        passes.append(r.n_pass)
        g = r.grid
    last = r
    I, V = np.array(I), np.array(V)
    sigma, err, chi2 = O.combine(I, V)
    ids = np.arange(0, N, SAMPLE_STRIDE, dtype=np.uint64)
    ws, flags = O.event_weights(proc, W.SQRT_S, pdf, grid_last, seed, n_iter - 1, ids,
                                n_threads=THREADS)
    assert np.array_equal(ws, last.weights_last[ids.astype(np.int64)])
    out = dict(
        process={"n_g": c["n_g"], **c["cuts"]}, n_events=N, n_iter=n_iter, seed=seed,
        oracle_threads=THREADS, seconds=round(time.time() - t0, 1),
        iter_sigma=I.tolist(), iter_var=V.tolist(), iter_pass=passes,
        sigma=sigma, sigma_err=err, chi2_dof=chi2, w_max=last.w_max,
        n_pass_last=last.n_pass, n_newton_fail_last=last.n_newton_fail,
        n_near_edge_last=last.n_near_edge,
        grid_last=grid_last.tolist(), grid=last.grid.tolist(), hist_last=last.hist_last.tolist(),
        sample_ids=ids.tolist(), sample_w=ws.tolist(), sample_flags=flags.tolist(),
    )
    return out


def contracted_run(name: str) -> dict:
    """The integration of `run` on the contracted build, in a child process
    (the build is chosen when the oracle's library is loaded)."""
    import subprocess
    subprocess.run(["make", "-C", os.path.join(ROOT, "oracle"), "-s", "libmfo_fma.so"], check=True)
    env = dict(os.environ, MFO_LIB=os.path.join(ROOT, "oracle", "libmfo_fma.so"))
    code = ("import json, sys; sys.path.insert(0, %r); import make_golden as M; "
            "r = M.run(%r); print(json.dumps(r))" % (HERE, name))
    out = subprocess.run([sys.executable, "-c", code], env=env, check=True, capture_output=True, text=True)
    return json.loads(out.stdout.strip().splitlines()[-1])


def drift(name: str) -> None:
    path = os.path.join(HERE, name + ".json")
    with open(path) as f:
        ref = json.load(f)
    alt = contracted_run(name)

    def rel(a, b):
        a, b = np.asarray(a, float), np.asarray(b, float)
        nz = b != 0
        return float(np.max(np.abs(a[nz] / b[nz] - 1))) if nz.any() else 0.0

    ref["drift"] = dict(
        build="oracle sources with -mfma -ffp-contract=fast", seconds=alt["seconds"],
        I=rel(alt["iter_sigma"], ref["iter_sigma"]), V=rel(alt["iter_var"], ref["iter_var"]),
        sigma=rel(alt["sigma"], ref["sigma"]), w_max=rel(alt["w_max"], ref["w_max"]),
        hist=rel(alt["hist_last"], ref["hist_last"]),
        grid=float(np.max(np.abs(np.asarray(alt["grid"]) - np.asarray(ref["grid"])))))
    # the last iteration's largest weight: which event it is
    c = CASES[name]
    proc = O.Process(n_g=c["n_g"], **c["cuts"])
    pdf = W.synthetic_pdf()
    w, _ = O.event_weights(proc, W.SQRT_S, pdf, np.asarray(ref["grid_last"]), ref["seed"], ref["n_iter"] - 1,
                           np.arange(ref["n_events"], dtype=np.uint64), n_threads=THREADS)
    e = int(np.argmax(w))
    assert w[e] == ref["w_max"]
    ref["w_max_event"] = e
    with open(path, "w") as f:
        json.dump(ref, f)
    print(f"{name}: drift {ref['drift']}, w_max event {e}", flush=True)


def main(names):
    if names and names[0] == "--drift":
        for name in names[1:] or CASES:
            drift(name)
        return
    for name in names or CASES:
        out = run(name)
        path = os.path.join(HERE, name + ".json")
        with open(path, "w") as f:
            json.dump(out, f)
        print(f"{name}: sigma {out['sigma']:.6f} +- {out['sigma_err']:.6f} pb, "
              f"chi2/dof {out['chi2_dof']:.3f}, {out['seconds']} s -> {path}", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
