"""Integration parity at the reduced sizes of the parity plan, full-size stage
isolation, and crafted edge inputs, all through the C ABI.

* g g -> t tbar at its full size, 1e5 events x 5 iterations: every output
  of the integration against the oracle's own run, including every weight of
  the last iteration.
* g g -> t tbar g at 1e6 x 10 and g g -> t tbar g g at 1e5 x 10 against the
  oracle's integrations stored in tests/golden/ (written by
  tests/golden/make_golden.py, which calls only the oracle): ten grid
  refinements, I_j, V_j, sigma, its error, chi^2/dof, w_max, the pass counts,
  the grids and the last histogram.  I_j and sigma are held to 1e-10; the
  grids, the histogram, w_max and V_j to ten times the rounding drift that the
  oracle shows against its own contracted build over the same iterations
  (stored with the reference), because each refinement feeds the grid's
  rounding back through the bin widths in J_V.  Sampled weights of the last
  iteration and its largest weight are held to 1e-12 against the oracle
  evaluated on the grid that iteration ran on.
* g g -> t tbar g g at its full size, 1e7 x 10: the oracle refines the GPU's
  last histogram from the grid that iteration ran on and must reproduce the
  GPU's final grid; the oracle's combination of the GPU's I_j and V_j must
  reproduce the GPU's sigma, error and chi^2/dof; every row of the histogram
  sums to the same sum of w^2, which the GPU's I_j and V_j fix; sampled events
  of the last iteration against the oracle.
* explicit uniforms at the edges of every dimension (y = 0, y = 1 - 2^-53,
  VEGAS bin edges), s_hat just above threshold, cos(theta) = -1 and 1, phi at
  0, pi and 2 pi, x on a PDF knot, mass variables at their ends: weights and
  per-stage flags against the oracle.
"""
import json
import math
import os
import sys

import numpy as np
import pytest

import oracle as O
from parity_checks import assert_integration_parity, drift_bars, newton_bar

pytestmark = pytest.mark.gpu

SQRT_S = 13000.0
HERE = os.path.dirname(os.path.abspath(__file__))
CUTS = {2: {}, 3: dict(ptmin_g=20.0, etamax_g=2.5), 4: dict(ptmin_g=20.0, drmin_gg=0.4)}
NAME = {2: "gg_ttx", 3: "gg_ttxg", 4: "gg_ttxgg"}


@pytest.fixture(scope="module")
def api():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2106_10279_amd import api
    return api


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def uniform_grid(D, nb=50):
    return np.tile(np.arange(nb + 1) / nb, (D, 1))


def test_ttx_full_size_1e5x5(api, pdf_table):
    N, iters = 100_000, 5
    say(f"\n  g g -> t tbar {N} x {iters}")
    g = api.integrate(api.Process("gg_ttx"), SQRT_S, pdf_table, N, iters, seed=0)
    o = O.integrate(O.Process(n_g=2), SQRT_S, pdf_table, N, iters, seed=0)
    say(f"  gpu {g.sigma:.8f} +- {g.sigma_err:.8f} chi2/dof {g.chi2_dof:.4f}; "
        f"oracle {o.sigma:.8f} +- {o.sigma_err:.8f} chi2/dof {o.chi2_dof:.4f}")
    assert_integration_parity(g, o, N, say=say)
    # every weight of the last iteration: the oracle's own grid after iters - 1
    # refinements gives the flags of R21/R22 for each event (near a cut edge,
    # ill-conditioned PDF value), which leave an event out of the 1e-12 bar
    o4 = O.integrate(O.Process(n_g=2), SQRT_S, pdf_table, N, iters - 1, seed=0, keep_weights=False)
    wo, fl, kap = O.event_weights(O.Process(n_g=2), SQRT_S, pdf_table, o4.grid, 0, iters - 1, np.arange(N),
                                  return_kappa=True)
    assert np.array_equal(wo, o.weights_last)
    wg = g.weights.cpu().numpy()
    skip = (fl & (8 | 16)) != 0
    zero = (wo == 0.0) & ~skip
    assert np.all(wg[zero] == 0.0)
    use = ~skip & ~zero
    cond = use & ((fl & 64) != 0)
    plain = use & ~cond
    rel = np.abs(wg[plain] / wo[plain] - 1)
    rel_c = np.abs(wg[cond] / wo[cond] - 1)
    bar_c = newton_bar(kap[cond], 2)
    rel_skip = np.abs(wg[skip] / wo[skip] - 1) if skip.any() else np.zeros(1)
    say(f"  all {N} weights of the last iteration: {int(plain.sum())} within {rel.max():.2e}, "
        f"{int(cond.sum())} near threshold (kappa_N up to {kap[cond].max() if cond.any() else 0:.1e}) at "
        f"{(rel_c / bar_c).max() if cond.any() else 0:.2f} of their bar, {int(zero.sum())} zero on both "
        f"sides, {int(skip.sum())} flagged (R21/R22) within {rel_skip.max():.2e}")
    assert rel.max() < 1e-12
    assert np.all(rel_c <= bar_c)


@pytest.mark.parametrize("name,n_g", [("integration_gg_ttxg_1e6x10", 3),
                                      ("integration_gg_ttxgg_1e5x10", 4)])
def test_integration_against_stored_oracle_run(api, pdf_table, name, n_g):
    path = os.path.join(HERE, "golden", name + ".json")
    with open(path) as f:
        ref = json.load(f)
    N, iters, seed = ref["n_events"], ref["n_iter"], ref["seed"]
    say(f"\n  {name}: {N} x {iters}, seed {seed}")
    g = api.integrate(api.Process(NAME[n_g], **CUTS[n_g]), SQRT_S, pdf_table, N, iters, seed=seed)
    say(f"  gpu {g.sigma:.6f} +- {g.sigma_err:.6f} chi2/dof {g.chi2_dof:.4f}; "
        f"oracle {ref['sigma']:.6f} +- {ref['sigma_err']:.6f} chi2/dof {ref['chi2_dof']:.4f}")
    bars = drift_bars(ref)
    d = ref["drift"]
    say(f"  rounding drift of the oracle's contracted build: grid {d['grid']:.1e}, w_max {d['w_max']:.1e}, "
        f"hist {d['hist']:.1e}, V {d['V']:.1e}, I {d['I']:.1e}, sigma {d['sigma']:.1e}")
    assert_integration_parity(g, ref, N, say=say, bars=bars)
    assert np.array_equal(np.asarray(g.iter_pass, dtype=np.int64), np.asarray(ref["iter_pass"]))
    assert np.abs(g.grid_last - np.asarray(ref["grid_last"])).max() <= bars["grid"]
    # stage isolation of the last iteration: the oracle evaluates the sampled
    # events and the event of the largest weight on the grid that iteration
    # ran on in this run; per-event bar 1e-12
    ids = np.asarray(ref["sample_ids"] + [ref["w_max_event"]], dtype=np.int64)
    op = O.Process(n_g=n_g, **CUTS[n_g])
    wo, fl = O.event_weights(op, SQRT_S, pdf_table, g.grid_last, seed, iters - 1, ids)
    wg = g.weights.cpu().numpy()[ids]
    skip = (fl & (8 | 16)) != 0
    zero = (wo == 0.0) & ~skip
    assert np.all(wg[zero] == 0.0)
    use = ~skip & ~zero
    rel = np.abs(wg[use] / wo[use] - 1)
    say(f"  {int(use.sum())} sampled weights of the last iteration on its grid, max rel {rel.max():.2e}; "
        f"{int(skip.sum())} excluded; w_max event {ref['w_max_event']}: {abs(wg[-1] / wo[-1] - 1):.2e}")
    assert rel.max() < 1e-12
    assert g.w_max == wg[-1] and abs(wg[-1] / wo[-1] - 1) < 1e-12


def test_ttxgg_full_size_stage_isolation(api, pdf_table):
    N, iters = 10_000_000, 10
    proc = api.Process("gg_ttxgg", **CUTS[4])
    say(f"\n  g g -> t tbar g g {N} x {iters}")
    g = api.integrate(proc, SQRT_S, pdf_table, N, iters, seed=0)
    # the oracle's refinement of the GPU's last histogram from the grid it ran on
    refined = O.vegas_refine(g.hist, g.grid_last)
    d_grid = float(np.abs(refined - g.grid).max())
    # the oracle's combination of the GPU's iteration estimates
    s, e, c = O.combine(g.iter_sigma, g.iter_var)
    say(f"  sigma {g.sigma:.6f} +- {g.sigma_err:.6f} pb, chi2/dof {g.chi2_dof:.4f}; "
        f"refinement of the GPU histogram vs GPU grid {d_grid:.1e}")
    assert d_grid <= 1e-12
    assert abs(g.sigma / s - 1) <= 1e-14 and abs(g.sigma_err / e - 1) <= 1e-14
    assert abs(g.chi2_dof - c) <= 1e-12 * c
    # every histogram row holds the same sum of w^2 = N (N - 1) V + N I^2
    rows = np.array([math.fsum(r) for r in g.hist])
    sw2 = N * (N - 1) * g.iter_var[-1] + N * g.iter_sigma[-1] ** 2
    say(f"  histogram rows {rows.min():.6e} .. {rows.max():.6e}, from I and V {sw2:.6e}")
    assert np.all(np.abs(rows / sw2 - 1) < 1e-9)
    assert np.all(np.abs(rows / rows[0] - 1) < 1e-12)
    w = g.weights
    assert float(w.sum().item()) / N == pytest.approx(g.iter_sigma[-1], rel=1e-12)
    assert float((w * w).sum().item()) == pytest.approx(sw2, rel=1e-9)
    assert int((w != 0).sum().item()) == g.n_pass
    assert float(w.max().item()) == g.w_max
    # sampled events of the last iteration, on the grid it ran on
    rng = np.random.default_rng(77)
    ids = np.sort(rng.choice(N, size=3000, replace=False))
    op = O.Process(n_g=4, **CUTS[4])
    wo, fl = O.event_weights(op, SQRT_S, pdf_table, g.grid_last, 0, iters - 1, ids)
    wg = w[ids].cpu().numpy()
    skip = (fl & (8 | 16)) != 0
    zero = (wo == 0.0) & ~skip
    assert np.all(wg[zero] == 0.0)
    use = ~skip & ~zero
    rel = np.abs(wg[use] / wo[use] - 1)
    say(f"  {int(use.sum())} of 3000 sampled events of iteration {iters - 1}, max rel {rel.max():.2e}")
    assert use.sum() > 2000 and rel.max() < 1e-12


TOP = 1.0 - 2.0**-53


def edge_points(n_g):
    """Uniform vectors at the edges of every dimension of the process."""
    D = 2 + 3 * n_g - 4
    rng = np.random.default_rng(500 + n_g)
    tau = 2 * 173.0 / SQRT_S
    base = np.array([0.31, 0.27] + list(rng.uniform(0.2, 0.8, D - 2)))
    pts = [base.copy()]
    for d in range(D):
        for v in (0.0, TOP, 0.5, 0.02, 0.98, 17 / 50, np.nextafter(17 / 50, 0), np.nextafter(0.5, 1)):
            y = base.copy()
            y[d] = v
            pts.append(y)
    # s_hat just above (and just below) threshold
    for f in (1 + 1e-12, 1 + 1e-9, 1 + 1e-6, 1 - 1e-12):
        y = base.copy()
        y[0] = y[1] = tau * f
        pts.append(y)
    # x on PDF knots x_k = 10^(-7 + 7k/99) (up to the rounding of the VEGAS map)
    for k in (90, 92, 95, 98):
        y = base.copy()
        y[0] = 10.0 ** (-7.0 + 7.0 * k / 99.0)
        y[1] = max(tau * tau / y[0] * 4.0, 0.05)
        pts.append(y)
    # every angle of the first two-body split at its ends together
    for a, b in ((0.0, 0.0), (TOP, TOP), (0.0, TOP), (TOP, 0.5)):
        y = base.copy()
        y[D - 2 * (n_g - 1)], y[D - 2 * (n_g - 1) + 1] = a, b
        pts.append(y)
    return np.ascontiguousarray(np.array(pts))


@pytest.mark.parametrize("n_g", [2, 3, 4])
def test_explicit_uniform_edge_cases(api, pdf_table, n_g):
    import torch
    y = edge_points(n_g)
    n, D = y.shape
    proc = api.Process(NAME[n_g], **CUTS[n_g])
    w, rec = api.evaluate_weights(proc, SQRT_S, pdf_table, n, y=torch.tensor(y, device="cuda"),
                                  return_record=True)
    w, rec = w.cpu().numpy(), rec.cpu().numpy()
    op = O.Process(n_g=n_g, **CUTS[n_g])
    grid = uniform_grid(D)
    worst, used, kinds = 0.0, 0, {"zero": 0, "newton": 0, "below": 0, "cut": 0}
    for e in range(n):
        ref, ev = O.event_weight_y(op, SQRT_S, pdf_table, grid, y[e])
        flags = int(rec[e][7])
        assert bool(flags & 1) == ev.pass_threshold, e
        if ev.pass_threshold:
            assert bool(flags & 2) == ev.newton_fail, e
        assert np.isfinite(w[e]), e
        if ev.near_edge or ev.ill_conditioned:
            continue
        assert bool(flags & 4) == ev.pass_cuts, e
        kinds["below"] += not ev.pass_threshold
        kinds["newton"] += ev.newton_fail
        kinds["cut"] += ev.pass_threshold and not ev.newton_fail and not ev.pass_cuts
        if ref == 0.0:
            kinds["zero"] += 1
            assert w[e] == 0.0, (e, w[e])
        else:
            used += 1
            worst = max(worst, abs(w[e] / ref - 1))
    say(f"\n  n_g={n_g}: {n} edge points, {used} nonzero within {worst:.2e}; {kinds}")
    assert used > n // 3
    assert worst < 1e-12
