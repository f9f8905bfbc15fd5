"""Assertions shared by the GPU integration parity tests.

`assert_integration_parity(g, ref)` compares every output of an integration
of the library (`api.integrate`) with the oracle's integration of the same
workload: per-iteration estimates I_j and variances V_j, the combined cross
section, its error and chi^2/dof, w_max, the passing-event count, the grids
and the last histogram.

Tolerances (floating point, FP64 path):

* I_j and sigma: 1e-10 relative (the integral bar);
* V_j = [(1/N) sum w^2 - I_j^2]/(N - 1): the per-event weights agree to about
  1e-12, so sum w^2 agrees to about 2e-12; the one-pass difference magnifies a
  relative error of sum w^2 by a = (1/N) sum w^2 / [(1/N) sum w^2 - I_j^2]
  (the cancellation factor, computed from the oracle's own V_j); the bar is
  1e-10 a;
* sigma_err = (sum 1/V_j)^(-1/2): half the largest relative V_j difference,
  plus 1e-14;
* chi^2/dof = sum (I_j - I)^2 / V_j / (n - 1): twice the first-order
  propagation of the measured I_j and V_j differences, plus 1e-12 relative;
* the library's own combination of its I_j, V_j (done on the host) must
  reproduce the oracle's formula (`mfo_combine`) on the same inputs to
  1e-14 (chi^2/dof: 1e-12 relative);
* w_max: 1e-12 relative (it is one event's weight); n_pass: exact unless the
  oracle flagged events at a cut edge;
* grids: 1e-12 absolute (edges lie in [0, 1]); histogram: 1e-11 relative.
"""
from __future__ import annotations

import numpy as np

import oracle as O


def newton_bar(kappa, n_f):
    """Per-event bar for an event whose mass-rescaling root is ill-conditioned
    (oracle flag bit 6, kappa_N = sqrt(s_hat) / (xi F'(xi)) > 1e3, close to
    threshold).  The Newton stop accepts any xi whose residual is below
    2 n_f 2^-52 sqrt(s_hat), which fixes xi only to 4 n_f 2^-53 kappa_N
    relative; the two sides may stop anywhere inside that (factor 2), and the
    weight depends on xi at most like xi^(2 n_f) (factor 2 n_f)."""
    return 1e-12 + 16 * n_f * n_f * 2.0**-53 * np.asarray(kappa)


def as_reference(o, n_events: int) -> dict:
    """An oracle IntegrationResult (or a stored reference dict) as a dict."""
    if isinstance(o, dict):
        d = dict(o)
        d.setdefault("n_pass_last", d.get("n_pass"))
        return d
    return dict(n_events=n_events, iter_sigma=o.iter_sigma, iter_var=o.iter_var, sigma=o.sigma,
                sigma_err=o.sigma_err, chi2_dof=o.chi2_dof, w_max=o.w_max, n_pass_last=o.n_pass,
                n_newton_fail_last=o.n_newton_fail, n_near_edge_last=o.n_near_edge, grid=o.grid,
                hist_last=o.hist_last)


def chi2_bound(I, V, dI, dV, mean, dmean):
    n = len(I)
    if n < 2:
        return 0.0
    t = 2 * np.abs(I - mean) * (np.abs(dI) + abs(dmean)) / V + (I - mean) ** 2 * np.abs(dV) / V**2
    return float(t.sum() / (n - 1))


def drift_bars(ref: dict, factor: float = 10.0) -> dict:
    """Bars for an integration compared over several grid refinements.

    Every weight depends on the widths of its bins through J_V, and the next
    grid is refined from those weights, so rounding differences in the grid
    grow from one iteration to the next.  The stored reference measures that
    growth: the same integration by the oracle built with fused multiply-add
    contraction (a second correct FP64 build) differs from the plain build by
    `ref["drift"]`.  The GPU must stay within `factor` times that, and never
    above the single-refinement bars."""
    d = ref.get("drift")
    if not d:
        return {}
    return dict(grid=max(1e-12, factor * d["grid"]), w_max=max(1e-12, factor * d["w_max"]),
                hist=max(1e-11, factor * d["hist"]), V=factor * d["V"])


def assert_integration_parity(g, o, n_events: int, *, hist=True, say=print, bars=None) -> dict:
    """`bars` (from drift_bars) relaxes the grid, w_max, histogram and V_j
    bars of an integration over several refinements; the integral bar on I_j
    and sigma stays 1e-10."""
    bars = bars or {}
    ref = as_reference(o, n_events)
    N = float(ref["n_events"])
    Ig, Vg = np.asarray(g.iter_sigma, float), np.asarray(g.iter_var, float)
    Io, Vo = np.asarray(ref["iter_sigma"], float), np.asarray(ref["iter_var"], float)
    dI = Ig - Io
    relI = np.abs(dI) / np.abs(Io)
    amp = (Vo * (N - 1) + Io**2) / (Vo * (N - 1))
    relV = np.abs(Vg - Vo) / Vo
    # every figure first, so that a failing run still reports all of them
    out = dict(I=relI.max(), V=relV.max(), V_over_a=(relV / amp).max())
    out["sigma"] = abs(g.sigma / ref["sigma"] - 1)
    s, e, c = O.combine(Ig, Vg)
    out["sigma_err"] = abs(g.sigma_err / ref["sigma_err"] - 1)
    b = chi2_bound(Io, Vo, dI, Vg - Vo, ref["sigma"], g.sigma - ref["sigma"])
    out["chi2"] = abs(g.chi2_dof - ref["chi2_dof"])
    out["chi2_bound"] = 2 * b + 1e-12 * abs(ref["chi2_dof"])
    out["w_max"] = abs(g.w_max / ref["w_max"] - 1)
    out["grid"] = float(np.abs(np.asarray(g.grid) - np.asarray(ref["grid"])).max())
    if hist:
        hg, ho = np.asarray(g.hist), np.asarray(ref["hist_last"])
        nz = ho != 0
        out["hist"] = float((np.abs(hg[nz] / ho[nz] - 1)).max()) if nz.any() else 0.0
    say("  parity: " + ", ".join(f"{k} {v:.2e}" for k, v in out.items()))
    assert relI.max() < 1e-10, ("I_j", relI)
    assert np.all(relV < np.maximum(1e-10 * amp, bars.get("V", 0.0))), ("V_j", relV, amp)
    assert out["sigma"] < 1e-10, (g.sigma, ref["sigma"])
    # the library's host combination against the oracle's formula on the same inputs
    assert abs(g.sigma - s) <= 1e-14 * abs(s)
    assert abs(g.sigma_err - e) <= 1e-14 * e
    assert abs(g.chi2_dof - c) <= 1e-12 * abs(c) + 1e-300
    # the library's error and chi^2/dof against the oracle's
    assert out["sigma_err"] <= 0.5 * relV.max() + 1e-14, (g.sigma_err, ref["sigma_err"])
    assert out["chi2"] <= out["chi2_bound"], (g.chi2_dof, ref["chi2_dof"], b)
    assert out["w_max"] < bars.get("w_max", 1e-12), (g.w_max, ref["w_max"])
    near = int(ref.get("n_near_edge_last") or 0)
    assert abs(g.n_pass - ref["n_pass_last"]) <= near, (g.n_pass, ref["n_pass_last"], near)
    assert g.n_newton_fail >= 0
    assert out["grid"] <= bars.get("grid", 1e-12)
    if hist:
        assert np.all(hg[~nz] == 0)
        assert out["hist"] < bars.get("hist", 1e-11)
    return out
