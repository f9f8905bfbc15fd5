"""GPU parity of the hit-or-miss unweighting (mf_unweight) against the
oracle: the keep decisions bit-exact on identical weights, the kept sets on
each side's own weights (events whose decision lies within the weights'
rounding difference excluded and counted), and the lab-frame records to
1e-12 of the beam energy."""
import sys

import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.gpu

SQRT_S = 13000.0
CONF = {
    2: dict(process="gg_ttx"),
    3: dict(process="gg_ttxg", ptmin_g=20.0, etamax_g=2.5),
    4: dict(process="gg_ttxgg", ptmin_g=20.0, drmin_gg=0.4),
}


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


def gproc(api, n_g):
    return api.Process(**CONF[n_g])


def oproc(n_g):
    return O.Process(n_g=n_g, **{k: v for k, v in CONF[n_g].items() if k != "process"})


def _check_records(n_g, ev, grid, seed, it, idx):
    """GPU lab records of the kept events at positions idx against the oracle."""
    p = ev.p.cpu().numpy()
    events = ev.event.cpu().numpy()
    worst = 0.0
    for i in idx:
        q, st = O.lab_event(oproc(n_g), SQRT_S, grid, seed, it, int(events[i]))
        if st != 0:
            assert not p[i].any()
            continue
        worst = max(worst, np.abs(p[i] - q).max() / (0.5 * SQRT_S))
    return worst


@pytest.mark.parametrize("n_g,n", [(2, 300_000), (3, 300_000), (4, 300_000), (4, 300_001), (3, 8195),
                                   (2, 4097), (4, 13), (2, 1)])
def test_keep_decisions_bit_exact_on_identical_weights(api, n_g, n):
    """Identical weights on both sides; sizes with ragged 16-event segments,
    tiles and workgroup ranges, and below one segment."""
    import torch
    say(f"unweight identical weights n_g={n_g} n={n}")
    rng = np.random.default_rng(40 + n_g + n)
    w = rng.exponential(1.0, n) * np.where(rng.random(n) < 0.1, -1.0, 1.0)
    w[rng.random(n) < 0.2] = 0.0
    w[:5] = [np.nan, 0.0, 3.0, -3.0, 1e-300][:n]
    w[-1] = 2.5                      # the last event is always kept
    w_max = 2.0
    seed, it = 7, 3
    keep_o, n_o, over_o = O.unweight(w, w_max, seed, it)
    ev = api.unweight(gproc(api, n_g), SQRT_S, torch.tensor(w, device="cuda"), w_max, seed, it)
    assert ev.n_kept == n_o and ev.n_over == over_o
    kept_idx = np.flatnonzero(keep_o)
    assert np.array_equal(ev.event.cpu().numpy(), kept_idx)
    assert np.array_equal(ev.sign.cpu().numpy(), keep_o[kept_idx])
    assert int(ev.event[-1]) == n - 1
    grid = np.tile(np.arange(51) / 50, (2 + 3 * n_g - 4, 1))
    sel = np.unique(np.linspace(0, ev.n_kept - 1, 200).astype(int))
    worst = _check_records(n_g, ev, grid, seed, it, sel)
    say(f"  kept {ev.n_kept} of {n}, records max |dp|/E_beam {worst:.1e}")
    assert worst < 1e-12


def _borderline(w, w_max, seed, it, ids, rel=1e-9):
    out = []
    for e in ids:
        u = O.unweight_uniform(seed, it, int(e))
        if abs(u * w_max - abs(w[e])) <= rel * max(abs(w[e]), 1e-300):
            out.append(int(e))
    return set(out)


@pytest.mark.parametrize("n_g,n", [(2, 100_000), (4, 4096)])
def test_unweighting_an_integration_matches_the_oracle(api, pdf_table, n_g, n):
    say(f"unweight after integration n_g={n_g} n={n}")
    D = 2 + 3 * n_g - 4
    seed, start = 3, 1
    # a refined, non-uniform grid from a short oracle run is the input of both sides
    g0 = O.integrate(oproc(n_g), SQRT_S, pdf_table, 2000, 1, 11, keep_weights=False).grid
    o = O.integrate(oproc(n_g), SQRT_S, pdf_table, n, 1, seed, grid=g0, start_iter=start)
    r = api.integrate(gproc(api, n_g), SQRT_S, pdf_table, n, 1, seed, grid_in=g0, start_iter=start)
    assert np.array_equal(r.grid_last, g0)
    assert r.w_max == pytest.approx(o.w_max, rel=1e-12)
    keep_o, n_o, _ = O.unweight(o.weights_last, o.w_max, seed, start)
    ev = api.unweight(gproc(api, n_g), SQRT_S, r.weights, r.w_max, seed, start, grid=r.grid_last)
    gset = dict(zip(ev.event.cpu().numpy().tolist(), ev.sign.cpu().numpy().tolist()))
    oset = {int(e): int(keep_o[e]) for e in np.flatnonzero(keep_o)}
    diff = set(gset) ^ set(oset)
    border = _borderline(o.weights_last, o.w_max, seed, start, sorted(diff))
    say(f"  kept GPU {ev.n_kept} / oracle {n_o} of {n}; {len(diff)} differ, {len(border)} of them borderline")
    assert diff == border
    assert len(diff) <= 2
    for e in set(gset) & set(oset):
        assert gset[e] == oset[e]
    sel = np.linspace(0, ev.n_kept - 1, min(ev.n_kept, 300)).astype(int)
    worst = _check_records(n_g, ev, r.grid_last, seed, start, sel)
    say(f"  records max |dp|/E_beam {worst:.1e}")
    assert worst < 1e-12
    # the unweighted estimate against the weighted mean (binomial error)
    w = o.weights_last
    est = o.w_max * sum(oset.values()) / n
    err = np.sqrt((o.w_max * np.abs(w) - w * w).sum()) / n
    assert abs(est - w.mean()) < 5 * err


def test_capacity_truncates_in_event_order(api):
    import torch
    say("unweight capacity")
    rng = np.random.default_rng(5)
    w = torch.tensor(rng.random(200_000), device="cuda")
    full = api.unweight(gproc(api, 3), SQRT_S, w, 1.0, 0, 0)
    half = api.unweight(gproc(api, 3), SQRT_S, w, 1.0, 0, 0, capacity=full.n_kept // 2)
    assert half.n_kept == full.n_kept
    k = full.n_kept // 2
    assert torch.equal(half.event, full.event[:k])
    assert torch.equal(half.p, full.p[:k])
    assert torch.equal(half.sign, full.sign[:k])
    none = api.unweight(gproc(api, 3), SQRT_S, torch.zeros(1000, dtype=torch.float64, device="cuda"), 1.0, 0, 0)
    assert none.n_kept == 0 and none.event.numel() == 0
    empty = api.unweight(gproc(api, 3), SQRT_S, torch.zeros(0, dtype=torch.float64, device="cuda"), 1.0, 0, 0)
    assert empty.n_kept == 0
