"""GPU parity of p p -> t tbar, t tbar g and t tbar g g (the g g channel
plus the q qbar channels u ubar, ubar u, d dbar, dbar d; Sec. 3, Table 1)
against the oracle: the q qbar |M|^2 for explicit momenta, per-event
weights, a short integration, and the requests these processes refuse."""
import sys

import numpy as np
import pytest

import oracle as O
import workloads as W
from parity_checks import assert_integration_parity, newton_bar

pytestmark = pytest.mark.gpu

SQRT_S = 13000.0
M = 173.0
# process, gluons, cuts, events for the weight and integration checks
CASES = {
    "pp_ttx": (2, {}, 20_000, 20_000),
    "pp_ttxg": (3, dict(ptmin_g=20.0, etamax_g=2.5), 6_000, 3_000),
    "pp_ttxgg": (4, dict(ptmin_g=20.0, drmin_gg=0.4), 1_500, 600),
}


@pytest.fixture(scope="module")
def api():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2106_10279_amd import api
    return api


@pytest.fixture(scope="module")
def pp_table():
    return W.synthetic_pdf(quarks=True)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("process", sorted(CASES))
def test_qqbar_matrix_element(api, process):
    import torch
    n_g = CASES[process][0]
    rng = np.random.default_rng(31)
    moms, ebs, refs = [], [], []
    for _ in range({2: 300, 3: 150, 4: 60}[n_g]):
        rs = 2 * M + 1.0 + rng.exponential(600.0)
        masses = [M, M] + [0.0] * (n_g - 2)
        k, w, st = O.phase_space(n_g, masses, rs, rng.random(3 * n_g - 4))
        E = rs / 2
        p = np.array([k[0], k[1], [-E, 0, 0, -E], [-E, 0, 0, E], *k[2:]])
        refs.append({2: lambda: O.me2_qqbar_ttx(p, M), 3: lambda: O.me2_qqbar_ttxg(p, M, 1.5),
                     4: lambda: O.me2_qqbar_ttxgg(p, M, 1.5)}[n_g]())
        moms.append(k.reshape(-1))
        ebs.append(E)
    mom = torch.tensor(np.array(moms), dtype=torch.float64, device="cuda").contiguous()
    eb = torch.tensor(np.array(ebs), dtype=torch.float64, device="cuda")
    say(f"\n  {process} q qbar |M|^2: {len(refs)} points")
    got = api.matrix_element(process, mom, eb, M, 1.5).cpu().numpy()
    rel = np.abs(got / np.array(refs) - 1)
    say(f"  max rel {rel.max():.2e}")
    assert rel.max() < 1e-12


@pytest.mark.parametrize("process", sorted(CASES))
@pytest.mark.parametrize("precision,bar", [("fp64", 1e-12), ("fp32_kahan", 2e-4)])
def test_event_weights_match_oracle(api, pp_table, process, precision, bar):
    """Per-event weights against the oracle.  The weight is the g g term plus
    the q qbar terms; where the interpolated tables go negative (x near 1)
    these have opposite signs, so the bar is relative to |g g| + |q qbar|
    of the oracle's own split."""
    n_g, cuts, n, _ = CASES[process]
    D = 3 * n_g - 2
    rng = np.random.default_rng(8)
    grid = np.sort(np.concatenate([np.zeros((D, 1)), rng.uniform(0, 1, (D, 49)), np.ones((D, 1))], axis=1), axis=1)
    say(f"\n  weights {process} {precision}: {n} events")
    w = api.evaluate_weights(api.Process(process, **cuts), SQRT_S, pp_table, n, seed=2, it=4, grid=grid,
                             precision=precision).cpu().numpy()
    w_o, flags, kap = O.event_weights(O.Process(n_g=n_g, initial="pp", **cuts), SQRT_S, pp_table, grid, 2, 4,
                                      np.arange(n), return_kappa=True)
    w_og, _ = O.event_weights(O.Process(n_g=n_g, **cuts), SQRT_S, pp_table, grid, 2, 4, np.arange(n))
    skip = (flags & (8 | 16)) != 0
    zero = (w_o == 0.0) & ~skip
    assert np.all(w[zero] == 0.0)
    use = ~skip & ~zero
    scale = np.abs(w_og) + np.abs(w_o - w_og)
    rel = np.abs(w - w_o)[use] / scale[use]
    limit = np.where((flags[use] & 64) != 0, np.maximum(bar, newton_bar(kap[use], n_g)), bar)
    say(f"  {int(use.sum())} nonzero, max rel {rel.max():.2e}, "
        f"{int(np.sum(np.sign(w_og[use]) != np.sign(w_o[use] - w_og[use])))} with opposite-sign channels")
    assert use.sum() > n // 3 and np.all(rel <= limit)
    # the q qbar channels separately: p p minus the g g process on the same events
    gg = "gg_" + process[3:]
    wg = api.evaluate_weights(api.Process(gg, **cuts), SQRT_S, pp_table, n, seed=2, it=4, grid=grid,
                              precision=precision).cpu().numpy()
    q, q_o = (w - wg)[use], (w_o - w_og)[use]
    assert np.all(np.abs(q - q_o) <= 2 * limit * scale[use])
    assert np.mean(np.abs(q_o) > 1e-3 * np.abs(w_og[use])) > 0.9


@pytest.mark.parametrize("process,N", [("pp_ttx", 100_000_000), ("pp_ttxg", 10_000_000),
                                       ("pp_ttxgg", 1_000_000)])
def test_full_size_sampled_events_and_properties(api, pp_table, process, N):
    """Each p p process at the size bench.py times (1e8, 1e7 and 1e6 events
    per iteration, the live-event lists and the q qbar kernels as launched
    there): 1500 events sampled over the whole second iteration against the
    oracle on that iteration's grid, and on all events finite weights, one
    nonzero weight per passing event and the mean equal to the iteration's
    estimate."""
    import torch
    n_g, cuts = CASES[process][0], CASES[process][1]
    proc = api.Process(process, **cuts)
    g1 = api.integrate(proc, SQRT_S, pp_table, N, 1, 0, keep_weights=False).grid
    r = api.integrate(proc, SQRT_S, pp_table, N, 2, 0, keep_weights=True)
    w = r.weights
    assert torch.isfinite(w).all()
    assert int((w != 0).sum()) == r.n_pass
    assert float(w.sum().item()) / N == pytest.approx(r.iter_sigma[-1], rel=1e-12)
    ids = np.sort(np.random.default_rng(12).choice(N, size=1500, replace=False))
    w_o, flags, kap = O.event_weights(O.Process(n_g=n_g, initial="pp", **cuts), SQRT_S, pp_table, g1, 0, 1, ids,
                                      return_kappa=True)
    w_og, _ = O.event_weights(O.Process(n_g=n_g, **cuts), SQRT_S, pp_table, g1, 0, 1, ids)
    wg = w[torch.as_tensor(ids, device=w.device)].cpu().numpy()
    skip = (flags & (8 | 16)) != 0
    zero = (w_o == 0.0) & ~skip
    assert np.all(wg[zero] == 0.0)
    use = ~skip & ~zero
    rel = np.abs(wg - w_o)[use] / (np.abs(w_og) + np.abs(w_o - w_og))[use]
    limit = np.where((flags[use] & 64) != 0, np.maximum(1e-12, newton_bar(kap[use], n_g)), 1e-12)
    say(f"\n  {process} {N:.0e}: {int(use.sum())} of 1500 sampled events up to id {ids.max()}, "
        f"max rel {rel.max():.2e}, {int(skip.sum())} at a cut edge or ill-conditioned")
    assert use.sum() > 500 and np.all(rel <= limit)
    del r, w
    torch.cuda.empty_cache()


@pytest.mark.parametrize("process", sorted(CASES))
def test_integration_matches_oracle(api, pp_table, process):
    n_g, cuts, _, n = CASES[process]
    iters = 3 if n_g == 2 else 2
    say(f"\n  integrate {process} n={n} iters={iters}")
    g = api.integrate(api.Process(process, **cuts), SQRT_S, pp_table, n, iters, seed=0)
    o = O.integrate(O.Process(n_g=n_g, initial="pp", **cuts), SQRT_S, pp_table, n, iters, seed=0)
    say(f"  gpu {g.sigma:.8g} +- {g.sigma_err:.3g}, oracle {o.sigma:.8g}")
    assert_integration_parity(g, o, n, say=say)
    # absolute floor: events whose g g and q qbar terms cancel (tables negative near x = 1)
    np.testing.assert_allclose(g.weights.cpu().numpy(), o.weights_last, rtol=1e-11,
                               atol=1e-14 * np.abs(o.weights_last).max())


@pytest.mark.parametrize("process", sorted(CASES))
def test_requests_refused(api, pp_table, process):
    from paper_2106_10279_amd import _lib as L
    cuts = CASES[process][1]
    with pytest.raises(L.MFError) as e:
        api.integrate(api.Process(process, **cuts), SQRT_S, W.synthetic_pdf(), 1000, 1, seed=0)
    assert e.value.status == L.MF_EINVAL
    for kw in (dict(colour="leading"), dict(helicity="sampled"), dict(static_scratch=True)):
        with pytest.raises(L.MFError) as e:
            api.integrate(api.Process(process, **cuts), SQRT_S, pp_table, 1000, 1, seed=0, **kw)
        assert e.value.status == L.MF_EUNSUPPORTED, kw
