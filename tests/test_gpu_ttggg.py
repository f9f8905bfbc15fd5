"""GPU parity of g g -> t tbar g g g (five gluons, 120 colour orderings, 128
helicity configurations; the gluon channel of the paper's largest process,
Sec. 3.2, Fig. 4) against the oracle: |M|^2 for explicit momenta, per-event
weights with every stage of the record, and a short integration; batching;
the requests this process does not serve."""
import math
import sys

import numpy as np
import pytest

import oracle as O
from parity_checks import assert_integration_parity, newton_bar

pytestmark = pytest.mark.gpu

SQRT_S = 13000.0
M = 173.0
CUTS = dict(ptmin_g=20.0, drmin_gg=0.4)


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


def gproc(api, **kw):
    c = dict(CUTS)
    c.update(kw)
    return api.Process("gg_ttxggg", **c)


def oproc(**kw):
    c = dict(CUTS)
    c.update(kw)
    return O.Process(n_g=5, **c)


def test_colour_matrix_table(api):
    assert np.array_equal(api.colour_matrix("gg_ttxggg"), O.colour_matrix(5))


def test_matrix_element(api):
    """Both precisions on phase-space points from threshold to 3 TeV, each
    event's amplitudes in its own workgroup (ragged count: 45)."""
    import torch
    rng = np.random.default_rng(105)
    moms, ebs, refs = [], [], []
    for _ in range(45):
        rs = 2 * M + 60.0 + rng.exponential(900.0)
        k, w, st = O.phase_space(5, [M, M, 0.0, 0.0, 0.0], rs, rng.random(11))
        E = rs / 2
        p = np.array([k[0], k[1], [-E, 0, 0, -E], [-E, 0, 0, E], k[2], k[3], k[4]])
        refs.append(O.me2_sum(5, p, M, 1.5))
        moms.append(k.reshape(-1))
        ebs.append(E)
    mom = torch.tensor(np.array(moms), dtype=torch.float64, device="cuda").contiguous()
    eb = torch.tensor(np.array(ebs), dtype=torch.float64, device="cuda")
    refs = np.array(refs)
    say("\n  matrix element t tbar g g g: 45 points")
    got = api.matrix_element("gg_ttxggg", mom, eb, M, 1.5).cpu().numpy()
    rel = np.abs(got / refs - 1)
    say(f"  fp64 max rel {rel.max():.3e}")
    assert rel.max() < 1e-12
    got32 = api.matrix_element("gg_ttxggg", mom, eb, M, 1.5, precision="fp32_kahan").cpu().numpy()
    rel32 = np.abs(got32 / refs - 1)
    say(f"  fp32 max rel {rel32.max():.3e}, median {np.median(rel32):.3e}")
    assert np.median(rel32) < 1e-4 and rel32.max() < 2e-3


@pytest.mark.parametrize("precision,bar", [("fp64", 1e-12), ("fp32_kahan", 2e-4)])
def test_event_weights_match_oracle(api, pdf_table, precision, bar):
    """Per-event weights and the record's stages on a refined grid, against
    the oracle event by event (excluded: cut-edge and ill-conditioned-PDF
    events; events with an ill-conditioned mass-rescaling root are held to
    that root's bar)."""
    D = 13
    n = 203
    rng = np.random.default_rng(55)
    grid = np.sort(np.concatenate([np.zeros((D, 1)), rng.uniform(0, 1, (D, 49)), np.ones((D, 1))], axis=1), axis=1)
    say(f"\n  weights t tbar g g g {precision}: {n} events")
    w, rec = api.evaluate_weights(gproc(api), SQRT_S, pdf_table, n, seed=3, it=1, grid=grid,
                                  precision=precision, return_record=True)
    w, rec = w.cpu().numpy(), rec.cpu().numpy()
    w_o, flags, kap = O.event_weights(oproc(), SQRT_S, pdf_table, grid, 3, 1, np.arange(n), return_kappa=True)
    skip = (flags & (8 | 16)) != 0
    zero = (w_o == 0.0) & ~skip
    assert np.all(w[zero] == 0.0)
    use = ~skip & ~zero
    rel = np.abs(w - w_o)[use] / np.abs(w_o[use])
    cond = (flags[use] & 64) != 0
    limit = np.where(cond, np.maximum(bar, newton_bar(kap[use], 5)), bar)
    say(f"  {int(use.sum())} nonzero, max rel {rel.max():.3e}, {int(cond.sum())} ill-conditioned roots")
    assert use.sum() > 40 and np.all(rel <= limit)
    if precision == "fp64":
        # the record's momenta and |M|^2 against the oracle's stages
        gs10 = (4 * math.pi * 0.118) ** 5 / (256 * 6)
        checked = 0
        for e in np.flatnonzero(use)[:25]:
            _, ev = O.event_weight(oproc(), SQRT_S, pdf_table, grid, 3, 1, int(e))
            kk = rec[e, 8:28].reshape(5, 4)
            assert np.abs(kk - ev.k).max() <= 1e-12 * math.sqrt(ev.shat)
            assert abs(rec[e, 6] * gs10 / ev.me2 - 1) < 1e-12
            checked += 1
        assert checked > 10


def test_integration_matches_oracle(api, pdf_table):
    n, iters = 420, 2
    say(f"\n  integrate t tbar g g g n={n} iters={iters}")
    g = api.integrate(gproc(api), SQRT_S, pdf_table, n, iters, seed=0)
    o = O.integrate(oproc(), SQRT_S, pdf_table, n, iters, seed=0)
    say(f"  gpu {g.sigma:.8g} +- {g.sigma_err:.3g}, oracle {o.sigma:.8g} +- {o.sigma_err:.3g}")
    assert_integration_parity(g, o, n, say=say)
    np.testing.assert_allclose(g.weights.cpu().numpy(), o.weights_last, rtol=1e-11, atol=0)
    assert g.n_pass == o.n_pass


def test_batches_give_identical_weights(api, pdf_table):
    n = 300
    r1 = api.integrate(gproc(api), SQRT_S, pdf_table, n, 1, seed=9)
    rb = api.integrate(gproc(api), SQRT_S, pdf_table, n, 1, seed=9, max_batch=97)
    assert rb.n_batches == 4
    assert np.array_equal(r1.weights.cpu().numpy(), rb.weights.cpu().numpy())
    assert rb.sigma == pytest.approx(r1.sigma, rel=1e-14)


def refined_grid(D, seed):
    rng = np.random.default_rng(seed)
    return np.sort(np.concatenate([np.zeros((D, 1)), rng.uniform(0, 1, (D, 49)), np.ones((D, 1))], axis=1), axis=1)


@pytest.mark.parametrize("precision,bar", [("fp64", 1e-12), ("fp32_kahan", 2e-4)])
def test_leading_colour_weights_match_oracle(api, pdf_table, precision, bar):
    """The leading-colour sum c_LC sum_sigma |A(sigma)|^2 (c_LC = 20.25; the
    amplitude kernel adds the squares per item and stores no amplitudes):
    per-event weights on a refined grid against the oracle; on the same
    events the ratio to the full-colour weight stays within the range that
    1/N^2 corrections allow."""
    n = 203
    grid = refined_grid(13, 56)
    say(f"\n  leading-colour weights t tbar g g g {precision}: {n} events")
    w = api.evaluate_weights(gproc(api), SQRT_S, pdf_table, n, seed=4, it=1, grid=grid, precision=precision,
                             colour="leading").cpu().numpy()
    w_o, flags, kap = O.event_weights(oproc(colour="leading"), SQRT_S, pdf_table, grid, 4, 1, np.arange(n),
                                      return_kappa=True)
    skip = (flags & (8 | 16)) != 0
    zero = (w_o == 0.0) & ~skip
    assert np.all(w[zero] == 0.0)
    use = ~skip & ~zero
    rel = np.abs(w - w_o)[use] / np.abs(w_o[use])
    cond = (flags[use] & 64) != 0
    limit = np.where(cond, np.maximum(bar, newton_bar(kap[use], 5)), bar)
    say(f"  {int(use.sum())} nonzero, max rel {rel.max():.3e}")
    assert use.sum() > 40 and np.all(rel <= limit)
    if precision == "fp64":
        wf = api.evaluate_weights(gproc(api), SQRT_S, pdf_table, n, seed=4, it=1, grid=grid).cpu().numpy()
        r = w[use] / wf[use]
        say(f"  leading / full colour in [{r.min():.4f}, {r.max():.4f}]")
        assert np.all((r > 0.5) & (r < 2.0)) and r.max() - r.min() > 0.01


def test_leading_colour_integration_matches_oracle(api, pdf_table):
    n, iters = 420, 2
    say(f"\n  integrate t tbar g g g, leading colour, n={n} iters={iters}")
    g = api.integrate(gproc(api), SQRT_S, pdf_table, n, iters, seed=1, colour="leading")
    o = O.integrate(oproc(colour="leading"), SQRT_S, pdf_table, n, iters, seed=1)
    say(f"  gpu {g.sigma:.8g} +- {g.sigma_err:.3g}, oracle {o.sigma:.8g} +- {o.sigma_err:.3g}")
    assert_integration_parity(g, o, n, say=say)
    np.testing.assert_allclose(g.weights.cpu().numpy(), o.weights_last, rtol=1e-11, atol=0)
    assert g.n_pass == o.n_pass


@pytest.mark.parametrize("colour", ["full", "leading"])
def test_1e6_sampled_events_and_properties(api, pdf_table, colour):
    """At the size bench.py times (1e6 events per iteration in 31 batches
    of up to 32 768): 400 events sampled over the second iteration against
    the oracle on that iteration's grid; on all events finite weights, one
    nonzero weight per passing event and the mean equal to the iteration's
    estimate."""
    import torch
    N = 1_000_000
    g1 = api.integrate(gproc(api), SQRT_S, pdf_table, N, 1, 0, keep_weights=False, colour=colour).grid
    r = api.integrate(gproc(api), SQRT_S, pdf_table, N, 2, 0, keep_weights=True, colour=colour)
    w = r.weights
    assert torch.isfinite(w).all()
    assert int((w != 0).sum()) == r.n_pass
    assert float(w.sum().item()) / N == pytest.approx(r.iter_sigma[-1], rel=1e-12)
    ids = np.sort(np.random.default_rng(13).choice(N, size=400, replace=False))
    w_o, flags, kap = O.event_weights(oproc(colour=colour), SQRT_S, pdf_table, g1, 0, 1, ids, return_kappa=True)
    wg = w[torch.as_tensor(ids, device=w.device)].cpu().numpy()
    skip = (flags & (8 | 16)) != 0
    zero = (w_o == 0.0) & ~skip
    assert np.all(wg[zero] == 0.0)
    use = ~skip & ~zero
    rel = np.abs(wg - w_o)[use] / np.abs(w_o[use])
    limit = np.where((flags[use] & 64) != 0, np.maximum(1e-12, newton_bar(kap[use], 5)), 1e-12)
    say(f"\n  t tbar g g g {colour} colour 1e6: {int(use.sum())} of 400 sampled events up to id {ids.max()}, "
        f"max rel {rel.max():.2e}, {r.n_batches} batches")
    assert use.sum() > 250 and np.all(rel <= limit)


def test_unsupported_requests(api, pdf_table):
    from paper_2106_10279_amd import _lib as L
    for kw in (dict(colour="sampled"), dict(colour="flow"), dict(helicity="sampled"),
               dict(static_scratch=True)):
        with pytest.raises(L.MFError) as e:
            api.integrate(gproc(api), SQRT_S, pdf_table, 100, 1, seed=0, **kw)
        assert e.value.status == L.MF_EUNSUPPORTED, kw
