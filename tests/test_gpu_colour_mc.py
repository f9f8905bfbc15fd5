"""GPU parity of the Monte Carlo over colours (colour = "sampled": one colour
assignment per event from Philox block 0x80000001) against the oracle, and
its unbiasedness against the full colour sum on the same events."""
import math
import sys

import numpy as np
import pytest

import oracle as O
from parity_checks import assert_integration_parity

pytestmark = pytest.mark.gpu

SQRT_S = 13000.0
CONF = {
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
    c = {k: v for k, v in CONF[n_g].items() if k != "process"}
    return O.Process(n_g=n_g, colour="sampled", **c)


@pytest.mark.parametrize("n_g,n,iters", [(3, 3_000, 2), (4, 700, 2)])
def test_sampled_colour_integration_matches_oracle(api, pdf_table, n_g, n, iters):
    say(f"sampled colour integrate n_g={n_g} n={n} iters={iters}")
    g = api.integrate(gproc(api, n_g), SQRT_S, pdf_table, n, iters, seed=0, colour="sampled")
    o = O.integrate(oproc(n_g), SQRT_S, pdf_table, n, iters, seed=0)
    say("  gpu", g.sigma, g.sigma_err, g.chi2_dof, "oracle", o.sigma, o.sigma_err, o.chi2_dof)
    assert_integration_parity(g, o, n, say=say)
    np.testing.assert_allclose(g.weights.cpu().numpy(), o.weights_last, rtol=1e-11, atol=1e-300)
    assert g.n_pass == o.n_pass


def test_sampled_colour_fp32_events_match_oracle(api, pdf_table):
    g = api.integrate(gproc(api, 4), SQRT_S, pdf_table, 700, 1, seed=2, colour="sampled",
                      precision="fp32_kahan")
    o = O.integrate(oproc(4), SQRT_S, pdf_table, 700, 1, seed=2)
    w, ref = g.weights.cpu().numpy(), o.weights_last
    nz = ref != 0
    assert np.all(w[~nz] == 0)
    rel = np.abs(w[nz] / ref[nz] - 1)
    say(f"  FP32 sampled colour: {int(nz.sum())} nonzero weights, max rel {rel.max():.2e}")
    assert rel.max() < 2e-4


def test_sampled_colour_unsupported_calls(api, pdf_table):
    from paper_2106_10279_amd import _lib as L
    with pytest.raises(L.MFError) as e:
        api.integrate(api.Process("gg_ttx"), SQRT_S, pdf_table, 1000, 1, 0, colour="sampled")
    assert e.value.status == L.MF_EUNSUPPORTED
    with pytest.raises(L.MFError) as e:
        api.evaluate_weights(gproc(api, 4), SQRT_S, pdf_table, 64, colour="sampled")
    assert e.value.status == L.MF_EUNSUPPORTED


def test_sampled_colour_ttxgg_1e7_sampled_events_and_unbiasedness(api, oracle_lib, pdf_table):
    """At the full t tbar g g size: 2000 sampled events of an iteration on a
    fixed grid against the oracle, and, on the same 1e7 events and grid, the
    mean difference to the full-colour weights against its own error (the
    estimator is unbiased), with the variance it adds."""
    import torch
    proc = gproc(api, 4)
    N = 10_000_000
    grid = api.integrate(proc, SQRT_S, pdf_table, N, 1, 0, keep_weights=False).grid
    rs = api.integrate(proc, SQRT_S, pdf_table, N, 1, 0, grid_in=grid, start_iter=1, colour="sampled")
    rf = api.integrate(proc, SQRT_S, pdf_table, N, 1, 0, grid_in=grid, start_iter=1)
    ws, wf = rs.weights, rf.weights
    assert torch.equal(ws != 0, (ws != 0) & (wf != 0))
    d = (ws - wf).double()
    mean, err = float(d.mean().item()), float(d.std().item()) / math.sqrt(N)
    vs, vf = float(ws.var().item()), float(wf.var().item())
    say(f"\n  1e7 ttgg: sampled {rs.iter_sigma[0]:.6g} full {rf.iter_sigma[0]:.6g} pb; mean difference "
        f"{mean:.3g} +- {err:.2g}; per-event variance ratio {vs / vf:.2f}")
    assert abs(mean) < 5 * err
    rng = np.random.default_rng(61)
    ids = np.sort(rng.choice(N, size=2000, replace=False))
    w_o, flags = oracle_lib.event_weights(oproc(4), SQRT_S, pdf_table, grid, 0, 1, ids)
    wg = ws[ids].cpu().numpy()
    skip = (flags & (8 | 16)) != 0
    zero = (w_o == 0.0) & ~skip
    assert np.all(wg[zero] == 0.0)
    use = ~skip & ~zero
    # bit 5: the sampled sum cancels between orderings (condition number kappa
    # above 50), which magnifies the rounding of the partial amplitudes; those
    # events are held to 1e-12 kappa / 50
    cond = (flags & 32) != 0
    rel = np.abs(wg[use & ~cond] / w_o[use & ~cond] - 1.0)
    worst = 0.0
    for i in np.nonzero(use & cond)[0]:
        wo, ev = O.event_weight(oproc(4), SQRT_S, pdf_table, grid, 0, 1, int(ids[i]))
        assert wo == w_o[i]
        r = abs(wg[i] / wo - 1.0)
        worst = max(worst, r / ev.colour_kappa)
        assert r < 1e-12 * ev.colour_kappa / 50
    say(f"  {int(use.sum())} of 2000 sampled events nonzero and usable, max rel {rel.max():.2e} "
        f"({int((use & cond).sum())} with kappa > 50: max rel / kappa {worst:.2e})")
    # most assignments give a vanishing colour factor for every ordering: about a
    # quarter of the passing events carry a nonzero weight
    assert use.sum() > 300
    assert rel.max() < 1e-12
