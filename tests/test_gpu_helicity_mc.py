"""GPU parity of the Monte Carlo over helicities (helicity = "sampled": one
configuration of top spins and linear gluon polarisations per event, uniform,
from Philox block 0x80000002, N_h |M_h|^2 for the colour sum) against the
oracle, alone and with the Monte Carlo over colour flows, and its
unbiasedness against the helicity sum on the same events at full size."""
import math
import sys

import numpy as np
import pytest

import oracle as O
from parity_checks import assert_integration_parity, newton_bar

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


def oproc(n_g, colour="full"):
    c = {k: v for k, v in CONF[n_g].items() if k != "process"}
    return O.Process(n_g=n_g, colour=colour, helicity="sampled", **c)


def compare_events(wg, w_o, flags, newton_kappa, n_g, w_sum, bar=1e-12):
    """Per-event comparison.  One configuration's |M_h|^2 can be far below the
    helicity sum, while the rounding of its amplitudes is set by the event's
    amplitude scale, the helicity sum: the difference is held to bar times the
    oracle's helicity-summed weight w_sum of the same event.  Events at a cut
    edge or with an ill-conditioned PDF value (bits 3, 4) are left out; an
    event whose mass-rescaling root is ill-conditioned (bit 6, close to
    threshold) is held to the bar of that conditioning (newton_bar)."""
    skip = (flags & (8 | 16)) != 0
    zero = (w_o == 0.0) & ~skip
    assert np.all(wg[zero] == 0.0)
    use = ~skip & ~zero
    cond = use & ((flags & 64) != 0)
    scale = np.maximum(np.abs(w_o), np.abs(w_sum))
    rel = np.abs(wg - w_o)[use & ~cond] / scale[use & ~cond]
    if cond.any():
        b = np.maximum(bar, newton_bar(newton_kappa[cond], n_g))
        assert np.all(np.abs(wg - w_o)[cond] / scale[cond] <= b)
    return rel, int(use.sum()), int(cond.sum())


def summed(n_g):
    c = {k: v for k, v in CONF[n_g].items() if k != "process"}
    return O.Process(n_g=n_g, **c)


@pytest.mark.parametrize("n_g,n,iters", [(2, 20_000, 3), (3, 3_000, 2), (4, 700, 2)])
def test_helicity_mc_integration_matches_oracle(api, pdf_table, n_g, n, iters):
    say(f"\n  helicity Monte Carlo integrate n_g={n_g} n={n} iters={iters}")
    g = api.integrate(gproc(api, n_g), SQRT_S, pdf_table, n, iters, seed=0, helicity="sampled")
    o = O.integrate(oproc(n_g), SQRT_S, pdf_table, n, iters, seed=0)
    say(f"  gpu {g.sigma:.6f} +- {g.sigma_err:.6f}, oracle {o.sigma:.6f} +- {o.sigma_err:.6f}")
    assert_integration_parity(g, o, n, say=say)
    np.testing.assert_allclose(g.weights.cpu().numpy(), o.weights_last, rtol=1e-11, atol=1e-300)
    assert g.n_pass == o.n_pass


@pytest.mark.parametrize("n_g", [3, 4])
def test_helicity_and_colour_flow_integration_matches_oracle(api, pdf_table, n_g):
    n = 3000 if n_g == 3 else 700
    g = api.integrate(gproc(api, n_g), SQRT_S, pdf_table, n, 2, seed=4, helicity="sampled", colour="flow")
    o = O.integrate(oproc(n_g, "flow"), SQRT_S, pdf_table, n, 2, seed=4)
    say(f"\n  helicity + flow n_g={n_g}: gpu {g.sigma:.6f}, oracle {o.sigma:.6f}")
    assert_integration_parity(g, o, n, say=say)
    wg, wo = g.weights.cpu().numpy(), o.weights_last
    assert np.array_equal(wg == 0, wo == 0)


@pytest.mark.parametrize("n_g,n", [(2, 3000), (3, 1500), (4, 300)])
@pytest.mark.parametrize("precision,bar", [("fp64", 1e-12), ("fp32_kahan", 2e-4)])
def test_helicity_mc_event_weights_match_oracle(api, pdf_table, n_g, n, precision, bar):
    """mf_evaluate with Philox counters (the fused event kernel) on a refined
    grid, every event against the oracle."""
    D = 3 * n_g - 2
    rng = np.random.default_rng(40 + n_g)
    grid = np.sort(np.concatenate([np.zeros((D, 1)), rng.uniform(0, 1, (D, 49)), np.ones((D, 1))], axis=1), axis=1)
    w = api.evaluate_weights(gproc(api, n_g), SQRT_S, pdf_table, n, seed=7, it=3, grid=grid,
                             precision=precision, helicity="sampled").cpu().numpy()
    w_o, flags, kap = O.event_weights(oproc(n_g), SQRT_S, pdf_table, grid, 7, 3, np.arange(n), return_kappa=True)
    w_sum, _ = O.event_weights(summed(n_g), SQRT_S, pdf_table, grid, 7, 3, np.arange(n))
    rel, used, _ = compare_events(w, w_o, flags, kap, n_g, w_sum, bar)
    say(f"\n  n_g={n_g} {precision}: {used} usable events, max difference / summed weight {rel.max():.2e}")
    assert used > n // 3 and rel.max() < bar


def test_helicity_mc_rejected_calls(api, pdf_table):
    import torch
    from paper_2106_10279_amd import _lib as L
    y = torch.full((8, 4), 0.4, dtype=torch.float64, device="cuda")
    with pytest.raises(L.MFError) as e:
        api.evaluate_weights(gproc(api, 2), SQRT_S, pdf_table, 8, y=y, helicity="sampled")
    assert e.value.status == L.MF_EINVAL
    opt = api._options(50, 1.5, 0, "fp64", False, 50, None, None, helicity="sampled")
    res, gr = L.mf_result(), L.mf_grad_result()
    pdf = api._Pdf(pdf_table)
    pc = gproc(api, 2).c()
    import ctypes as C
    st = L.lib.mf_integrate_grad(C.byref(pc), SQRT_S, C.byref(pdf.c), 1000, 1, 0, C.byref(opt), C.byref(res),
                                 C.byref(gr))
    assert st == L.MF_EUNSUPPORTED


@pytest.mark.parametrize("n_g", [2, 4])
def test_helicity_mc_1e7_sampled_events_and_unbiased(api, pdf_table, n_g):
    """Full size (1e7 events, the headline launch configuration for t tbar g g):
    2000 sampled events of an iteration on a fixed grid against the oracle; on
    the same events and grid the mean difference to the helicity sum against
    its own error, and the per-event variance ratio."""
    proc = gproc(api, n_g)
    N = 10_000_000
    grid = api.integrate(proc, SQRT_S, pdf_table, N, 1, 0, keep_weights=False).grid
    kw = dict(grid_in=grid, start_iter=1)
    rs = api.integrate(proc, SQRT_S, pdf_table, N, 1, 0, helicity="sampled", **kw)
    rf = api.integrate(proc, SQRT_S, pdf_table, N, 1, 0, **kw)
    ws, wf = rs.weights, rf.weights
    d = (ws - wf).double()
    mean, err = float(d.mean().item()), float(d.std().item()) / math.sqrt(N)
    ratio = float(ws.var().item()) / float(wf.var().item())
    del d
    say(f"\n  1e7 n_g={n_g}: sampled {rs.iter_sigma[0]:.6g} summed {rf.iter_sigma[0]:.6g} pb; mean difference "
        f"{mean:.3g} +- {err:.2g}; per-event variance ratio {ratio:.3f}")
    assert abs(mean) < 5 * err
    rng = np.random.default_rng(92 + n_g)
    ids = np.sort(rng.choice(N, size=2000, replace=False))
    w_o, flags, kap = O.event_weights(oproc(n_g), SQRT_S, pdf_table, grid, 0, 1, ids, return_kappa=True)
    w_sum, _ = O.event_weights(summed(n_g), SQRT_S, pdf_table, grid, 0, 1, ids)
    rel, used, _ = compare_events(ws[ids].cpu().numpy(), w_o, flags, kap, n_g, w_sum)
    say(f"  {used} of 2000 sampled events usable, max difference / summed weight {rel.max():.2e}")
    assert used > 1000 and rel.max() < 1e-12
