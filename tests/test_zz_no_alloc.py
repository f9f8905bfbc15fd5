"""mf_integrate_static (no device allocation) against mf_integrate, through the C ABI.

Two calls in a row per process, the second with fewer events and iterations,
so the second call reuses the static scratch the first left behind.  While a
call's events fit one batch of the static scratch both entry points run the
same launches in the same order, so every output must be identical bit for
bit.  With more events than one static batch holds, the per-event weights are
identical in the first iteration (they do not depend on the batching), the
sums agree to the integral bar of the FP64 path (1e-10 relative; grids 1e-12,
histogram 1e-11), and a later iteration's weights, whose grid was refined
from sums that differ in rounding, equal those mf_integrate computes on that
same grid.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

SQRT_S = 13000.0
CUTS = {"gg_ttx": {}, "gg_ttxg": dict(ptmin_g=20.0, etamax_g=2.5), "gg_ttxgg": dict(ptmin_g=20.0, drmin_gg=0.4)}


@pytest.fixture(scope="module")
def api():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2106_10279_amd import api
    return api


def same(a, b):
    assert a.sigma == b.sigma and a.sigma_err == b.sigma_err and a.chi2_dof == b.chi2_dof
    assert a.w_max == b.w_max and a.n_pass == b.n_pass and a.n_newton_fail == b.n_newton_fail
    for x, y in ((a.iter_sigma, b.iter_sigma), (a.iter_var, b.iter_var), (a.grid, b.grid),
                 (a.grid_last, b.grid_last), (a.hist, b.hist), (a.iter_pass, b.iter_pass)):
        assert np.array_equal(np.asarray(x), np.asarray(y))
    assert bool((a.weights == b.weights).all().item())


@pytest.mark.parametrize("name,sizes", [("gg_ttx", ((200_000, 3), (30_000, 2))),
                                        ("gg_ttxgg", ((300_000, 3), (50_000, 2))),
                                        ("gg_ttxg", ((400_000, 2), (70_001, 3)))])
def test_static_equals_integrate_two_calls(api, pdf_table, name, sizes):
    proc = api.Process(name, **CUTS[name])
    for n, it in sizes:
        print(f"\n  {name} {n} x {it}", flush=True)
        s = api.integrate(proc, SQRT_S, pdf_table, n, it, seed=3, static_scratch=True)
        g = api.integrate(proc, SQRT_S, pdf_table, n, it, seed=3)
        assert s.n_batches == g.n_batches == 1
        same(s, g)
        print(f"  sigma {s.sigma:.6f} +- {s.sigma_err:.6f}: identical", flush=True)


def test_static_several_batches(api, pdf_table):
    """More events than one static batch: the first iteration's weights are
    identical (they do not depend on the batching), its sums agree to
    rounding; the second call has fewer events and two iterations, whose
    second runs on a grid refined from those sums: its weights equal those of
    mf_integrate on the same grid."""
    proc = api.Process("gg_ttxgg", **CUTS["gg_ttxgg"])
    for n, it in ((1_500_000, 1), (600_000, 2)):
        print(f"\n  gg_ttxgg {n} x {it}", flush=True)
        s = api.integrate(proc, SQRT_S, pdf_table, n, it, seed=1, static_scratch=True)
        g = api.integrate(proc, SQRT_S, pdf_table, n, it, seed=1)
        ws, wg = s.weights, g.weights
        nz = wg != 0
        rel = float(((ws[nz] - wg[nz]) / wg[nz]).abs().max().item())
        print(f"  static: {s.n_batches} batches, sigma {s.sigma:.8f}; mf_integrate: {g.n_batches}, "
              f"{g.sigma:.8f}; weights max rel {rel:.2e}", flush=True)
        assert s.n_batches >= 2 and g.n_batches == 1
        assert bool((ws[~nz] == 0).all().item())
        # the last iteration: with one iteration both ran on the uniform grid;
        # with two, the second ran on a grid refined from sums that differ in
        # rounding, so mf_integrate repeats that iteration on the static call's grid
        last = g if it == 1 else api.integrate(proc, SQRT_S, pdf_table, n, 1, seed=1, grid_in=s.grid_last,
                                               start_iter=it - 1)
        assert bool((ws == last.weights).all().item())
        assert s.w_max == last.w_max and s.n_pass == last.n_pass
        hs, hl = np.asarray(s.hist), np.asarray(last.hist)
        nzh = hl != 0
        assert np.all(hs[~nzh] == 0) and np.abs(hs[nzh] / hl[nzh] - 1).max() < 1e-11
        assert np.all(np.abs(np.asarray(s.iter_sigma) / np.asarray(g.iter_sigma) - 1) < 1e-10)
        assert abs(s.sigma / g.sigma - 1) < 1e-10
        assert np.all(np.abs(np.asarray(s.iter_var) / np.asarray(g.iter_var) - 1) < 1e-9)
        assert np.abs(np.asarray(s.grid) - np.asarray(g.grid)).max() <= 1e-12
        assert np.abs(np.asarray(s.grid_last) - np.asarray(g.grid_last)).max() <= 1e-12
        assert np.array_equal(np.asarray(s.iter_pass), np.asarray(g.iter_pass))


def test_static_limits(api, pdf_table):
    proc = api.Process("gg_ttxgg", **CUTS["gg_ttxgg"])
    with pytest.raises(api.MFError) as e:
        api.integrate(proc, SQRT_S, pdf_table, 1000, 1, seed=0, n_bins=60, static_scratch=True)
    assert e.value.status == -1 and "512" in str(e.value)
    with pytest.raises(api.MFError) as e:
        api.integrate(proc, SQRT_S, pdf_table, 1000, 1, seed=0, profile=True, static_scratch=True)
    assert e.value.status == -5
    # still usable after the rejected calls
    s = api.integrate(proc, SQRT_S, pdf_table, 5000, 1, seed=0, static_scratch=True)
    g = api.integrate(proc, SQRT_S, pdf_table, 5000, 1, seed=0)
    same(s, g)
