"""GPU parity of the adjoint (g g -> t tbar): d w/d m_t, d w/d y, d sigma/d m_t,
d sigma/d alpha_s, against the oracle's analytic zero-width gradient and
against central finite differences of oracle and GPU weights (common random
numbers, frozen grids)."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

SQRT_S = 13000.0
NB = 50


@pytest.fixture(scope="module")
def api():
    import torch
    assert torch.cuda.is_available()
    from paper_2106_10279_amd import api as A
    return A


def uniform_grid(D=4):
    return np.tile(np.arange(NB + 1) / NB, (D, 1))


def fd4(f, x0, h):
    """Fourth-order central difference."""
    return (8.0 * (f(x0 + h) - f(x0 - h)) - (f(x0 + 2 * h) - f(x0 - 2 * h))) / (12.0 * h)


def test_dw_dmt_matches_the_analytic_zero_width_gradient(api, oracle_lib, pdf_table):
    import torch
    O = oracle_lib
    n = 3000
    y = W.random_uniforms(n, 4, seed=11)
    grid = uniform_grid()
    proc = api.Process("gg_ttx", w_top=0.0)
    w, dy, dm = api.evaluate_weights_grad(proc, SQRT_S, pdf_table, n, grid=grid,
                                          y=torch.tensor(y, device="cuda"))
    w, dm = w.cpu().numpy(), dm.cpu().numpy()
    op = O.Process(n_g=2, w_top=0.0)
    worst_w = worst_g = 0.0
    checked = 0
    for i in range(n):
        g_ref, w_ref = O.ttx_dweight_dmt_analytic(op, SQRT_S, pdf_table, grid, y[i])
        if w_ref == 0.0:
            assert w[i] == 0.0 and dm[i] == 0.0
            continue
        worst_w = max(worst_w, abs(w[i] / w_ref - 1.0))
        worst_g = max(worst_g, abs(dm[i] - g_ref) / abs(g_ref))
        checked += 1
    print(f"\n  {checked} events: weight max rel {worst_w:.2e}, dw/dm_t max rel {worst_g:.2e}")
    assert checked > 0.9 * n
    # closed form against the helicity sum: rounding, largest at small beta
    assert worst_w < 5e-12
    assert worst_g < 1e-9


def test_dw_dmt_matches_oracle_central_differences_with_width(api, oracle_lib, pdf_table):
    import torch
    O = oracle_lib
    n = 300
    y = W.random_uniforms(n, 4, seed=12)
    grid = uniform_grid()
    proc = api.Process("gg_ttx")
    _, _, dm = api.evaluate_weights_grad(proc, SQRT_S, pdf_table, n, grid=grid,
                                         y=torch.tensor(y, device="cuda"))
    dm = dm.cpu().numpy()
    m0 = 173.0
    h = 1e-4 * m0
    worst = 0.0
    checked = 0
    for i in range(n):
        def wt(m):
            return O.event_weight_y(O.Process(n_g=2, m_top=m), SQRT_S, pdf_table, grid, y[i])[0]
        # the stencil must stay above threshold, and away from it (dw/dm_t ~ 1/beta)
        info = O.event_weight_y(O.Process(n_g=2), SQRT_S, pdf_table, grid, y[i])[1]
        if info.w == 0.0 or 1.0 - 4.0 * m0 * m0 / info.shat < 0.04:
            continue
        ws = [wt(m0 + k * h) for k in (-2, -1, 0, 1, 2)]
        fd = (8.0 * (ws[3] - ws[1]) - (ws[4] - ws[0])) / (12.0 * h)
        err = abs(dm[i] - fd) / max(abs(fd), 1e-300)
        worst = max(worst, err)
        checked += 1
    print(f"\n  {checked} events: dw/dm_t vs oracle FD max rel {worst:.2e}")
    assert checked > 0.5 * n
    assert worst < 1e-6


def test_dw_dy_matches_oracle_central_differences(api, oracle_lib, pdf_table):
    import torch
    O = oracle_lib
    n = 200
    y = W.random_uniforms(n, 4, seed=13)
    grid = uniform_grid()
    proc = api.Process("gg_ttx")
    w, dy, _ = api.evaluate_weights_grad(proc, SQRT_S, pdf_table, n, grid=grid,
                                         y=torch.tensor(y, device="cuda"))
    w, dy = w.cpu().numpy(), dy.cpu().numpy()
    op = O.Process(n_g=2)
    h = 1e-6
    worst = 0.0
    checked = 0
    for i in range(n):
        if w[i] == 0.0:
            assert not dy[i].any()
            continue
        for d in range(4):
            ys = [y[i].copy() for _ in range(5)]
            for k, s in enumerate((-2, -1, 0, 1, 2)):
                ys[k][d] += s * h
            # the stencil must stay inside the event's VEGAS bin and above threshold
            if len({int(np.floor(v[d] * NB)) for v in ys}) != 1 or not all(0.0 <= v[d] < 1.0 for v in ys):
                continue
            ws = [O.event_weight_y(op, SQRT_S, pdf_table, grid, v)[0] for v in ys]
            if min(ws) <= 0.0:
                continue
            fd = (8.0 * (ws[3] - ws[1]) - (ws[4] - ws[0])) / (12.0 * h)
            # derivative scale: |w| per unit y (phi derivatives vanish up to the width)
            err = abs(dy[i, d] - fd) / max(abs(fd), abs(w[i]))
            worst = max(worst, err)
            checked += 1
    print(f"\n  {checked} (event, dim) pairs: dw/dy vs oracle FD max rel {worst:.2e}")
    assert checked > 2 * n
    assert worst < 1e-6


@pytest.fixture(scope="module")
def grad_run(api, pdf_table):
    proc = api.Process("gg_ttx")
    N, it = 100_000, 3
    rg, g = api.integrate_grad(proc, SQRT_S, pdf_table, N, it, 0)
    r = api.integrate(proc, SQRT_S, pdf_table, N, it, 0, keep_weights=False)
    return proc, N, it, rg, g, r


def test_integrate_grad_replays_the_integration_exactly(grad_run):
    proc, N, it, rg, g, r = grad_run
    assert np.array_equal(rg.iter_sigma, r.iter_sigma)
    assert np.array_equal(rg.iter_var, r.iter_var)
    assert np.array_equal(rg.grid, r.grid)
    assert rg.sigma == r.sigma


def test_dsigma_dalphas_is_n_g_sigma_over_alpha_s(grad_run):
    proc, N, it, rg, g, r = grad_run
    assert g.dsigma_dalphas == pytest.approx(2.0 * r.sigma / proc.alpha_s, rel=1e-12)
    assert np.allclose(g.iter_dalphas, 2.0 * r.iter_sigma / proc.alpha_s, rtol=1e-12, atol=0)


def test_dsigma_dmt_matches_finite_differences_on_frozen_grids(api, pdf_table, grad_run):
    """Per iteration j, on the grid of iteration j and the same Philox events:
    the adjoint's mean dw/dm_t equals the per-event adjoints, and on events
    whose stencil m +- 2h stays clear of threshold (beta^2 > 0.01) the summed
    adjoint equals the summed central differences.  Nearer threshold
    dw/dm_t ~ 1/beta is integrable but no finite difference resolves it; those
    events are pinned by the zero-width analytic test instead."""
    from dataclasses import replace
    proc, N, it, rg, g, r = grad_run
    m0 = proc.m_top
    h = 1e-4 * m0
    for j in range(it):
        grid_j = uniform_grid() if j == 0 else api.integrate(proc, SQRT_S, pdf_table, N, j, 0,
                                                             keep_weights=False).grid
        _, rec = api.evaluate_weights(proc, SQRT_S, pdf_table, N, seed=0, it=j, grid=grid_j,
                                      return_record=True)
        _, _, dm = api.evaluate_weights_grad(proc, SQRT_S, pdf_table, N, seed=0, it=j, grid=grid_j)
        ws = [api.evaluate_weights(replace(proc, m_top=m0 + k * h), SQRT_S, pdf_table, N, seed=0, it=j,
                                   grid=grid_j).cpu().numpy() for k in (-2, -1, 1, 2)]
        fd = (8.0 * (ws[2] - ws[1]) - (ws[3] - ws[0])) / (12.0 * h)
        rec = rec.cpu().numpy()
        dm = dm.cpu().numpy()
        shat = rec[:, 0] * rec[:, 1] * SQRT_S ** 2
        clear = shat * (1.0 - 0.01) > 4.0 * m0 * m0
        adj, num = dm[clear].sum() / N, fd[clear].sum() / N
        near = dm[~clear].sum() / N
        print(f"\n  iteration {j}: adjoint {adj:.10g} vs FD {num:.10g} on {clear.sum()} events "
              f"(rel {abs(adj / num - 1):.2e}); near-threshold share {near:.4g} of {g.iter_dmt[j]:.6g}")
        assert g.iter_dmt[j] == pytest.approx(dm.sum() / N, rel=1e-12)
        assert adj == pytest.approx(num, rel=1e-6)
    inv = 1.0 / r.iter_var
    assert g.dsigma_dmt == pytest.approx(float(np.sum(g.iter_dmt * inv) / np.sum(inv)), rel=1e-13)


def test_dsigma_dmt_agrees_with_the_quadrature_value(api, pdf_table):
    """Zero width, uniform start grid: the adaptive estimate of d sigma/d m_t at
    173 GeV against the 2-D quadrature of the closed form (-17.738 pb/GeV)
    within its Monte Carlo error plus the interpolation error of the grid PDF."""
    proc = api.Process("gg_ttx", w_top=0.0)
    rg, g = api.integrate_grad(proc, SQRT_S, pdf_table, 1_000_000, 5, 0)
    spread = np.std(g.iter_dmt[1:], ddof=1) / np.sqrt(len(g.iter_dmt) - 1)
    print(f"\n  dsigma/dm_t = {g.dsigma_dmt:.5f} pb/GeV (iteration spread {spread:.4f}); sigma = {rg.sigma:.4f}")
    assert abs(g.dsigma_dmt - (-17.738)) < 5.0 * spread + 2e-3 * 17.738


def test_autograd_cross_section(api, pdf_table, grad_run):
    import torch
    proc, N, it, rg, g, r = grad_run
    m = torch.tensor(proc.m_top, dtype=torch.float64, requires_grad=True)
    a = torch.tensor(proc.alpha_s, dtype=torch.float64, requires_grad=True)
    s = api.CrossSection.apply(m, a, proc, SQRT_S, pdf_table, N, it, 0)
    s.backward()
    assert s.item() == r.sigma
    assert m.grad.item() == g.dsigma_dmt
    assert a.grad.item() == g.dsigma_dalphas


def test_autograd_event_weights(api, pdf_table):
    import torch
    n = 4096
    y = torch.tensor(W.random_uniforms(n, 4, seed=14), device="cuda", requires_grad=True)
    m = torch.tensor(173.0, dtype=torch.float64, requires_grad=True)
    proc = api.Process("gg_ttx")
    grid = uniform_grid()
    w = api.EventWeights.apply(y, m, proc, SQRT_S, pdf_table, grid)
    c = torch.linspace(0.5, 1.5, n, dtype=torch.float64, device="cuda")
    (w * c).sum().backward()
    w2, dy, dm = api.evaluate_weights_grad(proc, SQRT_S, pdf_table, n, grid=grid, y=y.detach())
    # the adjoint kernel recomputes the weight with its own helicity loop;
    # the two agree to rounding (largest near threshold, where both are within
    # 2e-12 of the closed form)
    assert torch.allclose(w.detach(), w2, rtol=5e-12, atol=0)
    ref = c[:, None] * dy
    diff = (y.grad - ref).abs()
    print(f"\n  y.grad vs c dy: max abs diff {diff.max().item():.3e}, differing {(diff > 0).sum().item()}, "
          f"finite {bool(torch.isfinite(y.grad).all())}, dtype {y.grad.dtype}")
    assert torch.allclose(y.grad, ref, rtol=1e-15, atol=0)
    assert m.grad.item() == pytest.approx((c * dm).sum().item(), rel=1e-14)


def test_event_grads_of_the_last_iteration(api, pdf_table):
    """dw/dy and dw/dm_t stored by mf_integrate_grad for the last iteration
    equal mf_evaluate_grad on that iteration's grid and events."""
    proc = api.Process("gg_ttx")
    N, it = 20_000, 2
    rg, g = api.integrate_grad(proc, SQRT_S, pdf_table, N, it, 0, keep_event_grads=True)
    grid1 = api.integrate(proc, SQRT_S, pdf_table, N, 1, 0, keep_weights=False).grid
    _, dy, dm = api.evaluate_weights_grad(proc, SQRT_S, pdf_table, N, seed=0, it=1, grid=grid1)
    assert np.array_equal(g.dw_dy.cpu().numpy(), dy.cpu().numpy())
    assert np.array_equal(g.dw_dmt.cpu().numpy(), dm.cpu().numpy())
    assert g.iter_dmt[-1] == pytest.approx(dm.double().mean().item(), rel=1e-12)
